#!/usr/bin/env python3
"""FPW periodogram benchmark on one MI355X.

Workload (default): 1000 synthetic ZTF-like light curves (nightly cadence
with 120-day seasonal gaps over 1500 d, N ~ U{100..1000}, lognormal errors,
10% sinusoids, 10% box eclipses), 1e5 trial frequencies on 0.05-50 /d, M = 20
phase bins, FP64 phase, periodogram stored and top-5 peaks per curve.

One step = one fpw_eval_batch pass over the batch, inputs resident in HBM:
prepare (weights, centring, offsets, fixed-point packing) -> fold / bin /
accumulate / reduce with fused peak selection -> per-curve peak merge,
replayed as one hipGraph.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "observation×frequency evals/sec (G/s) + roofline %, batched mixed vs plain FP64"
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_PEAK = N_CU * 64 * CLOCK_HZ  # lane-ops/s: 64 lanes per CU per clock (FP64 FMA = 78.6 TFLOP/s / 2)
LDS_PEAK = N_CU * 128 * CLOCK_HZ  # bytes/s: 128 B per CU per clock
INT8_PEAK = 5.0e15  # int8 ops/s: dense matrix-core peak of MI355X
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batched_ztf1000.json")
# sources of the dominant (batched) kernel: its traffic figures are valid only for this exact code
KERNEL_SRCS = [os.path.join(ROOT, "paper_2502_00243_amd", "csrc", f) for f in ("fpw_batched.hip", "fpw_common.h")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------- CPU baseline (oracle)
def _oracle_curve(args):
    import numpy as np

    import oracle

    t, y, dy, freqs, n_bins = args
    S = oracle.curve_periodogram(t, y, dy, freqs, n_bins)
    return float(np.sum(S)), len(t) * len(freqs)


def cpu_baseline(batch, target_s: float = 15.0, freq_stride: int = 1):
    """The FP64 oracle on the host cores over a bounded sample of the same workload:
    the first curves (as many as fill about target_s of wall time) at every
    freq_stride-th frequency of the grid."""
    import multiprocessing as mp

    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    os.environ["OMP_NUM_THREADS"] = "1"
    freqs = batch.freqs[::freq_stride]
    t0 = time.perf_counter()
    _oracle_curve((*batch.curve(0), freqs[: max(1, min(len(freqs), 2000))], batch.n_bins))
    one = time.perf_counter() - t0
    per_eval = one / (batch.lengths[0] * max(1, min(len(freqs), 2000)))
    mean_curve = per_eval * batch.lengths.mean() * len(freqs)
    n_sample = int(min(batch.n_curves, max(cores, round(target_s * cores / max(mean_curve, 1e-9)))))
    n_sample = max(cores, (n_sample // cores) * cores) if n_sample >= cores else n_sample
    n_sample = min(n_sample, batch.n_curves)
    tasks = [(*batch.curve(c), freqs, batch.n_bins) for c in range(n_sample)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_curve, tasks[:cores])  # start-up outside the timed region
        t0 = time.perf_counter()
        res = pool.map(_oracle_curve, tasks, chunksize=1)
        wall = time.perf_counter() - t0
    evals = sum(r[1] for r in res)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    grid = f"all {len(batch.freqs)} frequencies" if freq_stride == 1 else \
        f"every {freq_stride}th of {len(batch.freqs)} frequencies"
    value = evals / wall / 1e9
    return {
        "value": value,
        "unit": "G evals/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"first {n_sample} of {batch.n_curves} curves x {grid} "
        f"({evals:.3g} evals, {wall:.1f} s wall, one single-threaded NumPy process per core, {cpu})",
        "extrapolated_full_s": batch.evals() / (value * 1e9),
    }


# ---------------------------------------------------------------- GPU
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--phase", default="fp64", choices=["fp64", "fp64_listing", "df32", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-latency", action="store_true", help="skip the single-curve latency run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--workload", default="ztf1000",
                    choices=["ztf1000", "uneven", "stress", "precision", "sweep", "shared", "baseline", "latency",
                             "small"],
                    help="ztf1000: the headline line (default); uneven: 1e5 uneven curves, 2e5 freqs, "
                         "M in {10,20,40}, top-5; stress: 2e4 x 3000-point curves, 1e6 freqs, M=50, top-5; "
                         "precision: phase-arithmetic study on the ztf1000 data; "
                         "sweep: launch shapes x M on the ztf1000 data; "
                         "shared: 1000 curves at 500 common epochs, 1e5 freqs, M=20, matrix-core vs general kernel; "
                         "baseline: the ztf1000 data with a marginalised 3-term baseline (App. A general case); "
                         "latency: one curve of 200 points, 1e4 freqs, M=10, fused vs three-kernel pass; "
                         "small: plans of 1-1000 curves x 1e3-1e5 freqs, fused vs three-kernel pass")
    ap.add_argument("--curves", type=int, default=0, help="curve count override for uneven/stress")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the FPW build has no multi-GPU path "
              "(curves shard across GPUs with no collective in the hot loop; see the design notes).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "uneven":
        return bench_uneven(args)
    if args.workload == "stress":
        return bench_stress(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "shared":
        return bench_shared(args)
    if args.workload == "baseline":
        return bench_baseline(args)
    if args.workload == "latency":
        return bench_latency(args)
    if args.workload == "small":
        return bench_small(args)

    import numpy as np

    from paper_2502_00243_amd import synth

    batch = synth.ztf_batch()
    n_bins = batch.n_bins
    evals = batch.evals()

    cpu = None if args.no_cpu_baseline else cpu_baseline(batch, args.cpu_seconds)
    if cpu:
        log(f"cpu baseline: {cpu['value']:.4f} G evals/s on {cpu['cores']} cores")

    import torch

    from paper_2502_00243_amd import fpw

    torch.cuda.set_device(0)
    log(f"planning {batch.n_curves} curves, {len(batch.freqs)} freqs, {evals:.3e} evals per pass")
    plan = fpw.Plan.from_batch(batch, topk=5, phase=args.phase, profile=True)
    info = plan.info()
    S = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
    idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
    val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        plan.eval(S_out=S, idx_out=idx, val_out=val)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.eval(S_out=S, idx_out=idx, val_out=val)
        kms.append(plan.timings())  # waits for this pass's last event
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    value = evals / (wall / args.steps) / 1e9
    kms = np.asarray(kms)
    k_batched = float(kms[:, 1].mean())
    log(f"step {ms_step:.3f} ms, batched kernel {k_batched:.3f} ms, prepare {kms[:, 0].mean():.3f} ms, "
        f"merge {kms[:, 2].mean():.3f} ms -> {value:.1f} G evals/s")

    # roofline of the dominant kernel: algorithmic VALU lane-ops (6 per evaluation
    # plus 6M per (curve, frequency) for the bin reduction and reset)
    mean_n = batch.n_points / batch.n_curves
    ops = evals * 6.0 + batch.n_curves * len(batch.freqs) * 6.0 * n_bins
    achieved = ops / (k_batched * 1e-3)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_sha") == kernel_hash() and tr.get("workload") == "ztf1000":
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": VALU_PEAK / 1e12,
        "unit": "T lane-ops/s",
        "frac": achieved / VALU_PEAK,
        "traffic": traffic,
        "kernel": "batched_kernel (fold/bin/accumulate/reduce + fused peaks)",
        "ops_per_eval": 6.0 + 6.0 * n_bins / mean_n,
        "kernel_ms": k_batched,
        "lds": {
            "bytes_per_eval": 8,
            "achieved_TBps": evals * 8 / (k_batched * 1e-3) / 1e12,
            "peak_TBps": LDS_PEAK / 1e12,
            "frac": evals * 8 / (k_batched * 1e-3) / LDS_PEAK,
        },
    }

    plain = None
    if not args.no_fp64_plain:
        S64 = plan.eval_fp64()  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        S64 = plan.eval_fp64()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        plain = {"value": evals / (ms * 1e-3) / 1e9, "unit": "G evals/s", "ms": ms,
                 "kernel": "plain per-curve FP64 kernel, one launch per curve"}
        del S64
        log(f"plain FP64: {ms:.2f} ms -> {plain['value']:.1f} G evals/s")

    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    lat_us = lat3_us = None
    if not args.no_latency:
        lat_us, lat3_us = single_curve_latency(50)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "G evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp64_listing": "f64", "df32": "f32x2", "fp32": "f32"}[args.phase],
        "dtype_detail": f"{args.phase} fold and bin, 64-bit integer fixed-point bin sums, f32 statistic",
        "data": "synthetic",
        "config": {
            "workload": "1000 ZTF-like light curves (N~U(100,1000), 1500 d, seasonal gaps), "
            "1e5 trial frequencies 0.05-50 /d, M=20, periodogram + top-5 peaks",
            "n_curves": batch.n_curves,
            "n_points": batch.n_points,
            "n_freq": len(batch.freqs),
            "n_bins": n_bins,
            "evals_per_step": evals,
            "phase": args.phase,
            "launch": {"freqs_per_lane": info.freqs_per_lane, "waves_per_group": info.waves_per_group,
                       "chunk_freqs": info.chunk_freqs, "grid_groups": info.grid_groups,
                       "work_items": info.work_items, "lds_bytes": info.lds_bytes},
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_plain": plain,
        "speedup_vs_fp64_plain": (value / plain["value"]) if plain else None,
        "latency_single_curve_us": lat_us,
        "latency_single_curve_three_kernels_us": lat3_us,
    }
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- other workloads
def _time_passes(plan, steps, warmup, **kw):
    import numpy as np
    import torch

    for _ in range(warmup):
        plan.eval(**kw)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.eval(**kw)
        kms.append(plan.timings())
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return wall, np.asarray(kms)


def _roofline(evals, n_curves, n_freq, n_bins, n_points, kernel_ms):
    ops = evals * 6.0 + n_curves * n_freq * 6.0 * n_bins
    return {"bound": "alu", "achieved": ops / (kernel_ms * 1e-3) / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "T lane-ops/s", "frac": ops / (kernel_ms * 1e-3) / VALU_PEAK,
            "ops_per_eval": 6.0 + 6.0 * n_bins / (n_points / n_curves), "kernel_ms": kernel_ms,
            "lds_frac": evals * 8 / (kernel_ms * 1e-3) / LDS_PEAK}


def _fp64_rate(plan, evals):
    import torch

    plan.eval_fp64()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.eval_fp64()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"value": evals / (ms * 1e-3) / 1e9, "unit": "G evals/s", "ms": ms}


def bench_shared(args):
    """One field: 1000 curves observed at the same 500 epochs, 1e5 freqs, M = 20, periodogram + top-5.

    The matrix-core kernel against the general kernel on the same data.  The
    matrix kernel's roofline counts the int8 operations of the contraction
    it performs: rows (curve, quantity, digit) = 8 per curve, columns
    (frequency, bin) = M per frequency, depth = points, i.e. 16 M int8
    operations per evaluation, against the dense int8 peak.
    """
    import numpy as np
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    batch = synth.shared_batch(args.curves or 1000, 500)
    t, y, dy = batch.as_shared()
    evals = batch.evals()
    M = batch.n_bins
    res = {}
    for kern in ("matrix", "general"):
        plan = fpw.Plan.shared(t, y, dy, batch.freqs, M, topk=5, shared_kernel=kern, profile=True)
        S = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
        idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
        val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
        wall, kms = _time_passes(plan, args.steps, args.warmup, S_out=S, idx_out=idx, val_out=val)
        info = plan.info()
        kernel_ms = float(np.mean(kms[:, 1]))
        r = {"ms_per_pass": wall * 1e3, "G_evals_per_s": evals / wall / 1e9, "kernel_ms": kernel_ms,
             "prepare_ms": float(np.mean(kms[:, 0])), "topk_ms": float(np.mean(kms[:, 2])),
             "grid_groups": info.grid_groups, "lds_bytes": info.lds_bytes}
        if kern == "matrix":
            ops = 16.0 * M * evals
            r["roofline"] = {"bound": "mfma", "achieved": ops / (kernel_ms * 1e-3) / 1e12, "peak": INT8_PEAK / 1e12,
                             "unit": "T int8 ops/s", "frac": ops / (kernel_ms * 1e-3) / INT8_PEAK,
                             "ops_per_eval": 16.0 * M, "kernel_ms": kernel_ms}
        else:
            r["roofline"] = _roofline(evals, batch.n_curves, len(batch.freqs), M, batch.n_points, kernel_ms)
        log(f"shared {kern}: {wall * 1e3:.3f} ms/pass, kernel {kernel_ms:.3f} ms, {evals / wall / 1e9:.0f} G evals/s")
        res[kern] = r
        plan.close()
    print(json.dumps({"workload": f"shared: {batch.n_curves} curves x 500 common epochs (one field, ZTF-like cadence "
                                  f"over 1500 d), {len(batch.freqs)} freqs 0.05-50 /d, M={M}, periodogram + top-5",
                      "evals": evals, "value": res["matrix"]["G_evals_per_s"], "unit": "G evals/s",
                      "matrix": res["matrix"], "general": res["general"],
                      "speedup_matrix_vs_general": res["general"]["ms_per_pass"] / res["matrix"]["ms_per_pass"]}),
          flush=True)


def bench_baseline(args):
    """The ztf1000 data with a marginalised baseline of K = 1, 2, 3 Chebyshev terms (App. A general
    case), periodogram + top-5, against the plain statistic on the same data.  Roofline: LDS
    atomics (two 64-bit sums per evaluation when K >= 2, one when K = 1)."""
    import numpy as np
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    batch = synth.ztf_batch()
    evals = batch.evals()
    S = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
    idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
    val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
    res = {}
    for K in (0, 1, 2, 3):
        plan = fpw.Plan.from_batch(batch, topk=5, baseline_terms=K, profile=True)
        wall, kms = _time_passes(plan, args.steps, args.warmup, S_out=S, idx_out=idx, val_out=val)
        kernel_ms = float(np.mean(kms[:, 1]))
        r = {"ms_per_pass": wall * 1e3, "G_evals_per_s": evals / wall / 1e9, "kernel_ms": kernel_ms,
             "prepare_ms": float(np.mean(kms[:, 0])), "peaks_ms": float(np.mean(kms[:, 2])),
             "grid_groups": plan.info().grid_groups}
        if K > 0:
            nbytes = {1: 8, 2: 12, 3: 16}[K]  # LDS bytes added per evaluation: (w, w x), then w T_1 (and w T_2)
            r["lds"] = {"bytes_per_eval": nbytes, "achieved_TBps": evals * nbytes / (kernel_ms * 1e-3) / 1e12,
                        "peak_TBps": LDS_PEAK / 1e12, "frac": evals * nbytes / (kernel_ms * 1e-3) / LDS_PEAK}
        r["hist_share"] = plan.info().hist_share
        log(f"baseline K={K}: {wall * 1e3:.3f} ms/pass, kernel {kernel_ms:.3f} ms, {evals / wall / 1e9:.0f} G evals/s")
        res[f"K{K}"] = r
        plan.close()
    # kernel time of the baseline kernel by point source and histogram sharing (waves per histogram)
    shares = {}
    for K in (1, 2, 3):
        for src in ("scalar", "dpp"):
            for share in (1, 2, 4):
                plan = fpw.Plan.from_batch(batch, topk=5, baseline_terms=K, hist_share=share, point_source=src,
                                           profile=True)
                _, kms = _time_passes(plan, 3, 1, S_out=S, idx_out=idx, val_out=val)
                shares[f"K{K}_{src}_share{share}"] = {"kernel_ms": float(np.median(kms[:, 1])),
                                                      "grid_groups": plan.info().grid_groups,
                                                      "lds_bytes": plan.info().lds_bytes}
                plan.close()
    print(json.dumps({"workload": "baseline: 1000 ZTF-like curves, 1e5 freqs 0.05-50 /d, M=20, periodogram + top-5, "
                                  "marginalised Chebyshev baseline of K terms (K=0: Eq. 1)",
                      "evals": evals, "value": res["K3"]["G_evals_per_s"], "unit": "G evals/s", "per_K": res,
                      "kernel_ms_by_shape": shares}),
          flush=True)


def bench_uneven(args):
    """1e5 curves of lognormal length (50-2000), 2e5 frequencies, M in {10, 20, 40}, fused top-5 only."""
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    batch = synth.uneven_batch(args.curves or 100_000)
    log(f"generated {batch.n_curves} curves ({batch.n_points} points) in {time.perf_counter() - t0:.1f} s")
    evals = batch.evals()
    res = {}
    total_ms = 0.0
    for M in (10, 20, 40):
        plan = fpw.Plan.from_batch(batch, n_bins=M, topk=5, profile=True)
        idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
        val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
        wall, kms = _time_passes(plan, max(1, min(args.steps, 3)), 1, store_s=False, idx_out=idx, val_out=val, topk=True)
        info = plan.info()
        total_ms += wall * 1e3
        res[f"M{M}"] = {"ms_per_pass": wall * 1e3, "G_evals_per_s": evals / wall / 1e9,
                        "kernel_ms": float(kms[:, 1].mean()), "merge_ms": float(kms[:, 2].mean()),
                        "chunk_freqs": info.chunk_freqs, "grid_groups": info.grid_groups,
                        "roofline": _roofline(evals, batch.n_curves, len(batch.freqs), M, batch.n_points,
                                              float(kms[:, 1].mean()))}
        log(f"M={M}: {wall * 1e3:.1f} ms/pass, {evals / wall / 1e9:.0f} G evals/s")
        plan.close()
        del idx, val
    # the three bin counts from one M = 40 pass (Sec. 3.4): offsets 0 only, then every offset
    multi = {}
    for all_off in (False, True):
        plan = fpw.Plan.from_batch(batch, n_bins=40, derived_bins=(20, 10), all_offsets=all_off, topk=5, profile=True)
        nv = plan.n_variants
        idx = torch.empty((nv, batch.n_curves, 5), dtype=torch.int32, device="cuda")
        val = torch.empty((nv, batch.n_curves, 5), dtype=torch.float32, device="cuda")
        wall, kms = _time_passes(plan, max(1, min(args.steps, 3)), 1, store_s=False, idx_out=idx, val_out=val, topk=True)
        multi["all_offsets" if all_off else "offset0"] = {
            "variants": nv, "ms_per_pass": wall * 1e3, "kernel_ms": float(kms[:, 1].mean()),
            "merge_ms": float(kms[:, 2].mean()),
            "speedup_vs_three_passes": total_ms / (wall * 1e3)}
        log(f"multi-M (40 -> 20, 10; {nv} variants): {wall * 1e3:.1f} ms/pass")
        plan.close()
        del idx, val
    cpu = None
    if not args.no_cpu_baseline:
        b20 = batch.subset(range(min(batch.n_curves, 4096)))
        b20.n_bins = 20
        cpu = cpu_baseline(b20, args.cpu_seconds)
        cpu["extrapolated_full_s"] = evals / (cpu["value"] * 1e9)  # one M over the whole batch
        cpu["sample"] = "M=20: " + cpu["sample"]
        log(f"cpu baseline: {cpu['value']:.4f} G evals/s on {cpu['cores']} cores")
    print(json.dumps({"workload": f"uneven: {batch.n_curves} curves (N lognormal 50-2000, sum {batch.n_points}), "
                                  f"{len(batch.freqs)} freqs 0.05-50 /d, M in {{10,20,40}}, top-5, periodogram not stored",
                      "evals_per_M": evals, "total_ms_three_M": total_ms,
                      "value": 3 * evals / (total_ms * 1e-3) / 1e9, "unit": "G evals/s", "per_M": res,
                      "multi_M_one_pass": multi, "cpu_baseline": cpu}), flush=True)


def bench_stress(args):
    """2e4 curves x 3000 points over 2000 d, 1e6 frequencies to 200 /d, M = 50, top-5; FP64 comparator on a subset."""
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    batch = synth.stress_batch(args.curves or 20_000)
    evals = batch.evals()
    plan = fpw.Plan.from_batch(batch, topk=5, profile=True)
    idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
    val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
    wall, kms = _time_passes(plan, 1, 1, store_s=False, idx_out=idx, val_out=val, topk=True)
    info = plan.info()
    log(f"stress: {wall:.2f} s/pass, {evals / wall / 1e9:.0f} G evals/s")
    plan.close()
    # batched vs plain FP64 on the same 200-curve subset (the comparator stores the periodogram)
    sub = batch.subset(range(min(200, batch.n_curves)))
    ps = fpw.Plan.from_batch(sub, profile=True)
    wall_s, kms_s = _time_passes(ps, 2, 1, store_s=True, topk=False)
    fp = _fp64_rate(ps, sub.evals())
    ps.close()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch.subset(range(min(batch.n_curves, 256))), args.cpu_seconds, freq_stride=10)
        cpu["extrapolated_full_s"] = evals / (cpu["value"] * 1e9)
        log(f"cpu baseline: {cpu['value']:.4f} G evals/s on {cpu['cores']} cores")
    print(json.dumps({"workload": f"stress: {batch.n_curves} curves x 3000 points over 2000 d, "
                                  f"{len(batch.freqs)} freqs 0.01-200 /d, M=50, top-5, periodogram not stored",
                      "evals": evals, "s_per_pass": wall, "value": evals / wall / 1e9, "unit": "G evals/s",
                      "chunk_freqs": info.chunk_freqs, "grid_groups": info.grid_groups,
                      "roofline": _roofline(evals, batch.n_curves, len(batch.freqs), 50, batch.n_points,
                                            float(kms[:, 1].mean())),
                      "subset200": {"batched_G_evals_per_s": sub.evals() / wall_s / 1e9,
                                    "fp64_plain": fp, "speedup": (sub.evals() / wall_s / 1e9) / fp["value"]},
                      "cpu_baseline": cpu}),
          flush=True)


def single_curve_latency(passes):
    """Back-to-back µs per pass of one curve (200 points, 1e4 frequencies, M = 10, top-1), outputs
    preallocated: (default plan = fused pass, three-kernel pass)."""
    import torch

    from paper_2502_00243_amd import fpw, synth

    b1 = synth.single_curve()
    S1 = torch.empty((1, len(b1.freqs)), dtype=torch.float32, device="cuda")
    i1 = torch.empty((1, 1), dtype=torch.int32, device="cuda")
    v1 = torch.empty((1, 1), dtype=torch.float32, device="cuda")
    lats = []
    for fuse in (0, -1):
        p1 = fpw.Plan.from_batch(b1, topk=1, fuse_prepare=fuse)
        for _ in range(3):
            p1.eval(S_out=S1, idx_out=i1, val_out=v1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(passes):
            p1.eval(S_out=S1, idx_out=i1, val_out=v1)
        torch.cuda.synchronize()
        lats.append((time.perf_counter() - t1) / passes * 1e6)
        p1.close()
    return lats[0], lats[1]


def bench_latency(args):
    import torch

    torch.cuda.set_device(0)
    fused, three = single_curve_latency(max(50, args.steps * 10))
    print(json.dumps({"workload": "single light curve: 200 points over 1000 d, 1e4 frequencies 0.01-10 /d, M=10, "
                                  "S + top-1, outputs preallocated, passes back to back",
                      "latency_us": fused, "latency_three_kernels_us": three, "unit": "us per pass",
                      "passes": max(50, args.steps * 10)}), flush=True)


def bench_small(args):
    """Small and mid-size plans (N ~ U(100, 1000), M = 20, S + top-5): µs per pass back to back with
    the fused pass forced on and off; one JSON line per plan size."""
    import numpy as np
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for C in (1, 4, 16, 64, 256, 1000):
        for nf in (1000, 10000, 100000):
            if C * nf > 2e7:
                continue
            freqs = np.linspace(0.05, 50.0, nf)
            b = synth.random_batch(5, C, 100, 1000, freqs, 20)
            us = {}
            for fuse in (1, -1):
                p = fpw.Plan.from_batch(b, topk=5, fuse_prepare=fuse)
                S = torch.empty((C, nf), dtype=torch.float32, device="cuda")
                i = torch.empty((C, 5), dtype=torch.int32, device="cuda")
                v = torch.empty((C, 5), dtype=torch.float32, device="cuda")
                for _ in range(3):
                    p.eval(S_out=S, idx_out=i, val_out=v)
                torch.cuda.synchronize()
                reps = 20 if C * nf < 1e6 else 5
                t = time.perf_counter()
                for _ in range(reps):
                    p.eval(S_out=S, idx_out=i, val_out=v)
                torch.cuda.synchronize()
                us[fuse] = (time.perf_counter() - t) / reps * 1e6
                p.close()
            default = fpw.Plan.from_batch(b, topk=5)
            chosen = "fused" if default.info().fuse_prepare else "three-kernel"
            default.close()
            items64 = C * ((nf + 63) // 64)
            print(json.dumps({"workload": "small", "n_curves": C, "n_freq": nf, "n_points": int(b.n_points),
                              "evals": int(b.n_points) * nf, "items64_per_cu": items64 / n_cu,
                              "fused_us": us[1], "three_kernel_us": us[-1], "default": chosen}), flush=True)


def bench_precision(args):
    """Phase arithmetic study on the ztf1000 data: bin flips, S error and speed of each phase mode."""
    import numpy as np
    import torch

    import oracle
    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    batch = synth.ztf_batch()
    evals = batch.evals()
    rng = np.random.default_rng(3)
    curves = rng.choice(batch.n_curves, 24, replace=False)
    fidx = np.sort(rng.choice(len(batch.freqs), 400, replace=False))
    # oracle references for the sample
    refs = {}
    for c in curves:
        t, y, dy = batch.curve(int(c))
        tau, w, x = oracle.prepare_curve(t, y, dy)
        f = batch.freqs[fidx]
        ob = oracle.phase_bins(tau[None, :], f[:, None], batch.n_bins)
        near = oracle.edge_distance(tau[None, :], f[:, None], batch.n_bins) < oracle.EPS_BIN
        S = np.array([oracle.statistic(*oracle.bin_sums(ob[r], w, x, batch.n_bins)[:2]) for r in range(len(f))])
        refs[int(c)] = (ob, near, S)
    out = {}
    for phase in ("fp64", "fp64_listing", "df32", "fp32"):
        plan = fpw.Plan.from_batch(batch, topk=5, phase=phase, profile=True)
        S_gpu = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
        wall, kms = _time_passes(plan, 5, 2, S_out=S_gpu, topk=False)
        S_host = S_gpu.cpu().numpy()
        flips = total = flips_off = 0
        rel = []
        for c, (ob, near, S) in refs.items():
            gb = plan.debug_bins(c, 0, len(batch.freqs)).cpu().numpy()[fidx]
            d = gb != ob
            flips += int(d.sum())
            flips_off += int((d & ~near).sum())
            total += d.size
            r = np.abs(S_host[c, fidx] - S) / np.maximum(S, 1e-300)
            rel.append(r)
        rel = np.concatenate(rel)
        out[phase] = {"kernel_ms": float(kms[:, 1].mean()), "G_evals_per_s": evals / (kms[:, 1].mean() * 1e-3) / 1e9,
                      "bin_flip_fraction": flips / total, "off_edge_flip_fraction": flips_off / total,
                      "S_rel_err_median": float(np.median(rel)), "S_rel_err_p99": float(np.quantile(rel, 0.99)),
                      "S_rel_err_max": float(rel.max())}
        log(f"{phase}: {out[phase]}")
        plan.close()
    base = out["fp64"]["kernel_ms"]
    for ph in out:
        out[ph]["speed_vs_fp64"] = base / out[ph]["kernel_ms"]
    print(json.dumps({"workload": "precision study on the ztf1000 data (1000 curves, 1e5 freqs, M=20); "
                                  "bins and S checked on 24 curves x 400 sampled frequencies against the FP64 oracle",
                      "modes": out}), flush=True)


def bench_sweep(args):
    """Kernel time of each point source, histogram sharing and bin count on the ztf1000 data (one JSON line per shape)."""
    import numpy as np
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    batch = synth.ztf_batch()
    evals = batch.evals()
    S = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
    idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
    val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
    for M in (10, 20, 32, 40, 50, 64, 80, 100, 160):
        for src in ("scalar", "dpp"):
            for share in (1, 2, 4):
                plan = fpw.Plan.from_batch(batch, n_bins=M, topk=5, point_source=src, hist_share=share, profile=True)
                info = plan.info()
                _, kms = _time_passes(plan, 4, 1, S_out=S, idx_out=idx, val_out=val)
                k = float(np.median(kms[:, 1]))
                print(json.dumps({"M": M, "point_source": src, "hist_share": share, "chunk_freqs": info.chunk_freqs,
                                  "grid_groups": info.grid_groups, "lds_bytes": info.lds_bytes,
                                  "kernel_ms": k, "G_evals_per_s": evals / (k * 1e-3) / 1e9,
                                  "roofline_frac": _roofline(evals, batch.n_curves, len(batch.freqs), M, batch.n_points, k)["frac"]}),
                      flush=True)
                plan.close()
    # several bin counts from one pass (M = 40 giving 20 and 10): offset 0 only and every offset
    Sv = torch.empty((8, batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
    idv = torch.empty((8, batch.n_curves, 5), dtype=torch.int32, device="cuda")
    vav = torch.empty((8, batch.n_curves, 5), dtype=torch.float32, device="cuda")
    for all_offsets in (False, True):
        for src in ("scalar", "dpp"):
            for share in (1, 2, 4):
                plan = fpw.Plan.from_batch(batch, n_bins=40, derived_bins=(20, 10), all_offsets=all_offsets, topk=5,
                                           point_source=src, hist_share=share, profile=True)
                nv = plan.n_variants
                _, kms = _time_passes(plan, 4, 1, S_out=Sv[:nv], idx_out=idv[:nv], val_out=vav[:nv])
                k = float(np.median(kms[:, 1]))
                print(json.dumps({"M": 40, "derived": [20, 10], "all_offsets": all_offsets, "variants": nv,
                                  "point_source": src, "hist_share": share, "kernel_ms": k}), flush=True)
                plan.close()
    del Sv, idv, vav
    # launch shapes of the headline configuration (M = 20, scalar source)
    for fl in (1, 2):
        for wpg in (1, 2, 4):
            for chunk in (0, 1024, 4096):
                plan = fpw.Plan.from_batch(batch, topk=5, point_source="scalar", freqs_per_lane=fl, waves_per_group=wpg,
                                           chunk_freqs=chunk, profile=True)
                info = plan.info()
                _, kms = _time_passes(plan, 4, 1, S_out=S, idx_out=idx, val_out=val)
                k = float(np.median(kms[:, 1]))
                print(json.dumps({"M": 20, "freqs_per_lane": fl, "waves_per_group": wpg, "chunk_freqs": info.chunk_freqs,
                                  "grid_groups": info.grid_groups, "kernel_ms": k,
                                  "G_evals_per_s": evals / (k * 1e-3) / 1e9}), flush=True)
                plan.close()


if __name__ == "__main__":
    main()
