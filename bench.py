#!/usr/bin/env python3
"""FPW periodogram benchmark on one MI355X.

Workload (default): the long-baseline stress batch, the largest
configuration one GPU holds: 2e4 synthetic light curves of 3000 times
uniform over 2000 d (mixed waveforms at SNR 3-20, lognormal errors),
1e6 trial frequencies on 0.01-200 /d (fold products up to 4e5 cycles),
M = 50 phase bins, top-5 peaks per curve (the 80 GB periodogram is not
stored).  6e13 observation x frequency evaluations per pass.

One step = one fpw_eval_batch pass over the batch, inputs resident in HBM:
prepare (weights, centring, offsets, fixed-point packing) -> fold / bin /
accumulate / reduce with fused peak selection -> per-curve peak merge,
replayed as one hipGraph.  Beside it: the batched kernel's duration from a
profiled pass (HIP events on its stream) for the roofline, the plain
per-curve FP64 kernel against the batched one on a 1000-curve subset at the
full grid, the FP64 oracle on the host cores over a bounded sample, the
1000-curve ZTF-like batch (1e5 frequencies, M = 20) and the single-curve
latency.  Prints one JSON line.
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
TRAFFIC_FILE_STRESS = os.path.join(ROOT, "profiles", "traffic_batched_stress.json")
DTYPE = "f64-fold/i32-fixed-sums/f32-stat"  # FP64 phase and bin, exact 32-bit fixed-point bin sums, FP32 statistic
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

    # one worker per core of the machine's CPU share (16 per GPU), never more than the affinity mask allows
    available = len(os.sched_getaffinity(0))
    cores = max(1, min(16, available))
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
        "cores_available": available,
        "kind": "oracle",
        "sample": f"first {n_sample} of {batch.n_curves} curves x {grid} "
        f"({evals:.3g} evals, {wall:.1f} s wall, one single-threaded NumPy process per core, {cpu})",
        "extrapolated_full_s": batch.evals() / (value * 1e9),
    }


# ---------------------------------------------------------------- GPU
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--phase", default="fp64", choices=["fp64", "fp64_listing", "df32", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-latency", action="store_true", help="skip the single-curve latency run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--workload", default="stress",
                    choices=["ztf1000", "uneven", "stress", "precision", "sweep", "shared", "baseline", "latency",
                             "small"],
                    help="stress: the headline line (default): 2e4 x 3000-point curves, 1e6 freqs, M=50, top-5; "
                         "ztf1000: 1000 ZTF-like curves, 1e5 freqs, M=20, periodogram + top-5; "
                         "uneven: 1e5 uneven curves, 2e5 freqs, M in {10,20,40}, top-5; "
                         "precision: phase-arithmetic study on the ztf1000 data; "
                         "sweep: launch shapes x M on the ztf1000 data; "
                         "shared: 1000 curves at 500 common epochs, 1e5 freqs, M=20, matrix-core vs general kernel; "
                         "baseline: the ztf1000 data with a marginalised 3-term baseline (App. A general case); "
                         "latency: one curve of 200 points, 1e4 freqs, M=10, fused vs three-kernel pass; "
                         "small: plans of 1-1000 curves x 1e3-1e5 freqs, fused vs three-kernel pass")
    ap.add_argument("--curves", type=int, default=0, help="curve count override for uneven/stress")
    ap.add_argument("--kernel-only", action="store_true",
                    help="headline: only the timed graph passes (for profiler runs): no profiled pass, comparator, "
                         "CPU baseline, 1000-curve line or latency")
    ap.add_argument("--plain-curves", type=int, default=1000,
                    help="curves of the subset on which the plain FP64 kernel is timed against the batched one")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the FPW build has no multi-GPU path "
              "(curves shard across GPUs with no collective in the hot loop; see the design notes).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "uneven":
        return bench_uneven(args)
    if args.workload == "stress":
        return bench_headline(args)
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

    return bench_ztf1000(args)


# ---------------------------------------------------------------- timing helpers
def graph_passes(plan, steps, warmup, **kw):
    """Passes replayed from the plan's captured graph: (wall seconds per pass, HIP-event ms of each pass).

    The events are recorded on torch's current stream, the stream fpw_eval_batch launches the graph on;
    the timed region is bracketed by device synchronisations."""
    import torch

    for _ in range(warmup):
        plan.eval(**kw)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        plan.eval(**kw)
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return wall, [a.elapsed_time(b) for a, b in ev]


def profiled_kernel_ms(batch, passes, warmup=1, store_s=False, **opts):
    """Kernel durations (prepare, fold, merge) in ms, averaged over `passes` passes of a plan made with
    profile=True (after `warmup` untimed ones): HIP events recorded by the library on the stream each
    kernel runs on (direct launches); the passes store S or not as `store_s` says."""
    import numpy as np
    import torch

    from paper_2502_00243_amd import fpw

    plan = fpw.Plan.from_batch(batch, profile=True, **opts)
    S = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda") if store_s else None
    for _ in range(warmup):
        plan.eval(S_out=S, store_s=store_s)
    kms = []
    for _ in range(passes):
        plan.eval(S_out=S, store_s=store_s)
        pre, fold, merge = plan.timings()
        wide = plan.wide_ms()
        kms.append((pre, fold - wide, merge, wide))  # the batched kernel alone, then the wide one
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return np.asarray(kms).mean(axis=0), info


def copy_calibration():
    """A 256 MiB device copy: the reference that scales the HBM byte counters of a PMC run."""
    import torch

    src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _traffic(path, workload):
    if os.path.exists(path):
        tr = json.load(open(path))
        if tr.get("kernel_sha") == kernel_hash() and tr.get("workload") == workload:
            return tr.get("hbm_bytes_per_launch")
    return None


def headline_roofline(evals, n_curves, n_freq, n_bins, n_points, kernel_ms, traffic):
    """The dominant kernel against the VALU roofline: 6 algorithmic lane-ops per evaluation (fold product,
    fractional part, scale, bin index, two accumulates) plus 6M per (curve, frequency) for the bin
    reduction and reset, over the kernel's own duration; the LDS side (8 algorithmic bytes per evaluation)
    beside it.  evals, n_curves and n_points are the kernel's own (its curves)."""
    mean_n = n_points / n_curves
    ops = evals * 6.0 + n_curves * n_freq * 6.0 * n_bins
    achieved = ops / (kernel_ms * 1e-3)
    return {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": VALU_PEAK / 1e12,
        "unit": "T lane-ops/s",
        "frac": achieved / VALU_PEAK,
        "traffic": traffic,
        "kernel": "batched_kernel (fold/bin/accumulate/reduce + fused peaks)",
        "ops_per_eval": 6.0 + 6.0 * n_bins / mean_n,
        "ops_per_launch": ops,
        "evals_per_launch": evals,
        "kernel_ms": kernel_ms,
        "lds": {
            "bytes_per_eval": 8,
            "achieved_TBps": evals * 8 / (kernel_ms * 1e-3) / 1e12,
            "peak_TBps": LDS_PEAK / 1e12,
            "frac": evals * 8 / (kernel_ms * 1e-3) / LDS_PEAK,
        },
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------- the headline line
def bench_headline(args):
    """2e4 curves x 3000 points, 1e6 frequencies, M = 50, top-5 (the periodogram is not stored)."""
    import torch

    from paper_2502_00243_amd import fpw, synth

    t_gen = time.perf_counter()
    batch = synth.stress_batch(args.curves or 20_000)
    log(f"generated {batch.n_curves} curves ({batch.n_points} points) in {time.perf_counter() - t_gen:.1f} s")
    n_bins, n_freq = batch.n_bins, len(batch.freqs)
    evals = batch.evals()
    if args.kernel_only:
        args.no_cpu_baseline = args.no_fp64_plain = args.no_latency = True
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch.subset(range(min(batch.n_curves, 256))), args.cpu_seconds, freq_stride=10)
        cpu["extrapolated_full_s"] = evals / (cpu["value"] * 1e9)
        log(f"cpu baseline: {cpu['value']:.4f} G evals/s on {cpu['cores']} of {cpu['cores_available']} cores")

    torch.cuda.set_device(0)
    t_plan = time.perf_counter()
    plan = fpw.Plan.from_batch(batch, topk=5, phase=args.phase)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t_plan
    info = plan.info()
    log(f"planned in {plan_s:.1f} s: {info.work_items} items, chunk {info.chunk_freqs}, grid {info.grid_groups}, "
        f"{info.hist_share} waves per histogram, {info.n_wide_curves} wide curves")
    idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
    val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
    wall, ev_ms = graph_passes(plan, args.steps, args.warmup, store_s=False, idx_out=idx, val_out=val, topk=True)
    value = evals / wall / 1e9
    log(f"{wall:.3f} s per pass (events {min(ev_ms):.1f}-{max(ev_ms):.1f} ms) -> {value:.1f} G evals/s")
    plan.close()

    if args.copy_calibration:
        copy_calibration()
    if args.kernel_only:
        print(json.dumps({"workload": "stress", "value": value, "ms_per_step": wall * 1e3, "steps": args.steps,
                          "pass_event_ms": ev_ms}), flush=True)
        return

    # the batched kernel's own duration, from a profiled pass of the same plan
    # (no warm-up: a cold first launch adds ~1 ms to a 9.6 s kernel)
    kms, _ = profiled_kernel_ms(batch, 1, warmup=0, topk=5, phase=args.phase)
    log(f"profiled pass: prepare {kms[0]:.2f} ms, batched {kms[1]:.1f} ms, wide {kms[3]:.2f} ms, "
        f"merge {kms[2]:.2f} ms")
    # the batched kernel folds the narrow-format curves (the wide-format ones go to the wide kernel)
    n_narrow, p_narrow = batch.n_curves - info.n_wide_curves, batch.n_points - info.n_wide_points
    roofline = headline_roofline(p_narrow * n_freq, n_narrow, n_freq, n_bins, p_narrow, float(kms[1]),
                                 _traffic(TRAFFIC_FILE_STRESS, "stress"))

    # batched mixed-precision form vs the plain per-curve FP64 kernel, same curves, full grid
    plain = None
    if not args.no_fp64_plain:
        sub = batch.subset(range(min(args.plain_curves, batch.n_curves)))
        ps = fpw.Plan.from_batch(sub, topk=5, phase=args.phase)
        S = torch.empty((sub.n_curves, n_freq), dtype=torch.float32, device="cuda")
        wall_b, _ = graph_passes(ps, 2, 1, S_out=S, topk=False)
        # one comparator call (a thousand launches of seconds in all): timed with events on its stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        S64 = ps.eval_fp64()
        e1.record()
        torch.cuda.synchronize()
        fp = {"value": sub.evals() / (e0.elapsed_time(e1) * 1e-3) / 1e9, "ms": e0.elapsed_time(e1)}
        # agreement where S is not a cancellation residue (median and p99 over a sample, the fraction above
        # 1e-5 and the max over all): the two kernels fold in different FP64 orders (fused vs listing), so a
        # point within ~1e-8 bin widths of an edge may take either bin, and such a point moves S by O(1)
        rel = (S.double() - S64).abs() / S64.abs().clamp_min(1e-30)
        relb = rel[S64 > 1e-3 * S64.amax(dim=1, keepdim=True)]
        smp = relb[:: max(1, relb.numel() // 4_000_000)]
        agree = {"median": float(smp.median()), "p99": float(torch.quantile(smp, 0.99)),
                 "frac_above_1e-5": float((relb > 1e-5).double().mean()), "max": float(relb.max()),
                 "note": "values above 1e-5 come from points within ~1e-8 bin widths of an edge, which the "
                         "fused and the listing-order FP64 folds may place in neighbouring bins"}
        # the batched kernel folding in the listing order bins every point exactly as the comparator does
        pl = fpw.Plan.from_batch(sub, topk=5, phase="fp64_listing")
        pl.eval(S_out=S, topk=False)
        torch.cuda.synchronize()
        rel = (S.double() - S64).abs() / S64.abs().clamp_min(1e-30)
        relb = rel[S64 > 1e-3 * S64.amax(dim=1, keepdim=True)]
        agree["listing_order_batched"] = {"frac_above_1e-5": float((relb > 1e-5).double().mean()),
                                          "max": float(relb.max())}
        pl.close()
        del S64, rel, relb, smp, S
        ps.close()
        batched_rate = sub.evals() / wall_b / 1e9
        plain = {"value": fp["value"], "unit": "G evals/s", "ms": fp["ms"],
                 "kernel": "plain per-curve FP64 kernel (listing-order FP64 fold, FP64 LDS sums, FP64 statistic), "
                           "one launch per curve",
                 "subset": f"first {sub.n_curves} of {batch.n_curves} curves x all {n_freq} frequencies "
                           f"({sub.evals():.3g} evals)",
                 "batched_same_subset": batched_rate,
                 "speedup": batched_rate / fp["value"],
                 "S_rel_diff_vs_batched": agree}
        log(f"plain FP64 on {sub.n_curves} curves: {fp['value']:.1f} G evals/s; batched {batched_rate:.1f}; "
            f"S agreement median {agree['median']:.2e} max {agree['max']:.2e}")

    config2 = ztf1000_summary(args)
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
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {
            "workload": f"long-baseline stress: {batch.n_curves} light curves x 3000 times uniform over 2000 d, "
                        f"{n_freq} trial frequencies 0.01-200 /d, M={n_bins}, top-5 peaks per curve "
                        f"(periodogram not stored), FP64 fold",
            "n_curves": batch.n_curves,
            "n_points": batch.n_points,
            "n_freq": n_freq,
            "n_bins": n_bins,
            "evals_per_step": evals,
            "phase": args.phase,
            "timed_path": "fpw_eval_batch replayed from its captured hipGraph (prepare, batched kernel, merge)",
            "plan_s": plan_s,
            "launch": {"freqs_per_lane": info.freqs_per_lane, "waves_per_group": info.waves_per_group,
                       "hist_share": info.hist_share, "chunk_freqs": info.chunk_freqs,
                       "grid_groups": info.grid_groups, "work_items": info.work_items, "lds_bytes": info.lds_bytes,
                       "wide_curves": info.n_wide_curves},
        },
        "pass_event_ms": {"min": min(ev_ms), "max": max(ev_ms), "mean": sum(ev_ms) / len(ev_ms)},
        "kernel_ms": {"prepare": float(kms[0]), "batched": float(kms[1]), "wide": float(kms[3]),
                      "merge": float(kms[2])},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_plain": plain,
        "speedup_vs_fp64_plain": plain["speedup"] if plain else None,
        "config2_ztf1000": config2,
        "latency_single_curve_us": lat_us,
        "latency_single_curve_three_kernels_us": lat3_us,
    }
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- 1000 ZTF-like curves
def ztf1000_summary(args, steps=20, warmup=3):
    """The 1000-curve ZTF-like batch (1e5 frequencies, M = 20, periodogram + top-5), graph-replayed,
    with the batched kernel's duration from a profiled pass."""
    import torch

    from paper_2502_00243_amd import fpw, synth

    batch = synth.ztf_batch()
    evals = batch.evals()
    plan = fpw.Plan.from_batch(batch, topk=5, phase=args.phase)
    S = torch.empty((batch.n_curves, len(batch.freqs)), dtype=torch.float32, device="cuda")
    idx = torch.empty((batch.n_curves, 5), dtype=torch.int32, device="cuda")
    val = torch.empty((batch.n_curves, 5), dtype=torch.float32, device="cuda")
    wall, ev_ms = graph_passes(plan, steps, warmup, S_out=S, idx_out=idx, val_out=val)
    info = plan.info()
    plan.close()
    kms, _ = profiled_kernel_ms(batch, 10, warmup=2, store_s=True, topk=5, phase=args.phase)
    roof = headline_roofline(evals, batch.n_curves, len(batch.freqs), batch.n_bins, batch.n_points, float(kms[1]),
                             _traffic(TRAFFIC_FILE, "ztf1000"))
    log(f"ztf1000: {wall * 1e3:.3f} ms per pass -> {evals / wall / 1e9:.1f} G evals/s; batched {kms[1]:.3f} ms, "
        f"frac {roof['frac']:.3f}")
    return {"workload": "1000 ZTF-like light curves (N~U(100,1000), 1500 d, seasonal gaps), 1e5 trial frequencies "
                        "0.05-50 /d, M=20, periodogram stored + top-5 peaks",
            "value": evals / wall / 1e9, "unit": "G evals/s", "ms_per_step": wall * 1e3, "steps": steps,
            "evals_per_step": evals, "kernel_ms": {"prepare": float(kms[0]), "batched": float(kms[1]),
                                                   "merge": float(kms[2])},
            "hist_share": info.hist_share, "chunk_freqs": info.chunk_freqs, "roofline": roof}


def bench_ztf1000(args):
    """The 1000-curve ZTF-like batch as its own line, with the FP64 comparator and the CPU baseline."""
    from paper_2502_00243_amd import synth

    batch = synth.ztf_batch()
    cpu = None if args.no_cpu_baseline else cpu_baseline(batch, args.cpu_seconds)
    import torch

    from paper_2502_00243_amd import fpw

    torch.cuda.set_device(0)
    summary = ztf1000_summary(args, steps=max(args.steps, 20), warmup=max(args.warmup, 3))
    if args.copy_calibration:
        copy_calibration()
    plain = None
    if not args.no_fp64_plain:
        plan = fpw.Plan.from_batch(batch, topk=5, phase=args.phase)
        plain = _fp64_rate(plan, batch.evals())
        plan.close()
    print(json.dumps({**summary, "metric": METRIC, "dtype": DTYPE, "cpu_baseline": cpu, "fp64_plain": plain,
                      "speedup_vs_fp64_plain": summary["value"] / plain["value"] if plain else None}), flush=True)


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
    matrix kernel is bound by instruction issue: its matrix products and its
    VALU work (one-hot operands, folds, epilogue) do not overlap, and PMC
    counters put them at about 52 % and 49 % of the SIMD cycles.  Its line
    therefore reports the bound as "issue", with two live figures beside it:
    the per-evaluation model of the general kernel (6 + 6M/N lane-ops per
    evaluation against the VALU peak; above 1 it only says the fold is
    shared by the field's curves) and the int8 contraction it performs (rows
    (curve, quantity, digit) = 8 per curve, columns (frequency, bin) = M per
    frequency, depth = points: 16 M int8 operations per evaluation, a dense
    equivalent, not the method's work) against the dense int8 peak.
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
            r["roofline"] = {
                "bound": "issue",
                "note": "matrix products and VALU work do not overlap: MFMA busy ~52 % plus VALU issue ~49 % of "
                        "SIMD cycles (profiles/pmc_shared_field1000.md); every VALU instruction removed shortens it",
                "kernel_ms": kernel_ms,
                "per_eval_model": _roofline(evals, batch.n_curves, len(batch.freqs), M, batch.n_points, kernel_ms),
                "int8_contraction": {"achieved": ops / (kernel_ms * 1e-3) / 1e12, "peak": INT8_PEAK / 1e12,
                                     "unit": "T int8 ops/s", "frac": ops / (kernel_ms * 1e-3) / INT8_PEAK,
                                     "ops_per_eval": 16.0 * M}}
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
        t_warm = time.perf_counter()  # steady-state clocks first (see bench_small)
        while time.perf_counter() - t_warm < 0.2:
            for _ in range(20):
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
    the fused pass forced on and off; one JSON line per plan size.  Each plan first runs passes back to
    back for 200 ms: the GPU lowers its clocks when idle for a fraction of a second, and passes this
    short, timed after a few warm-up passes only, measured 6-10 % slower than in steady state."""
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
                t_warm = time.perf_counter()
                while time.perf_counter() - t_warm < 0.2:  # synchronised: the host must not queue ahead
                    p.eval(S_out=S, idx_out=i, val_out=v)
                    torch.cuda.synchronize()
                reps = 50 if C * nf < 1e6 else 20
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
    """Phase arithmetic study over the whole ztf1000 data (1000 curves, 1e5 freqs, M = 20: 5.47e10
    evaluations per mode): speed, bin flips and S error of each phase mode.

    Both references run on the GPU.  Bins: the listing-order FP64 fold (the fold rule's own steps in
    FP64, which the parity tests find bit-identical to the oracle's bins); a flip counts as off-edge
    when that point lies at least 1e-6 bin widths from an edge (distance from tau f in FP64).  S: the
    plain per-curve FP64 comparator (listing-order FP64 fold, FP64 sums and statistic), which the
    parity tests check against the oracle.  The parity bar is |dS| <= 1e-5 S + 1e-7 S_abs, where
    S_abs = sum_m (sum over bin m of |w x|)^2 / (W_m + 1/alpha^2) is the statistic of |x| with no
    further centring (a plan of its own over |y - mu|, mu the weighted mean); per mode the line reports
    the fraction that needed the second term (the cancellation guard) and the fraction beyond both
    (near-edge points that the mode and the listing-order reference place in neighbouring bins)."""
    import numpy as np
    import torch

    from paper_2502_00243_amd import fpw, synth

    torch.cuda.set_device(0)
    batch = synth.ztf_batch()
    C, F, M = batch.n_curves, len(batch.freqs), batch.n_bins
    evals = batch.evals()
    ref = fpw.Plan.from_batch(batch, phase="fp64_listing")
    S64 = ref.eval_fp64()
    w = 1.0 / (batch.dy * batch.dy)
    seg = np.repeat(np.arange(C), np.diff(batch.offsets))
    mu = np.bincount(seg, weights=w * batch.y, minlength=C) / np.bincount(seg, weights=w, minlength=C)
    p_abs = fpw.Plan(batch.offsets, batch.t, np.abs(batch.y - mu[seg]), batch.dy, batch.freqs, M, center="none",
                     phase="fp64_listing")
    S_abs = p_abs.eval(topk=False)[0].double()
    p_abs.close()
    torch.cuda.synchronize()
    freqs_d = torch.as_tensor(batch.freqs, dtype=torch.float64, device="cuda")
    out = {}
    for phase in ("fp64", "fp64_listing", "df32", "fp32"):
        plan = fpw.Plan.from_batch(batch, topk=5, phase=phase, profile=True)
        S_gpu = torch.empty((C, F), dtype=torch.float32, device="cuda")
        _, kms = _time_passes(plan, 5, 2, S_out=S_gpu, topk=False)
        t0 = time.perf_counter()
        flips = off_edge = 0
        if phase != "fp64_listing":  # the reference bins themselves
            for c in range(C):
                d = plan.debug_bins(c, 0, F) != ref.debug_bins(c, 0, F)
                fi, pi = d.nonzero(as_tuple=True)
                flips += int(fi.numel())
                if fi.numel():
                    tau = torch.as_tensor(batch.curve(c)[0], dtype=torch.float64, device="cuda")  # t_ref = 0
                    u = tau[pi] * freqs_d[fi]
                    u = (u - torch.floor(u)) * M
                    off_edge += int(((u - torch.round(u)).abs() >= 1e-6).sum())
                del d, fi, pi
        err = (S_gpu.double() - S64).abs()
        bar = 1e-5 * S64.abs()
        guard_hits = float(((err > bar) & (err <= bar + 1e-7 * S_abs)).double().mean())
        beyond = float((err > bar + 1e-7 * S_abs).double().mean())
        del err, bar
        rel = ((S_gpu.double() - S64).abs() / S64.abs().clamp_min(1e-300)).flatten()
        srt = torch.sort(rel).values
        n = srt.numel()
        out[phase] = {"kernel_ms": float(kms[:, 1].mean()), "G_evals_per_s": evals / (kms[:, 1].mean() * 1e-3) / 1e9,
                      "bin_evals_compared": evals if phase != "fp64_listing" else 0,
                      "bin_flip_fraction": flips / evals, "off_edge_flip_fraction": off_edge / evals,
                      "bin_flips": flips, "off_edge_flips": off_edge,
                      "S_values_compared": n,
                      "S_rel_err_median": float(srt[n // 2]), "S_rel_err_p99": float(srt[int(0.99 * (n - 1))]),
                      "S_rel_err_p99_99": float(srt[int(0.9999 * (n - 1))]), "S_rel_err_max": float(srt[-1]),
                      "S_frac_above_1e-5": float((rel > 1e-5).double().mean()),
                      "guard_hit_fraction": guard_hits, "S_frac_beyond_bar": beyond}
        del rel, srt
        log(f"{phase}: {out[phase]} ({time.perf_counter() - t0:.1f} s of checks)")
        plan.close()
    ref.close()
    base = out["fp64"]["kernel_ms"]
    for ph in out:
        out[ph]["speed_vs_fp64"] = base / out[ph]["kernel_ms"]
    print(json.dumps({"workload": f"precision study over the whole ztf1000 data ({C} curves, {F} freqs 0.05-50 /d, "
                                  f"M={M}; {evals:.3g} evaluations per mode)",
                      "bin_reference": "listing-order FP64 fold on the GPU (fp64_listing bins)",
                      "S_reference": "plain per-curve FP64 comparator on the GPU (fpw_eval_fp64)",
                      "off_edge": "flip of a point at least 1e-6 bin widths from an edge",
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
