"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bins: identical off-edge (listing-order FP64: identical everywhere).
S: within 1e-5 relative of the oracle, with the cancellation guard.
Peaks: equal to the peak rule applied to the GPU's own S, and to the oracle's
top-k up to near-ties.
"""
import numpy as np
import pytest

import oracle
from paper_2502_00243_amd import synth
from tests import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU runs deselect this module with -m "not gpu"
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]
else:
    from paper_2502_00243_amd import fpw


def _say(msg):
    print(msg, flush=True)


def _check_plan_against_oracle(b, plan, opts, curves=None, exact_bins=False, freq_idx=None,
                               max_guard=parity.MAX_GUARD_FRACTION):
    """Compares S (and bins) of the selected curves with the oracle; returns the guard-hit fraction."""
    S_gpu, _, _ = plan.eval(topk=False)
    torch.cuda.synchronize()
    S_gpu = S_gpu.cpu().numpy()
    opt = parity.oracle_options(**opts)
    curves = range(b.n_curves) if curves is None else curves
    fi = np.arange(len(b.freqs)) if freq_idx is None else np.asarray(freq_idx)
    guard = []
    for c in curves:
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()[fi]
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[fi], plan.n_bins, opt, gpu_bins=gb,
                                                     exact_bins=exact_bins)
        guard.append(parity.assert_s_close(S_gpu[c, fi], S_ref, S_abs, what=f"curve {c}", max_guard=max_guard))
    _say(f"  guard fraction {np.mean(guard):.2e} (max per curve {np.max(guard):.2e})")
    return float(np.mean(guard)), S_gpu


@pytest.mark.parametrize("phase", ["fp64", "fp64_listing", "df32"])
def test_single_curve_full(phase):
    _say(f"single curve phase={phase}")
    b = synth.single_curve()
    plan = fpw.Plan.from_batch(b, phase=phase, topk=5)
    g, S_gpu = _check_plan_against_oracle(b, plan, {}, exact_bins=phase == "fp64_listing")
    assert g < 1e-3
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    idx, val = idx.cpu().numpy(), val.cpu().numpy()
    assert abs(b.freqs[idx[0, 0]] - 1 / 0.37) <= 2 * (b.freqs[1] - b.freqs[0])
    parity.assert_topk_matches_rule(S.cpu().numpy(), idx, val, 5)
    ref = oracle.curve_periodogram(*b.curve(0), b.freqs, b.n_bins)
    parity.assert_topk_near_oracle(ref, idx[0], val[0], 5)
    plan.close()


RAGGED = [
    # (seed, M, phase, freqs_per_lane, waves_per_group, chunk[, point source])
    (1, 10, "fp64", 1, 1, 128),
    (9, 10, "fp64", 1, 2, 128, "dpp"),
    (10, 20, "fp64_listing", 1, 1, 192, "dpp"),
    (11, 50, "fp64", 1, 1, 128, "scalar"),
    (12, 33, "df32", 1, 1, 64, "dpp"),
    (2, 20, "fp64", 2, 4, 256),
    (3, 1, "fp64", 1, 2, 128),
    (4, 3, "fp64_listing", 1, 1, 192),
    (5, 50, "fp64_listing", 2, 1, 128),
    (6, 7, "df32", 1, 4, 64),
    (7, 40, "fp64", 1, 4, 0),
    (8, 2, "fp64", 2, 2, 128),
]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: "-".join(map(str, c)))
def test_ragged_batch(case):
    """Uneven curves (1..300 points), 477 frequencies (ragged last tile), several chunks per curve."""
    seed, M, phase, fl, waves, chunk = case[:6]
    src = case[6] if len(case) > 6 else "auto"
    _say(f"ragged seed={seed} M={M} phase={phase} fl={fl} waves={waves} chunk={chunk} source={src}")
    freqs = np.linspace(0.05, 30.0, 477)
    b = synth.random_batch(seed, 12, 1, 300, freqs, M)
    plan = fpw.Plan.from_batch(b, phase=phase, topk=4, freqs_per_lane=fl, waves_per_group=waves, chunk_freqs=chunk,
                               point_source=src)
    if src != "auto":
        assert plan.info().point_source == (1 if src == "scalar" else 2)
    # with M <= 3 the bin sums of weighted-centred data nearly cancel at a few
    # frequencies per curve (for M = 2, Y_1 = -Y_0 exactly), where only the
    # guard can apply
    _check_plan_against_oracle(b, plan, {}, exact_bins=phase == "fp64_listing",
                               max_guard=1e-2 if M <= 3 else parity.MAX_GUARD_FRACTION)
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), 4)
    # standalone peak selection over the stored periodogram agrees bit for bit
    i2, v2 = plan.topk(torch.from_numpy(S).cuda(), 4)
    np.testing.assert_array_equal(i2.cpu().numpy(), idx.cpu().numpy())
    np.testing.assert_array_equal(v2.cpu().numpy(), val.cpu().numpy())
    plan.close()


@pytest.mark.parametrize(
    "opts",
    [
        dict(center="mean"),
        dict(center="none"),
        dict(tref="first"),
        dict(tref="given", t_ref=-3.25),
        dict(inv_alpha2=2.5e3),
        dict(stat_scale="listing_half"),
    ],
)
def test_options(opts):
    _say(f"options {opts}")
    freqs = np.linspace(0.1, 12.0, 300)
    b = synth.random_batch(11, 6, 20, 250, freqs, 12)
    plan = fpw.Plan.from_batch(b, **opts)
    _check_plan_against_oracle(b, plan, opts)
    plan.close()


def test_fp64_comparator():
    _say("fp64 comparator")
    freqs = np.linspace(0.05, 25.0, 700)
    b = synth.random_batch(21, 5, 1, 400, freqs, 16)
    plan = fpw.Plan.from_batch(b)
    S = plan.eval_fp64()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    ref = oracle.periodogram(b.offsets, b.t, b.y, b.dy, freqs, 16)
    for c in range(b.n_curves):
        t, y, dy = b.curve(c)
        tau, w, x = oracle.prepare_curve(t, y, dy)
        scale = np.sum(np.abs(w * x)) ** 2 / np.sum(w)
        assert np.all(np.abs(S[c] - ref[c]) <= 1e-10 * np.abs(ref[c]) + 1e-13 * scale), c
        gb = plan.debug_bins(c, 0, len(freqs), phase="fp64_listing").cpu().numpy()
        np.testing.assert_array_equal(gb, oracle.curve_bins(t, freqs, 16))
    plan.close()


def test_precision_study_references_on_ztf1000():
    """The precision study's references, on its own data (the 1000 ZTF-like curves at M = 20): the
    listing-order FP64 bins equal the oracle's bin for bin, and the FP64 comparator's S the oracle's
    within 1e-10, on four curves (the longest and shortest among them) at every 10th frequency."""
    _say("precision references on ztf1000")
    b = synth.ztf_batch()
    plan = fpw.Plan.from_batch(b, phase="fp64_listing")
    S = plan.eval_fp64()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    fi = np.arange(0, len(b.freqs), 10)
    for c in (int(np.argmax(b.lengths)), int(np.argmin(b.lengths)), 17, 503):
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()[fi]
        np.testing.assert_array_equal(gb, oracle.curve_bins(t, b.freqs[fi], b.n_bins), err_msg=f"curve {c}")
        ref = oracle.curve_periodogram(t, y, dy, b.freqs[fi], b.n_bins)
        tau, w, x = oracle.prepare_curve(t, y, dy)
        scale = np.sum(np.abs(w * x)) ** 2 / np.sum(w)
        assert np.all(np.abs(S[c, fi] - ref) <= 1e-10 * np.abs(ref) + 1e-13 * scale), c
    plan.close()


def test_edge_cases():
    _say("edge cases")
    # one frequency; two frequencies; curves of one point; M at its maximum
    for nf, M in ((1, 5), (2, 5), (65, 255), (130, 64)):
        freqs = np.linspace(0.3, 5.0, nf)
        b = synth.random_batch(30 + nf, 4, 1, 40, freqs, M)
        k = min(3, nf)
        plan = fpw.Plan.from_batch(b, topk=k, chunk_freqs=64)
        _check_plan_against_oracle(b, plan, {})
        S, idx, val = plan.eval()
        torch.cuda.synchronize()
        parity.assert_topk_matches_rule(S.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), k)
        plan.close()


def test_graph_replays_are_identical():
    _say("graph replays")
    freqs = np.linspace(0.05, 20.0, 999)
    b = synth.random_batch(41, 9, 50, 500, freqs, 20)
    plan = fpw.Plan.from_batch(b, topk=5, fuse_prepare=-1)  # (the fused pass of small plans is not captured)
    outs = []
    for _ in range(3):
        S, idx, val = plan.eval()
        torch.cuda.synchronize()
        outs.append((S.cpu().numpy().copy(), idx.cpu().numpy().copy(), val.cpu().numpy().copy()))
        # eager work between replays
        torch.ones(1000, device="cuda").sum().item()
    for o in outs[1:]:
        for a, b_ in zip(outs[0], o):
            np.testing.assert_array_equal(a, b_)
    plan2 = fpw.Plan.from_batch(b, topk=5, use_graph=False, fuse_prepare=-1)
    S2, i2, v2 = plan2.eval()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S2.cpu().numpy(), outs[0][0])
    np.testing.assert_array_equal(i2.cpu().numpy(), outs[0][1])
    plan.close()
    plan2.close()


def test_ztf1000_full_size_sampled():
    """The benchmark's workload and launch configuration; sampled outputs against the oracle."""
    _say("ztf1000 full size")
    b = synth.ztf_batch()
    plan = fpw.Plan.from_batch(b, topk=5)
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    idx, val = idx.cpu().numpy(), val.cpu().numpy()
    assert np.isfinite(S).all()
    parity.assert_topk_matches_rule(S, idx, val, 5)
    rng = np.random.default_rng(2)
    opt = parity.oracle_options()
    for c in rng.choice(b.n_curves, 25, replace=False):
        fi = np.sort(rng.choice(len(b.freqs), 60, replace=False))
        t, y, dy = b.curve(int(c))
        gb = plan.debug_bins(int(c), 0, len(b.freqs)).cpu().numpy()[fi]
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[fi], b.n_bins, opt, gpu_bins=gb)
        parity.assert_s_close(S[c, fi], S_ref, S_abs, what=f"ztf1000 curve {c}")
    # whole periodograms of two curves, and their peaks
    for c in (int(np.argmax(b.lengths)), 7):
        ref = oracle.curve_periodogram(*b.curve(c), b.freqs, b.n_bins)
        parity.assert_topk_near_oracle(ref, idx[c], val[c], 5)
    plan.close()


def test_uneven_subset_full_grid():
    """Uneven lengths (50-2000 points) at the full 2e5-frequency grid, M = 40, fused top-5."""
    _say("uneven subset")
    b = synth.uneven_batch(300)
    plan = fpw.Plan.from_batch(b, n_bins=40, topk=5)
    _, idx_f, val_f = plan.eval(store_s=False)  # fused only: the periodogram never leaves the chip
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    np.testing.assert_array_equal(idx_f.cpu().numpy(), idx.cpu().numpy())
    np.testing.assert_array_equal(val_f.cpu().numpy(), val.cpu().numpy())
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), 5)
    rng = np.random.default_rng(4)
    opt = parity.oracle_options()
    for c in list(rng.choice(b.n_curves, 10, replace=False)) + [int(np.argmax(b.lengths)), int(np.argmin(b.lengths))]:
        c = int(c)
        fi = np.sort(rng.choice(len(b.freqs), 80, replace=False))
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()[fi]
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[fi], 40, opt, gpu_bins=gb)
        parity.assert_s_close(S[c, fi], S_ref, S_abs, what=f"uneven curve {c}")
    c = int(np.argmin(b.lengths))
    ref = oracle.curve_periodogram(*b.curve(c), b.freqs, 40)
    parity.assert_topk_near_oracle(ref, idx.cpu().numpy()[c], val.cpu().numpy()[c], 5)
    plan.close()


@pytest.mark.parametrize("phase", ["fp64", "df32"])
def test_stress_subset_full_grid(phase):
    """3000-point curves over 2000 d at the full 1e6-frequency grid to 200 /d, M = 50 (folds up to 4e5 cycles)."""
    _say(f"stress subset phase={phase}")
    b = synth.stress_batch(24)
    plan = fpw.Plan.from_batch(b, topk=5, phase=phase)
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), 5)
    rng = np.random.default_rng(5)
    opt = parity.oracle_options()
    nf = len(b.freqs)
    for c in range(0, b.n_curves, 3):
        # the highest frequencies carry the largest folds
        f0 = int(rng.integers(nf - 20000, nf - 64))
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, f0, f0 + 64).cpu().numpy()
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[f0:f0 + 64], 50, opt, gpu_bins=gb)
        parity.assert_s_close(S[c, f0:f0 + 64], S_ref, S_abs, what=f"stress curve {c}")
        fi = np.sort(rng.choice(nf, 40, replace=False))
        gb = np.stack([plan.debug_bins(c, int(k), int(k) + 1).cpu().numpy()[0] for k in fi])
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[fi], 50, opt, gpu_bins=gb)
        parity.assert_s_close(S[c, fi], S_ref, S_abs, what=f"stress curve {c} sampled")
    plan.close()


def test_fp32_naive_phase_flips_bins_at_large_folds():
    """The naive FP32 fold is a study mode: at 1e5+ cycles it must visibly disagree with the FP64 bins."""
    _say("naive fp32 flips")
    b = synth.stress_batch(2)
    plan = fpw.Plan.from_batch(b, phase="fp32")
    nf = len(b.freqs)
    gb = plan.debug_bins(0, nf - 64, nf).cpu().numpy()
    ob = oracle.curve_bins(b.curve(0)[0], b.freqs[nf - 64:], 50)
    assert (gb != ob).mean() > 0.05
    plan.close()


@pytest.mark.parametrize("M_max,derived,all_offsets,src", [(40, (20, 10), True, "auto"), (60, (20, 12, 4), False, "auto"),
                                                           (20, (10, 5), False, "scalar"), (12, (6,), True, "dpp")])
def test_multi_m_variants(M_max, derived, all_offsets, src):
    """Sec. 3.4: every (M, offset) variant combined from the M_max sums of one pass."""
    _say(f"multi-M {M_max} {derived} all_offsets={all_offsets} source={src}")
    freqs = np.linspace(0.05, 30.0, 477)
    b = synth.random_batch(50 + M_max, 10, 1, 300, freqs, M_max)
    plan = fpw.Plan.from_batch(b, topk=4, derived_bins=derived, all_offsets=all_offsets, chunk_freqs=128,
                               point_source=src)
    nv = plan.n_variants
    expect = 1 + sum((M_max // m) if all_offsets else 1 for m in derived)
    assert nv == expect
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S, idx, val = S.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
    opt = parity.oracle_options()
    for v in range(nv):
        M, o = plan.variant(v)
        parity.assert_topk_matches_rule(S[v], idx[v], val[v], 4)
        for c in range(0, b.n_curves, 2):
            t, y, dy = b.curve(c)
            gb = plan.debug_bins(c, 0, len(freqs)).cpu().numpy()
            S_ref, S_abs = parity.reference_for_variant(t, y, dy, freqs, M_max, M, o, opt, gb)
            parity.assert_s_close(S[v, c], S_ref, S_abs, what=f"variant {v} (M={M}, o={o}) curve {c}")
    # variant 0 is bit-identical to a plan without derived bin counts
    p0 = fpw.Plan.from_batch(b, topk=4, chunk_freqs=128, point_source=src)
    S0, i0, v0 = p0.eval()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S0.cpu().numpy(), S[0])
    np.testing.assert_array_equal(i0.cpu().numpy(), idx[0])
    plan.close()
    p0.close()


@pytest.mark.parametrize("phase", ["fp64", "fp64_listing"])
def test_phase_entropy_at_peaks(phase):
    """App. C: phase entropy of the observation times at each curve's top peaks, with its Hutcheson moments."""
    _say(f"phase entropy {phase}")
    b = synth.ztf_batch(40)
    plan = fpw.Plan.from_batch(b, topk=5, phase=phase)
    _, idx, _ = plan.eval(store_s=False)
    idx[3, 2] = -1  # a skipped slot
    H, E, V = plan.phase_entropy(idx)
    torch.cuda.synchronize()
    idx, H, E, V = idx.cpu().numpy(), H.cpu().numpy(), E.cpu().numpy(), V.cpu().numpy()
    assert np.isnan(H[3, 2]) and np.isnan(E[3, 2]) and np.isnan(V[3, 2])
    M = b.n_bins
    for c in range(b.n_curves):
        t, _, _ = b.curve(c)
        n = len(t)
        for r in range(5):
            k = int(idx[c, r])
            if k < 0:
                continue
            gb = plan.debug_bins(c, k, k + 1).cpu().numpy()[0]
            ob = oracle.phase_bins(t, b.freqs[k], M)
            near = oracle.edge_distance(t, b.freqs[k], M) < oracle.EPS_BIN
            assert not ((gb != ob) & ~near).any()
            cnt = np.bincount(gb, minlength=M)
            p = cnt[cnt > 0] / n
            H_ref = float(-np.sum(p * np.log(p)))
            if not near.any():
                assert H_ref == pytest.approx(oracle.phase_entropy(t, b.freqs[k], M), abs=1e-12)
            assert abs(H[c, r] - H_ref) <= 2e-6 * max(1.0, H_ref)
            assert E[c, r] == pytest.approx(oracle.entropy_expectation(M, n), rel=1e-6)
            assert V[c, r] == pytest.approx(oracle.entropy_variance(M, n), rel=1e-6)
    plan.close()
