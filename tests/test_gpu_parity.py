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


def _check_plan_against_oracle(b, plan, opts, curves=None, exact_bins=False, freq_idx=None):
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
        guard.append(parity.assert_s_close(S_gpu[c, fi], S_ref, S_abs, what=f"curve {c}"))
    return float(np.mean(guard)), S_gpu


@pytest.mark.parametrize("phase", ["fp64", "fp64_listing", "df32"])
def test_config1_full(phase):
    _say(f"config1 phase={phase}")
    b = synth.config1()
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
    # (seed, M, phase, freqs_per_lane, waves_per_group, chunk)
    (1, 10, "fp64", 1, 1, 128),
    (2, 20, "fp64", 2, 4, 256),
    (3, 1, "fp64", 1, 2, 128),
    (4, 3, "fp64_listing", 1, 1, 192),
    (5, 50, "fp64_listing", 2, 1, 128),
    (6, 7, "df32", 1, 4, 64),
    (7, 40, "fp64", 1, 4, 0),
    (8, 2, "fp64", 2, 2, 128),
]


@pytest.mark.parametrize("seed,M,phase,fl,waves,chunk", RAGGED)
def test_ragged_batch(seed, M, phase, fl, waves, chunk):
    """Uneven curves (1..300 points), 477 frequencies (ragged last tile), several chunks per curve."""
    _say(f"ragged seed={seed} M={M} phase={phase} fl={fl} waves={waves} chunk={chunk}")
    freqs = np.linspace(0.05, 30.0, 477)
    b = synth.random_batch(seed, 12, 1, 300, freqs, M)
    plan = fpw.Plan.from_batch(b, phase=phase, topk=4, freqs_per_lane=fl, waves_per_group=waves, chunk_freqs=chunk)
    _check_plan_against_oracle(b, plan, {}, exact_bins=phase == "fp64_listing")
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
    plan = fpw.Plan.from_batch(b, topk=5)
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
    plan2 = fpw.Plan.from_batch(b, topk=5, use_graph=False)
    S2, i2, v2 = plan2.eval()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S2.cpu().numpy(), outs[0][0])
    np.testing.assert_array_equal(i2.cpu().numpy(), outs[0][1])
    plan.close()
    plan2.close()


def test_config2_full_size_sampled():
    """The benchmark's workload and launch configuration; sampled outputs against the oracle."""
    _say("config2 full size")
    b = synth.config2()
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
        parity.assert_s_close(S[c, fi], S_ref, S_abs, what=f"config2 curve {c}")
    # whole periodograms of two curves, and their peaks
    for c in (int(np.argmax(b.lengths)), 7):
        ref = oracle.curve_periodogram(*b.curve(c), b.freqs, b.n_bins)
        parity.assert_topk_near_oracle(ref, idx[c], val[c], 5)
    plan.close()
