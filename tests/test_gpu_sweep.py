"""Randomised GPU parity sweep: every plan kind on seeded random shapes, options and
frequency grids in arbitrary order (unsorted, with repeats), against the oracle."""
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


BINS = (1, 2, 3, 5, 8, 13, 20, 31, 47, 64)


def _draw(seed, max_freq=700):
    rng = np.random.default_rng(np.random.SeedSequence([2502, 243, 9000 + seed]))
    nf = int(rng.integers(1, max_freq))
    freqs = rng.uniform(0.01, 30.0, nf)
    if nf > 4:
        freqs[rng.integers(0, nf, nf // 5)] = freqs[0]  # repeats
    opts = {}
    if rng.random() < 0.3:
        opts["center"] = str(rng.choice(["mean", "none"]))
    if rng.random() < 0.3:
        opts["tref"] = "first"
    if rng.random() < 0.3:
        opts["inv_alpha2"] = float(10 ** rng.uniform(0, 4))
    phase = "fp64_listing" if rng.random() < 0.3 else "fp64"
    M = int(rng.choice(BINS))
    return rng, freqs, opts, phase, M


def _compare_general_like(b, plan, opts, exact):
    S = plan.eval(topk=False)[0].cpu().numpy()
    opt = parity.oracle_options(**opts)
    for c in range(b.n_curves):
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs, plan.n_bins, opt, gpu_bins=gb, exact_bins=exact)
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"curve {c}")
    return S


def _shape(rng, fused=True):
    """A random launch shape: waves per histogram and point source (defaults included), and where
    it allows the fused pass, that pass by default, forced or refused."""
    shape = dict(hist_share=int(rng.choice([0, 1, 2, 4])), point_source=str(rng.choice(["auto", "scalar", "dpp"])))
    if fused and shape["hist_share"] in (0, 4) and shape["point_source"] == "auto":
        shape["fuse_prepare"] = int(rng.choice([0, 1, -1]))
    return shape


@pytest.mark.parametrize("seed", range(16))
def test_general_random(seed):
    rng, freqs, opts, phase, M = _draw(seed)
    opts.update(_shape(rng))
    C = int(rng.integers(1, 20))
    _say(f"general sweep seed={seed} C={C} nf={len(freqs)} M={M} phase={phase} opts={opts}")
    b = synth.random_batch(500 + seed, C, 1, int(rng.integers(2, 400)), freqs, M)
    k = int(min(len(freqs), rng.integers(1, 9)))
    plan = fpw.Plan.from_batch(b, phase=phase, topk=k, **opts)
    S = _compare_general_like(b, plan, opts, phase == "fp64_listing")
    _, idx, val = plan.eval()
    torch.cuda.synchronize()
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), k)
    plan.close()


@pytest.mark.parametrize("seed", range(10, 18))
def test_shared_random(seed):
    rng, freqs, opts, phase, M = _draw(seed)
    C, N = int(rng.integers(1, 40)), int(rng.integers(1, 700))
    _say(f"shared sweep seed={seed} C={C} N={N} nf={len(freqs)} M={M} phase={phase} opts={opts}")
    b = synth.random_shared_batch(500 + seed, C, N, freqs, M)
    t, y, dy = b.as_shared()
    k = int(min(len(freqs), rng.integers(1, 9)))
    plan = fpw.Plan.shared(t, y, dy, b.freqs, M, phase=phase, topk=k, **opts)
    S = _compare_general_like(b, plan, opts, phase == "fp64_listing")
    _, idx, val = plan.eval()
    torch.cuda.synchronize()
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), k)
    plan.close()


@pytest.mark.parametrize("seed", range(20, 30))
def test_baseline_random(seed):
    rng, freqs, opts, phase, M = _draw(seed, max_freq=200)
    opts.update(_shape(rng, fused=False))
    K = int(rng.integers(1, 4))
    beta = float(10 ** rng.uniform(-2, 2))
    C = int(rng.integers(1, 8))
    _say(f"baseline sweep seed={seed} C={C} nf={len(freqs)} M={M} K={K} beta={beta:.3g} phase={phase} opts={opts}")
    b = synth.random_batch(500 + seed, C, 1, 150, freqs, M)
    plan = fpw.Plan.from_batch(b, phase=phase, baseline_terms=K, baseline_scale=beta, **opts)
    S = plan.eval(topk=False)[0].cpu().numpy()
    opt = parity.oracle_options(**opts)
    for c in range(b.n_curves):
        t, y, dy = b.curve(c)
        tau = oracle.time_offsets(t, opt)
        ob = oracle.phase_bins(tau[None, :], b.freqs[:, None], M)
        near = oracle.edge_distance(tau[None, :], b.freqs[:, None], M) < parity.EPS_BIN
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()
        assert not ((gb != ob) & ~near).any()
        bins = np.where(near, gb, ob)
        ref = oracle.bm_periodogram(t, y, dy, b.freqs, M, K, beta, opt, bins=bins)
        _, w, x = oracle.prepare_curve(t, y, dy, opt)
        S_abs = np.array([oracle.statistic(np.bincount(bb, weights=w, minlength=M),
                                           np.bincount(bb, weights=np.abs(w * x), minlength=M),
                                           opt.inv_alpha2, opt.stat_scale) for bb in bins])
        parity.assert_s_close(S[c], ref, S_abs, what=f"curve {c}")
    plan.close()
