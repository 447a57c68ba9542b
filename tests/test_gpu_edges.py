"""GPU: points exactly on a phase-bin edge take the bin floor() gives (App. A
phase-bin equation), in every fold and kernel.

Dyadic times and frequencies make tau * f exact in FP64, so the oracle's
listing-order bins are the exact floor(M frac(tau f)) everywhere and many
points sit exactly on an edge; the default (fused FP64) fold must then agree
with the oracle on every point, not only off the edges.
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


def _dyadic_batch(seed, n_curves, n_max, M, n_freq=300, shared=False):
    """Times on a 1/8-day grid over [0, 2000) d (every other curve on a 1/64 grid) and frequencies on
    a 1/16 grid: every tau * f * M is exact in FP64 and a few per cent of them are integers."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2502, 243, 3000 + seed])))
    freqs = np.sort(rng.choice(np.arange(1, 16 * 40), size=n_freq, replace=False)) / 16.0
    curves, labels = [], []
    t_common = np.sort(rng.choice(np.arange(0, 2000 * 8), size=n_max, replace=False)) / 8.0
    for c in range(n_curves):
        n = n_max if shared else int(rng.integers(1, n_max + 1))
        g = 8 if c % 2 == 0 else 64
        t = t_common if shared else np.sort(rng.choice(np.arange(0, 2000 * g), size=n, replace=False)) / g
        dy = 0.02 * np.exp(0.5 * rng.standard_normal(n))
        y = 0.1 * np.sin(2 * np.pi * 0.75 * t) + dy * rng.standard_normal(n)
        curves.append((t, y, dy))
        labels.append(dict(kind="sinusoid", f0=0.75))
    return synth._assemble(curves, freqs, M, labels, f"dyadic{seed}")


def _exact_edge_count(b, M):
    n = 0
    for c in range(b.n_curves):
        t = b.curve(c)[0]
        x = t[None, :] * b.freqs[:, None] * M  # exact: dyadic products of few bits
        n += int(np.sum(x == np.round(x)))
    return n


@pytest.mark.parametrize("M", [3, 7, 10, 12, 20, 50, 64, 255])
@pytest.mark.parametrize("phase", ["fp64", "fp64_listing"])
def test_exact_edges_general_kernel(M, phase):
    _say(f"exact edges general M={M} phase={phase}")
    b = _dyadic_batch(M, 6, 400, M)
    assert _exact_edge_count(b, M) > 100  # the grid really puts points on edges
    plan = fpw.Plan.from_batch(b, phase=phase, topk=3)
    S_gpu = plan.eval(topk=False)[0]
    torch.cuda.synchronize()
    S_gpu = S_gpu.cpu().numpy()
    opt = parity.oracle_options()
    for c in range(b.n_curves):
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()
        # the oracle's bins are exact here, so the GPU's must equal them on every point
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs, M, opt, gpu_bins=gb, exact_bins=True)
        parity.assert_s_close(S_gpu[c], S_ref, S_abs, what=f"curve {c}")
    plan.close()


@pytest.mark.parametrize("M", [10, 20, 50])
def test_exact_edges_shared_and_baseline_kernels(M):
    _say(f"exact edges shared/baseline M={M}")
    b = _dyadic_batch(100 + M, 8, 300, M, shared=True)
    opt = parity.oracle_options()
    t, Y, DY = b.as_shared()
    plan = fpw.Plan.shared(t, Y, DY, b.freqs, M, shared_kernel="matrix")
    assert plan.info().kernel == 1
    S_gpu = plan.eval(topk=False)[0].cpu().numpy()
    gb = plan.debug_bins(0, 0, len(b.freqs)).cpu().numpy()
    for c in range(b.n_curves):
        S_ref, S_abs, _ = parity.reference_for_curve(*b.curve(c), b.freqs, M, opt, gpu_bins=gb, exact_bins=True)
        parity.assert_s_close(S_gpu[c], S_ref, S_abs, what=f"shared curve {c}")
    plan.close()
    # baseline kernel with K = 0 terms is Eq. 1: K = 1 with a vanishing prior reduces to it
    if M <= 64:
        bm = fpw.Plan.from_batch(b, baseline_terms=1, baseline_scale=1e-6)
        S_bm = bm.eval(topk=False)[0].cpu().numpy()
        for c in range(b.n_curves):
            S_ref, S_abs, _ = parity.reference_for_curve(*b.curve(c), b.freqs, M, opt, gpu_bins=gb, exact_bins=True)
            parity.assert_s_close(S_bm[c], S_ref, S_abs, what=f"baseline curve {c}")
        bm.close()


@pytest.mark.parametrize("M", [10, 20, 50])
def test_first_observation_is_in_bin_zero_with_tref_first(M):
    """App. A takes t_ref as the first observation: its phase is 0 at every frequency, so its bin is 0."""
    _say(f"tref=first M={M}")
    freqs = np.linspace(0.05, 50.0, 2000)
    b = synth.random_batch(60 + M, 5, 2, 300, freqs, M)
    plan = fpw.Plan.from_batch(b, tref="first")
    for c in range(b.n_curves):
        t = b.curve(c)[0]
        first = int(np.argmin(t))
        gb = plan.debug_bins(c, 0, len(freqs)).cpu().numpy()
        assert np.all(gb[:, first] == 0), (c, np.unique(gb[:, first]))
    # the fold kernel bins through the same fold: S against the oracle, whose
    # exact-edge bins (here the first point's) are never excused
    S_gpu = plan.eval(topk=False)[0].cpu().numpy()
    for c in range(b.n_curves):
        gb = plan.debug_bins(c, 0, len(freqs)).cpu().numpy()
        S_ref, S_abs, _ = parity.reference_for_curve(*b.curve(c), freqs, M, parity.oracle_options(tref="first"),
                                                     gpu_bins=gb)
        parity.assert_s_close(S_gpu[c], S_ref, S_abs, what=f"curve {c}")
    plan.close()


def test_large_fold_range_uses_listing_order():
    """Where the fused fold's shift would blur edges by more than 1e-7 bin widths the plan folds in the listing order."""
    _say("large fold range")
    freqs = np.linspace(1000.0, 5000.0, 128)
    b = synth.random_batch(77, 3, 10, 100, freqs, 50, t_max=4000.0)
    plan = fpw.Plan.from_batch(b)
    assert plan.info().phase == fpw.PHASE["fp64_listing"]
    S_gpu = plan.eval(topk=False)[0].cpu().numpy()
    for c in range(b.n_curves):
        gb = plan.debug_bins(c, 0, len(freqs)).cpu().numpy()
        np.testing.assert_array_equal(gb, oracle.curve_bins(b.curve(c)[0], freqs, 50))
        S_ref, S_abs, _ = parity.reference_for_curve(*b.curve(c), freqs, 50, parity.oracle_options(), gpu_bins=gb,
                                                     exact_bins=True)
        parity.assert_s_close(S_gpu[c], S_ref, S_abs, what=f"curve {c}")
    plan.close()
