"""GPU: per-bin sum formats against the oracle on weights that span wide ranges.

Eq. 1 and Sec. 2 give every observation its own error, so one curve's
weights w = 1/dy^2 can span many decades.  The library keeps each curve's bin
sums in the narrow format (one packed 64-bit word) where its bounds allow
and in the wide format (two 64-bit words) otherwise; these tests put curves
on both sides of that line (one very precise point among ordinary ones,
errors log-uniform over five decades, two instruments whose precision
differs tenfold, ordinary ZTF-like errors) and check S at the 1e-5 bar,
bins, peaks and the routing itself, in general plans, in shared-timestamp
plans (which leave the 30-bit matrix-core kernel for the general one) and
with every curve forced wide.
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


def weight_batch(kind, seed, n_curves, n, freqs, M):
    """Curves of n uniform times over 1500 d with a sinusoid and noise; errors by `kind`:
    ("dominant", s): 0.02 everywhere but one point at s; "loguniform": 10^U(-5, 0);
    "twoclass": 0.01 in the first half of the time range, 0.1 in the second; "ztf": lognormal, median 0.02."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2502, 243, 4000 + seed])))
    curves, labels = [], []
    for c in range(n_curves):
        t = np.sort(rng.uniform(0.0, 1500.0, n))
        if isinstance(kind, tuple):
            dy = np.full(n, 0.02)
            dy[int(rng.integers(0, n))] = kind[1]
        elif kind == "loguniform":
            dy = 10.0 ** rng.uniform(-5.0, 0.0, n)
        elif kind == "twoclass":
            dy = np.where(t < 750.0, 0.01, 0.1)
        else:
            dy = np.clip(0.02 * np.exp(0.5 * rng.standard_normal(n)), 0.002, 0.5)
        f0 = float(np.exp(rng.uniform(np.log(0.1), np.log(20.0))))
        y = 0.05 * np.sin(2 * np.pi * f0 * t + rng.uniform(0, 2 * np.pi)) + dy * rng.standard_normal(n)
        if kind == "twoclass":
            y = y + np.where(t < 750.0, 0.0, 0.3)  # the noisy instrument also sits offset
        curves.append((t, y, dy))
        labels.append(dict(kind="sinusoid", f0=f0))
    return synth._assemble(curves, np.asarray(freqs, dtype=np.float64), M, labels, f"weights-{kind}")


def _check(b, plan, opts=None, fi=None):
    opts = opts or {}
    S_gpu = plan.eval(topk=False)[0]
    torch.cuda.synchronize()
    S_gpu = S_gpu.cpu().numpy()
    opt = parity.oracle_options(**opts)
    fi = np.arange(len(b.freqs)) if fi is None else fi
    guard = []
    for c in range(b.n_curves):
        t, y, dy = b.curve(c)
        gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()[fi]
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[fi], plan.n_bins, opt, gpu_bins=gb)
        guard.append(parity.assert_s_close(S_gpu[c, fi], S_ref, S_abs, what=f"curve {c}"))
    _say(f"  guard fraction {np.mean(guard):.2e}")
    return S_gpu


FREQS = np.linspace(0.05, 30.0, 1500)


@pytest.mark.parametrize("sigma,want_wide", [(1e-4, False), (1e-5, True), (1e-6, True)])
@pytest.mark.parametrize("M", [10, 20, 50])
def test_one_dominant_point(sigma, want_wide, M):
    """One point far more precise than the rest holds almost all of sum(w): the narrow unit
    sum(w)/2^32 is then coarse for every other point."""
    _say(f"dominant sigma={sigma} M={M}")
    b = weight_batch(("dominant", sigma), int(-np.log10(sigma)) * 100 + M, 6, 1000, FREQS, M)
    plan = fpw.Plan.from_batch(b, topk=5)
    assert plan.info().n_wide_curves == (b.n_curves if want_wide else 0)
    S = _check(b, plan)
    _, idx, val = plan.eval()
    torch.cuda.synchronize()
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), 5)
    plan.close()


@pytest.mark.parametrize("M", [4, 20, 64, 156])
def test_log_uniform_errors(M):
    """Errors log-uniform over 1e-5..1: weights over ten decades; every curve takes the wide format."""
    _say(f"log-uniform M={M}")
    b = weight_batch("loguniform", M, 5, 700, FREQS, M)
    plan = fpw.Plan.from_batch(b, topk=3)
    assert plan.info().n_wide_curves == b.n_curves
    _check(b, plan)
    plan.close()


def test_two_instruments_round_alike():
    """Two error classes (0.01 and 0.1, one per half of the baseline): the 0.1 points share one weight,
    so their rounding errors are equal and a bin of them alone keeps that error; the plan routes the
    curves wide (e_dup), and S is within the bar at every frequency, the low ones where the halves
    fill separate bins included."""
    _say("two classes")
    freqs = np.concatenate([np.linspace(2e-5, 2e-3, 200), FREQS])
    b = weight_batch("twoclass", 7, 4, 3000, freqs, 50)
    plan = fpw.Plan.from_batch(b)
    assert plan.info().n_wide_curves == b.n_curves
    _check(b, plan)
    plan.close()


@pytest.mark.parametrize("M", [1, 2, 7, 20, 50, 64, 100, 156])
@pytest.mark.parametrize("phase", ["fp64", "fp64_listing"])
def test_forced_wide_on_ordinary_data(M, phase):
    """Every curve wide on request: the same S as the oracle (and as the narrow format) on ZTF-like
    errors, short and long curves, each histogram sharing (private below 8 bins, two waves below 16,
    four beyond), peaks by the rule."""
    _say(f"forced wide M={M} phase={phase}")
    freqs = np.linspace(0.05, 20.0, 611)
    b = synth.random_batch(500 + M, 9, 1, 400, freqs, M)
    plan = fpw.Plan.from_batch(b, phase=phase, topk=4, sum_format="wide")
    assert plan.info().n_wide_curves == b.n_curves
    S = _check(b, plan, fi=np.arange(0, len(freqs), 3))
    _, idx, val = plan.eval()
    torch.cuda.synchronize()
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), 4)
    narrow = fpw.Plan.from_batch(b, phase=phase, topk=4)
    assert narrow.info().n_wide_curves == 0
    Sn = narrow.eval(topk=False)[0].cpu().numpy()
    # the two formats agree where S is not a cancellation residue
    big = S > np.maximum(1e-3 * np.max(S, axis=1, keepdims=True), 1e-6)
    if big.any():
        assert np.quantile(np.abs(Sn - S)[big] / S[big], 0.99) < 2e-6
    plan.close()
    narrow.close()


def test_mixed_batch_both_kernels_one_pass_and_graph_replays():
    """Narrow and wide curves in one plan: one pass runs both fold kernels, the per-curve peak merge
    takes both, replays of the captured pass are bit-identical."""
    _say("mixed batch")
    kinds = [("dominant", 1e-6), "ztf", "loguniform", "ztf", ("dominant", 1e-4), "twoclass"]
    parts = [weight_batch(k, 40 + i, 2, 500, FREQS, 20) for i, k in enumerate(kinds)]
    offs = [0]
    for p in parts:
        offs.extend((offs[-1] + np.asarray(p.offsets[1:])).tolist())
    b = synth.Batch(offsets=np.asarray(offs, dtype=np.int64), t=np.concatenate([p.t for p in parts]),
                    y=np.concatenate([p.y for p in parts]), dy=np.concatenate([p.dy for p in parts]),
                    freqs=FREQS, n_bins=20, labels=sum([p.labels for p in parts], []), name="mixed")
    plan = fpw.Plan.from_batch(b, topk=5)
    info = plan.info()
    # wide: the two 1e-6-dominated and the two log-uniform curves; the 1e-4-dominated ones and the
    # 500-point two-instrument ones stay within the narrow bounds (e_dup 4.7e-6 and 3.0e-6)
    assert info.n_wide_curves == 4 and info.fuse_prepare == 0
    S = _check(b, plan)
    outs = []
    for _ in range(3):
        Sg, idx, val = plan.eval()
        torch.cuda.synchronize()
        outs.append((Sg.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()))
        torch.cuda.synchronize()
    for o in outs[1:]:
        for a, c in zip(outs[0], o):
            np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(outs[0][0], S)
    parity.assert_topk_matches_rule(S, outs[0][1], outs[0][2], 5)
    for c in range(b.n_curves):
        ref = oracle.curve_periodogram(*b.curve(c), FREQS, 20)
        parity.assert_topk_near_oracle(ref, outs[0][1][c], outs[0][2][c], 5)
    plan.close()


def test_shared_plan_leaves_the_matrix_kernel_for_wide_weights():
    """A shared-timestamp batch with one curve beyond the 30-bit sums of the matrix-core kernel: the
    automatic choice takes the general kernel (that curve wide), the explicit one is refused."""
    _say("shared plan with wide weights")
    b = synth.random_shared_batch(31, 12, 400, FREQS, 20)
    t, Y, DY = b.as_shared()
    DY = DY.copy()
    DY[5, 123] = 1e-6
    plan = fpw.Plan.shared(t, Y, DY, FREQS, 20)
    info = plan.info()
    assert info.kernel == 0 and info.n_wide_curves == 1
    S = plan.eval(topk=False)[0].cpu().numpy()
    opt = parity.oracle_options()
    gb = plan.debug_bins(0, 0, len(FREQS)).cpu().numpy()
    for c in range(12):
        S_ref, S_abs, _ = parity.reference_for_curve(t, Y[c], DY[c], FREQS, 20, opt, gpu_bins=gb)
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"curve {c}")
    plan.close()
    with pytest.raises(fpw.FpwError) as e:
        fpw.Plan.shared(t, Y, DY, FREQS, 20, shared_kernel="matrix")
    assert e.value.status == fpw.EUNSUPPORTED
