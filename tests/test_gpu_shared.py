"""GPU parity of shared-timestamp plans (the batch of curves observed at common times).

The matrix-core kernel and the general kernel on the same plan are both
compared with the FP64 oracle under the usual protocol: bins identical off
edge (everywhere in listing order), S within 1e-5 relative with the
cancellation guard, peaks equal to the peak rule on the GPU's own S.
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


def _shared_plan(b, **opts):
    t, y, dy = b.as_shared()
    n_bins = opts.pop("n_bins", b.n_bins)
    return fpw.Plan.shared(t, y, dy, b.freqs, n_bins, **opts)


def _check(b, plan, opts, curves=None, freq_idx=None, exact_bins=False):
    S_gpu, _, _ = plan.eval(topk=False)
    torch.cuda.synchronize()
    S_gpu = S_gpu.cpu().numpy()
    opt = parity.oracle_options(**opts)
    fi = np.arange(len(b.freqs)) if freq_idx is None else np.asarray(freq_idx)
    # bins are a property of the common times: one fold check serves every curve
    gb = plan.debug_bins(0, 0, len(b.freqs)).cpu().numpy()[fi]
    guard = []
    for c in range(b.n_curves) if curves is None else curves:
        t, y, dy = b.curve(c)
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, b.freqs[fi], plan.n_bins, opt, gpu_bins=gb,
                                                     exact_bins=exact_bins)
        guard.append(parity.assert_s_close(S_gpu[c, fi], S_ref, S_abs, what=f"curve {c}"))
    return float(np.mean(guard)), S_gpu


FREQS = np.linspace(0.05, 12.0, 477)

# (seed, curves, points, M, phase): curve counts off the 16-curve blocks, point counts
# off the 32-point K-blocks, more than one 512-point LDS chunk, every bin count class
CASES = [
    (1, 37, 300, 20, "fp64"),
    (2, 16, 64, 10, "fp64_listing"),
    (3, 5, 1, 4, "fp64"),
    (4, 21, 1300, 50, "fp64"),
    (5, 3, 45, 1, "fp64"),
    (6, 40, 200, 7, "fp64_listing"),
    (7, 9, 531, 64, "fp64"),
    (8, 18, 95, 33, "fp64_listing"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_matrix_kernel_against_oracle(case):
    seed, C, N, M, phase = case
    _say(f"shared matrix seed={seed} C={C} N={N} M={M} phase={phase}")
    b = synth.random_shared_batch(seed, C, N, FREQS, M)
    plan = _shared_plan(b, phase=phase, shared_kernel="matrix")
    assert plan.info().kernel == 1
    g, _ = _check(b, plan, {}, exact_bins=phase == "fp64_listing")
    # every curve's fraction is gated at MAX_GUARD_FRACTION inside _check; with one bin S is
    # Y^2/W with Y = sum(w x) = 0, a structural zero that the gate does not count
    _say(f"  guard fraction {g:.2e}")
    assert g <= parity.MAX_GUARD_FRACTION
    plan.close()


def test_general_kernel_on_shared_plan_and_kernels_agree():
    _say("shared general vs matrix")
    b = synth.random_shared_batch(11, 24, 410, FREQS, 20)
    pg = _shared_plan(b, shared_kernel="general")
    pm = _shared_plan(b, shared_kernel="matrix")
    assert pg.info().kernel == 0 and pm.info().kernel == 1
    g, Sg = _check(b, pg, {})
    _say(f"  guard fraction {g:.2e}")
    assert g <= parity.MAX_GUARD_FRACTION
    Sm = pm.eval(topk=False)[0].cpu().numpy()
    rel = np.abs(Sm - Sg) / np.maximum(np.abs(Sg), 1e-30)
    assert np.median(rel) < 1e-6
    pg.close()
    pm.close()


@pytest.mark.parametrize(
    "opts",
    [dict(inv_alpha2=2000.0), dict(center="mean"), dict(center="none"), dict(tref="first"),
     dict(stat_scale="listing_half")],
    ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()),
)
def test_matrix_kernel_options(opts):
    _say(f"shared options {opts}")
    b = synth.random_shared_batch(12, 20, 180, FREQS, 16)
    plan = _shared_plan(b, shared_kernel="matrix", **opts)
    g, _ = _check(b, plan, opts)
    _say(f"  guard fraction {g:.2e}")
    assert g <= parity.MAX_GUARD_FRACTION
    plan.close()


def test_matrix_kernel_peaks_and_replays():
    _say("shared top-k and graph replays")
    b = synth.random_shared_batch(13, 33, 250, FREQS, 20)
    plan = _shared_plan(b, topk=5)
    assert plan.info().kernel == 1
    runs = [plan.eval() for _ in range(3)]
    torch.cuda.synchronize()
    S0 = runs[0][0].cpu().numpy()
    for S, idx, val in runs[1:]:
        np.testing.assert_array_equal(S.cpu().numpy(), S0)
        np.testing.assert_array_equal(idx.cpu().numpy(), runs[0][1].cpu().numpy())
    idx, val = runs[0][1].cpu().numpy(), runs[0][2].cpu().numpy()
    parity.assert_topk_matches_rule(S0, idx, val, 5)
    for c in range(0, b.n_curves, 8):
        ref = oracle.curve_periodogram(*b.curve(c), b.freqs, b.n_bins)
        parity.assert_topk_near_oracle(ref, idx[c], val[c], 5)
    # peaks without storing the periodogram (the plan's own buffer)
    _, idx2, val2 = plan.eval(store_s=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(idx2.cpu().numpy(), idx)
    np.testing.assert_array_equal(val2.cpu().numpy(), val)
    plan.close()


def test_matrix_kernel_matches_oracle_shared_form():
    """Against the oracle's shared-timestamp form (bins once per frequency, reused for every curve)."""
    _say("shared vs oracle shared form")
    b = synth.random_shared_batch(14, 12, 140, np.linspace(0.1, 6.0, 150), 12)
    t, y, dy = b.as_shared()
    plan = fpw.Plan.shared(t, y, dy, b.freqs, 12)
    S = plan.eval(topk=False)[0].cpu().numpy()
    ref = oracle.shared_periodogram(t, y, dy, b.freqs, 12)
    tau, w, x = oracle.prepare_curve(t, y[0], dy[0])
    near = (oracle.edge_distance(tau[None, :], b.freqs[:, None], 12) < parity.EPS_BIN).any(axis=1)
    for c in range(b.n_curves):
        _, w, x = oracle.prepare_curve(t, y[c], dy[c])
        S_abs = np.sum(np.abs(w * x)) ** 2 / np.sum(w)
        ok = np.abs(S[c] - ref[c]) <= parity.REL_TOL * ref[c] + parity.GUARD * S_abs
        assert np.all(ok | near), c
    plan.close()


def test_field_of_1000_curves_sampled():
    """The benchmark shape (1000 curves x 500 common epochs, 1e5 frequencies, M = 20), sampled."""
    _say("shared field 1000 x 500, 1e5 freqs, sampled")
    b = synth.shared_batch(1000, 500)
    plan = _shared_plan(b, topk=5)
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    fi = np.sort(rng.choice(len(b.freqs), 300, replace=False))
    curves = list(rng.choice(b.n_curves, 12, replace=False)) + [0, b.n_curves - 1]
    g, S_gpu = _check(b, plan, {}, curves=curves, freq_idx=fi)
    _say(f"  guard fraction {g:.2e}")
    assert g <= parity.MAX_GUARD_FRACTION
    Sn = S.cpu().numpy()
    np.testing.assert_array_equal(Sn[curves], S_gpu[curves])
    idx, val = idx.cpu().numpy(), val.cpu().numpy()
    parity.assert_topk_matches_rule(Sn[curves], idx[curves], val[curves], 5)
    plan.close()
