"""GPU parity of the baseline-marginalised statistic (App. A, general case).

The kernel's S is compared with the oracle's step-by-step form of App. A
(itself pinned against the dense definition): bins identical off edge, S
within 1e-5 relative with the cancellation guard, peaks equal to the peak
rule on the GPU's own S.
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


FREQS = np.linspace(0.05, 12.0, 477)


def _drift(t, amp):
    """A smooth quadratic-plus-sinusoidal trend over the time span (a slow baseline drift)."""
    u = (t - t.min()) / max(t.max() - t.min(), 1.0)
    return amp * (0.7 * u - 1.1 * u * u + 0.2 * np.sin(2.0 * np.pi * 0.4 * u))


def _with_drift(b, amp):
    y = b.y.copy()
    for c in range(b.n_curves):
        a, e = int(b.offsets[c]), int(b.offsets[c + 1])
        y[a:e] += _drift(b.t[a:e], amp)
    return y


def _reference(plan, b, y, K, beta, opts, c, freq_idx=None, exact_bins=False):
    a, e = int(b.offsets[c]), int(b.offsets[c + 1])
    t, yc, dy = b.t[a:e], y[a:e], b.dy[a:e]
    opt = parity.oracle_options(**opts)
    fi = np.arange(len(b.freqs)) if freq_idx is None else np.asarray(freq_idx)
    freqs = b.freqs[fi]
    tau = oracle.time_offsets(t, opt)
    ob = oracle.phase_bins(tau[None, :], freqs[:, None], plan.n_bins)
    near = oracle.edge_distance(tau[None, :], freqs[:, None], plan.n_bins) < parity.EPS_BIN
    gb = plan.debug_bins(c, 0, len(b.freqs)).cpu().numpy()[fi]
    if exact_bins:
        assert np.array_equal(gb, ob)
    else:
        assert not ((gb != ob) & ~near).any(), "off-edge bins differ"
    bins = np.where(near, gb, ob)
    S = oracle.bm_periodogram(t, yc, dy, freqs, plan.n_bins, K, beta, opt, bins=bins)
    # guard scale: the plain statistic's absolute form
    _, w, x = oracle.prepare_curve(t, yc, dy, opt)
    S_abs = np.array([oracle.statistic(np.bincount(bb, weights=w, minlength=plan.n_bins),
                                       np.bincount(bb, weights=np.abs(w * x), minlength=plan.n_bins),
                                       opt.inv_alpha2, opt.stat_scale) for bb in bins])
    return S, S_abs


CASES = [
    # (seed, M, K, beta, inv_alpha2, phase, drift amplitude)
    (1, 20, 3, 1.0, 0.0, "fp64", 0.3),
    (2, 10, 2, 0.05, 0.0, "fp64_listing", 0.1),
    (3, 7, 1, 1.0, 50.0, "fp64", 0.0),
    (4, 40, 3, 30.0, 0.0, "fp64", 1.0),
    (5, 64, 2, 1.0, 5.0, "fp64_listing", 0.2),
    (6, 1, 3, 1.0, 0.0, "fp64", 0.2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_baseline_kernel_against_oracle(case):
    seed, M, K, beta, ia2, phase, amp = case
    _say(f"baseline seed={seed} M={M} K={K} beta={beta} ia2={ia2} phase={phase} drift={amp}")
    b = synth.random_batch(seed + 40, 10, 1, 260, FREQS, M)
    y = _with_drift(b, amp)
    opts = dict(inv_alpha2=ia2)
    plan = fpw.Plan(b.offsets, b.t, y, b.dy, b.freqs, M, phase=phase, baseline_terms=K, baseline_scale=beta, **opts)
    assert plan.info().kernel == 2
    S = plan.eval(topk=False)[0]
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    guard = []
    for c in range(b.n_curves):
        ref, S_abs = _reference(plan, b, y, K, beta, opts, c, exact_bins=phase == "fp64_listing")
        guard.append(parity.assert_s_close(S[c], ref, S_abs, what=f"curve {c}"))
    print(f"  guard fraction {np.mean(guard):.2e}", flush=True)
    assert np.mean(guard) <= parity.MAX_GUARD_FRACTION
    plan.close()


@pytest.mark.parametrize("opts", [dict(center="mean"), dict(center="none"), dict(tref="first"),
                                  dict(stat_scale="listing_half")],
                         ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()))
def test_baseline_kernel_options(opts):
    _say(f"baseline options {opts}")
    b = synth.random_batch(61, 6, 20, 200, FREQS, 16)
    y = _with_drift(b, 0.2)
    plan = fpw.Plan(b.offsets, b.t, y, b.dy, b.freqs, 16, baseline_terms=3, **opts)
    S = plan.eval(topk=False)[0].cpu().numpy()
    for c in range(b.n_curves):
        ref, S_abs = _reference(plan, b, y, 3, 1.0, opts, c)
        parity.assert_s_close(S[c], ref, S_abs, what=f"curve {c}")
    plan.close()


def test_baseline_kernel_removes_drifts_and_peaks():
    """A strong drift leaves the marginalised periodogram unchanged (broad prior), and peaks
    follow the peak rule on the GPU's own S."""
    _say("baseline drift invariance and peaks")
    b = synth.random_batch(62, 8, 150, 300, FREQS, 20)
    p0 = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 20, baseline_terms=3, baseline_scale=1e3, topk=5)
    y1 = b.y.copy()
    for c in range(b.n_curves):
        a, e = int(b.offsets[c]), int(b.offsets[c + 1])
        u = 2 * (b.t[a:e] - b.t[a:e].min()) / (b.t[a:e].max() - b.t[a:e].min()) - 1
        y1[a:e] += 0.5 - 2.0 * u + 1.5 * (2 * u * u - 1)
    p1 = fpw.Plan(b.offsets, b.t, y1, b.dy, b.freqs, 20, baseline_terms=3, baseline_scale=1e3, topk=5)
    S0, i0, v0 = p0.eval()
    S1, i1, v1 = p1.eval()
    torch.cuda.synchronize()
    S0, S1 = S0.cpu().numpy(), S1.cpu().numpy()
    np.testing.assert_allclose(S1, S0, rtol=2e-4, atol=1e-4 * np.max(S0))
    parity.assert_topk_matches_rule(S0, i0.cpu().numpy(), v0.cpu().numpy(), 5)
    # the plain statistic is not protected from the drift
    pp = fpw.Plan(b.offsets, b.t, y1, b.dy, b.freqs, 20)
    Sp = pp.eval(topk=False)[0].cpu().numpy()
    assert np.median(Sp) > 10 * np.median(S0)
    for p in (p0, p1, pp):
        p.close()


def test_baseline_on_shared_plan_uses_general_path():
    _say("baseline on a shared-timestamp plan")
    b = synth.random_shared_batch(63, 9, 120, FREQS, 12)
    t, y, dy = b.as_shared()
    plan = fpw.Plan.shared(t, y, dy, b.freqs, 12, baseline_terms=2)
    assert plan.info().kernel == 2
    S = plan.eval(topk=False)[0].cpu().numpy()
    for c in (0, 4, 8):
        ref, S_abs = _reference(plan, b, b.y, 2, 1.0, {}, c)
        parity.assert_s_close(S[c], ref, S_abs, what=f"curve {c}")
    plan.close()


def test_ztf1000_with_baseline_sampled():
    """The benchmark data (1000 curves, 1e5 frequencies, M = 20) with K = 3, sampled against the oracle."""
    _say("baseline ztf1000 sampled")
    b = synth.ztf_batch()
    plan = fpw.Plan.from_batch(b, baseline_terms=3, topk=5)
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    rng = np.random.default_rng(9)
    fi = np.sort(rng.choice(len(b.freqs), 200, replace=False))
    for c in list(rng.choice(b.n_curves, 6, replace=False)) + [0]:
        ref, S_abs = _reference(plan, b, b.y, 3, 1.0, {}, int(c), freq_idx=fi)
        parity.assert_s_close(S[c, fi], ref, S_abs, what=f"curve {c}")
    parity.assert_topk_matches_rule(S[:50], idx.cpu().numpy()[:50], val.cpu().numpy()[:50], 5)
    plan.close()


@pytest.mark.parametrize("M,K,share,n_max,src", [(20, 3, 2, 260, "scalar"), (64, 3, 4, 260, "dpp"),
                                                 (1, 2, 2, 3, "scalar"), (7, 1, 4, 3, "dpp"), (40, 2, 2, 260, "dpp"),
                                                 (13, 3, 4, 5, "scalar"), (33, 1, 1, 200, "scalar"),
                                                 (5, 2, 1, 40, "scalar"), (64, 3, 1, 300, "dpp")],
                         ids=lambda v: str(v))
def test_baseline_kernel_shared_histograms(M, K, share, n_max, src):
    """Histograms shared by 2 or 4 waves (each folds a slice of the observations, the epilogue
    sums are split by bins) and either point source: same parity bar, also for curves with fewer
    observations than waves."""
    _say(f"baseline histograms M={M} K={K} share={share} n_max={n_max} source={src}")
    b = synth.random_batch(66 + M + n_max, 10, 1, n_max, FREQS, M)
    y = _with_drift(b, 0.3)
    plan = fpw.Plan(b.offsets, b.t, y, b.dy, b.freqs, M, baseline_terms=K, hist_share=share, topk=3, point_source=src)
    info = plan.info()
    assert (info.kernel, info.hist_share, info.waves_per_group) == (2, share, share)
    assert info.point_source == (1 if src == "scalar" else 2)
    S, idx, val = plan.eval()
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    for c in range(b.n_curves):
        ref, S_abs = _reference(plan, b, y, K, 1.0, {}, c)
        parity.assert_s_close(S[c], ref, S_abs, what=f"curve {c}")
    parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), 3)
    # private histograms on the same data: the FP64 epilogue sums differ only in order
    priv = fpw.Plan(b.offsets, b.t, y, b.dy, b.freqs, M, baseline_terms=K, hist_share=1,
                    point_source="dpp" if src == "scalar" else "scalar")
    Sp = priv.eval(topk=False)[0].cpu().numpy()
    np.testing.assert_allclose(S, Sp, rtol=1e-6, atol=1e-9 * float(np.abs(Sp).max()))
    for p in (plan, priv):
        p.close()


def test_baseline_default_share_by_histogram_size():
    _say("baseline default share")
    b = synth.random_batch(67, 4, 20, 80, FREQS, 10)
    # histogram bytes per wave: (8, 12, 16 for K = 1, 2, 3) x (M + 1) x 64; two waves from 8704, four from 12288
    for M, K, sh in [(15, 1, 1), (16, 1, 2), (20, 1, 2), (22, 1, 2), (23, 1, 4), (20, 2, 4), (20, 3, 4), (10, 2, 1),
                     (11, 2, 2), (15, 2, 4), (32, 1, 4), (7, 3, 1), (8, 3, 2), (11, 3, 4), (64, 2, 4)]:
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, M, baseline_terms=K)
        assert (p.info().hist_share, p.info().point_source) == (sh, 1), (M, K)
        p.close()
