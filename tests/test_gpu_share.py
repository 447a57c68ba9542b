"""GPU parity of the batched kernel with histograms shared by 2 or 4 waves.

Each wave of a group folds a contiguous slice of a curve's observations into
one LDS histogram and reduces a range of its bins; the result must satisfy
the same protocol as private histograms (bins identical off edge, S within
1e-5 relative with the cancellation guard, peaks equal to the peak rule on
the GPU's own S), also for curves with fewer observations than waves, for
M = 1 and for the largest M; and since S is summed in one fixed order, it
must equal the private histograms' S bit for bit.
"""
import numpy as np
import pytest

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


def _ragged(seed, freqs, M):
    """Curves of 1, 2, 3 and 5 observations followed by curves of 30-400 (CSR arrays)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n in (1, 2, 3, 5):
        t = np.sort(rng.uniform(0.0, 1500.0, n))
        dy = rng.uniform(0.01, 0.05, n)
        parts.append((t, 0.05 * rng.standard_normal(n), dy))
    long = synth.random_batch(seed + 1, 10, 30, 400, freqs, M)
    for c in range(long.n_curves):
        parts.append(long.curve(c))
    lens = [len(p[0]) for p in parts]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    t, y, dy = (np.concatenate([p[i] for p in parts]) for i in range(3))
    return off, t, y, dy


def _check_against_oracle(plan, off, t, y, dy, freqs, M, opts, exact):
    S = plan.eval(topk=False)[0]
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    opt = parity.oracle_options(**opts)
    for c in range(len(off) - 1):
        a, e = int(off[c]), int(off[c + 1])
        gb = plan.debug_bins(c, 0, len(freqs)).cpu().numpy()
        S_ref, S_abs, _ = parity.reference_for_curve(t[a:e], y[a:e], dy[a:e], freqs, M, opt, gpu_bins=gb, exact_bins=exact)
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"curve {c} (n={e - a})")
    return S


CASES = [
    # (M, share, point source, phase, topk)
    (1, 2, "scalar", "fp64", 3),
    (3, 4, "dpp", "fp64_listing", 0),
    (7, 4, "scalar", "fp64", 5),
    (20, 2, "scalar", "fp64", 5),
    (33, 2, "dpp", "fp64", 5),
    (50, 2, "scalar", "fp64_listing", 5),
    (50, 4, "dpp", "fp64", 8),
    (64, 4, "scalar", "fp64", 16),
    (100, 4, "dpp", "fp64", 5),
    (255, 4, "dpp", "fp64", 5),
    (255, 2, "scalar", "fp64_listing", 2),
    (20, 2, "scalar", "df32", 5),
    (50, 4, "dpp", "df32", 3),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_shared_histogram_against_oracle(case):
    M, share, src, phase, k = case
    _say(f"shared histogram M={M} share={share} src={src} phase={phase} topk={k}")
    freqs = np.linspace(0.02, 9.0, 301)
    off, t, y, dy = _ragged(70 + M, freqs, M)
    plan = fpw.Plan(off, t, y, dy, freqs, M, phase=phase, topk=k, hist_share=share, point_source=src)
    info = plan.info()
    assert (info.hist_share, info.waves_per_group, info.kernel) == (share, share, 0)
    S = _check_against_oracle(plan, off, t, y, dy, freqs, M, {}, phase == "fp64_listing")
    if k:
        S2, idx, val = plan.eval()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(S2.cpu().numpy(), S)  # the fused peaks leave S unchanged
        parity.assert_topk_matches_rule(S, idx.cpu().numpy(), val.cpu().numpy(), k)
    plan.close()


@pytest.mark.parametrize("M,phase", [(1, "fp64"), (5, "fp64"), (20, "fp64"), (50, "fp64"), (130, "fp64"),
                                     (20, "df32"), (40, "fp32")])
def test_shared_equals_private_bit_for_bit(M, phase):
    """S is summed in one fixed order for every launch shape: private and shared histograms, either
    point source, one or two frequencies per lane give identical S and peaks (in every phase mode,
    the naive FP32 one included)."""
    _say(f"shared vs private M={M} phase={phase}")
    b = synth.random_batch(80 + M, 40, 1, 600, np.linspace(0.05, 20.0, 1500), M)
    ref = fpw.Plan.from_batch(b, hist_share=1, point_source="scalar", topk=5, phase=phase)
    S1, i1, v1 = (x.cpu().numpy() for x in ref.eval())
    shapes = [dict(hist_share=sh, point_source=src) for sh in (1, 2, 4) for src in ("scalar", "dpp")]
    if phase == "fp64":
        shapes += [dict(freqs_per_lane=2)]
    shapes += [dict(waves_per_group=4)] if 4 * (M + 1) * 512 <= 160 * 1024 else []
    for opts in shapes:
        p = fpw.Plan.from_batch(b, topk=5, phase=phase, **opts)
        S2, i2, v2 = (x.cpu().numpy() for x in p.eval())
        np.testing.assert_array_equal(S2, S1, err_msg=str(opts))
        np.testing.assert_array_equal(i2, i1, err_msg=str(opts))
        np.testing.assert_array_equal(v2, v1, err_msg=str(opts))
        p.close()
    ref.close()


@pytest.mark.parametrize("share", [2, 4])
def test_shared_histogram_multi_m(share):
    """Derived bin counts (Sec. 3.4) from a shared fine histogram: every variant against the oracle,
    and identical to private histograms."""
    _say(f"multi-M with shared histograms share={share}")
    freqs = np.linspace(0.05, 30.0, 333)
    b = synth.random_batch(95 + share, 10, 1, 300, freqs, 40)
    plan = fpw.Plan.from_batch(b, topk=4, derived_bins=(20, 10), all_offsets=True, hist_share=share)
    assert plan.info().hist_share == share and plan.n_variants == 7
    S, idx, val = (x.cpu().numpy() for x in plan.eval())
    opt = parity.oracle_options()
    for v in range(plan.n_variants):
        M, o = plan.variant(v)
        parity.assert_topk_matches_rule(S[v], idx[v], val[v], 4)
        for c in range(0, b.n_curves, 3):
            t, y, dy = b.curve(c)
            gb = plan.debug_bins(c, 0, len(freqs)).cpu().numpy()
            S_ref, S_abs = parity.reference_for_variant(t, y, dy, freqs, 40, M, o, opt, gb)
            parity.assert_s_close(S[v, c], S_ref, S_abs, what=f"variant {v} (M={M}, o={o}) curve {c}")
    priv = fpw.Plan.from_batch(b, topk=4, derived_bins=(20, 10), all_offsets=True, hist_share=1)
    Sp, ip, vp = (x.cpu().numpy() for x in priv.eval())
    np.testing.assert_array_equal(S, Sp)
    np.testing.assert_array_equal(idx, ip)
    single = fpw.Plan.from_batch(b, topk=4, hist_share=share)
    np.testing.assert_array_equal(single.eval()[0].cpu().numpy(), S[0])
    for p in (plan, priv, single):
        p.close()


def test_default_share_by_bin_count():
    _say("default share by M")
    b = synth.random_batch(90, 6, 20, 100, np.linspace(0.1, 5.0, 200), 10)
    one = dict(fuse_prepare=-1)  # a batch this small would otherwise run the fused pass
    # M: (waves per histogram, point source 1 scalar / 2 DPP)
    # (a plan this small takes four waves from M = 16: below 1.5e8 evaluations per CU)
    expect = {10: (1, 1), 15: (1, 1), 16: (4, 1), 31: (4, 1), 32: (4, 1), 127: (4, 1), 128: (4, 2), 255: (4, 2)}
    for M, (sh, src) in expect.items():
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, M, **one)
        assert (p.info().hist_share, p.info().point_source) == (sh, src), M
        p.close()
    p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 40, hist_share=1, **one)
    assert p.info().point_source == 2  # private histograms at large M: DPP source
    p.close()
    # private where no shared form is built or another group shape was asked for
    for opts in (dict(phase="df32", derived_bins=(20,)), dict(waves_per_group=2), dict(freqs_per_lane=2)):
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 40, **opts, **one)
        assert p.info().hist_share == 1, opts
        p.close()
    p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 20, derived_bins=(10,), **one)
    assert p.info().hist_share == 2  # the small-plan rule takes one variant only
    p.close()
    p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 40, derived_bins=(20,), **one)
    assert (p.info().hist_share, p.info().point_source) == (4, 1)  # derived bin counts share too, scalar source
    p.close()
    p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 40, derived_bins=(20, 10), all_offsets=True, **one)
    assert (p.info().hist_share, p.info().point_source) == (4, 2)  # more than four variants: DPP source
    p.close()
    for phase in ("df32", "fp32"):  # the study modes share with one variant
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, b.freqs, 40, phase=phase, **one)
        assert p.info().hist_share == 4, phase
        p.close()


def test_shared_histogram_repeated_passes_and_graph_replays():
    """Each pass restarts the queue (its prepare kernel zeroes the counter): back-to-back passes (graph replays
    and plain launches) agree."""
    _say("shared histogram repeated passes")
    b = synth.random_batch(91, 30, 50, 500, np.linspace(0.05, 15.0, 2000), 50)
    for use_graph in (True, False):
        p = fpw.Plan.from_batch(b, topk=5, hist_share=2, use_graph=use_graph)
        first = [x.cpu().numpy() for x in p.eval()]
        for _ in range(3):
            again = [x.cpu().numpy() for x in p.eval()]
            torch.cuda.synchronize()
            for u, v in zip(first, again):
                np.testing.assert_array_equal(u, v)
        p.close()


def test_stress_shape_with_shared_histograms_sampled():
    """A slice of the long-baseline stress batch (3000 points over 2000 d, M = 50) at its fold range."""
    _say("stress slice with shared histograms")
    b = synth.stress_batch(8)
    fi = np.sort(np.random.default_rng(3).choice(len(b.freqs), 400, replace=False))
    freqs = b.freqs[fi]
    p = fpw.Plan(b.offsets, b.t, b.y, b.dy, freqs, b.n_bins, topk=5, fuse_prepare=-1)
    assert p.info().hist_share == 4 and p.info().fuse_prepare == 0
    _check_against_oracle(p, b.offsets, b.t, b.y, b.dy, freqs, b.n_bins, {}, False)
    p.close()


def test_default_share_by_plan_size():
    """16 <= M < 32: four waves per histogram below 1.5e8 evaluations per CU, two from there."""
    _say("default share by plan size")
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    nf = 100000
    freqs = np.linspace(0.05, 50.0, nf)
    for evals_per_cu, want in ((1.4e8, 4), (1.6e8, 2)):
        C = int(np.ceil(evals_per_cu * n_cu / (nf * 100)))
        b = synth.random_batch(7, C, 100, 100, freqs[:10], 20)
        assert b.n_points == 100 * C
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, freqs, 20, topk=5)
        info = p.info()
        assert (info.fuse_prepare, info.hist_share) == (0, want), (C, n_cu)
        p.close()
