"""GPU parity of the fused pass (small plans: the fold kernel prepares its curves itself,
then one workgroup per curve merges the peaks).

Its curve constants and records come from the prepare kernel's own functions
and its S from the same fixed summation order, so S and peaks must equal the
three-kernel pass bit for bit, in every phase mode, for ragged curves (1-5
observations), M = 1 .. 255, k = 0 .. 16, forced chunkings and the centring /
reference-time / prior options, and stay the same over repeated passes.
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


def _ragged(seed, freqs, M, n_long=6):
    """Curves of 1, 2, 3 and 5 observations, then curves of 30-400 (CSR arrays)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n in (1, 2, 3, 5):
        t = np.sort(rng.uniform(0.0, 1500.0, n))
        parts.append((t, 0.05 * rng.standard_normal(n), rng.uniform(0.01, 0.05, n)))
    long = synth.random_batch(seed + 1, n_long, 30, 400, freqs, M)
    for c in range(long.n_curves):
        parts.append(long.curve(c))
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])]).astype(np.int64)
    t, y, dy = (np.concatenate([p[i] for p in parts]) for i in range(3))
    return off, t, y, dy


def _both(off, t, y, dy, freqs, M, **opts):
    """(fused plan, three-kernel plan) of the same batch and options."""
    one = fpw.Plan(off, t, y, dy, freqs, M, fuse_prepare=1, **opts)
    three = fpw.Plan(off, t, y, dy, freqs, M, fuse_prepare=-1, **opts)
    assert one.info().fuse_prepare == 1 and three.info().fuse_prepare == 0
    return one, three


def _same(p, q, topk):
    a = [x.cpu().numpy() if x is not None else None for x in p.eval(topk=topk)]
    b = [x.cpu().numpy() if x is not None else None for x in q.eval(topk=topk)]
    for u, v in zip(a, b):
        if u is None:
            assert v is None
        else:
            np.testing.assert_array_equal(u, v)
    return a


def test_single_curve_default_is_fused():
    _say("single curve, default plan")
    b = synth.single_curve()
    p = fpw.Plan.from_batch(b, topk=1)
    info = p.info()
    assert (info.fuse_prepare, info.hist_share, info.waves_per_group, info.chunk_freqs) == (1, 4, 4, 64)
    assert info.point_source == 3
    assert info.grid_groups == info.work_items == (len(b.freqs) + 63) // 64
    q = fpw.Plan.from_batch(b, topk=1, fuse_prepare=-1)
    S, idx, val = _same(p, q, True)
    # against the oracle, on the GPU's own bins at edges
    gb = p.debug_bins(0, 0, len(b.freqs)).cpu().numpy()
    S_ref, S_abs, _ = parity.reference_for_curve(*b.curve(0), b.freqs, b.n_bins, parity.oracle_options(), gpu_bins=gb)
    parity.assert_s_close(S[0], S_ref, S_abs, what="single curve")
    assert abs(b.freqs[idx[0, 0]] - 1 / 0.37) <= 2 * (b.freqs[1] - b.freqs[0])
    parity.assert_topk_matches_rule(S, idx, val, 1)
    ref = oracle.curve_periodogram(*b.curve(0), b.freqs, b.n_bins)
    parity.assert_topk_near_oracle(ref, idx[0], val[0], 1)
    p.close()
    q.close()


CASES = [
    # (M, phase, topk)
    (1, "fp64", 3),
    (7, "fp64", 0),
    (10, "fp64", 1),
    (20, "fp64_listing", 5),
    (20, "df32", 5),
    (20, "fp32", 4),
    (50, "fp64", 16),
    (64, "fp64_listing", 8),
    (255, "fp64", 9),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_fused_equals_three_kernels(case):
    M, phase, k = case
    _say(f"fused vs three kernels M={M} phase={phase} topk={k}")
    freqs = np.linspace(0.02, 9.0, 477)  # 7 full sub-tiles and a ragged one
    off, t, y, dy = _ragged(300 + M, freqs, M)
    one, three = _both(off, t, y, dy, freqs, M, phase=phase, topk=k)
    S, idx, val = _same(one, three, k > 0)
    if k:
        parity.assert_topk_matches_rule(S, idx, val, k)
    # S against the oracle on every curve, bins taken from the GPU at edges (not for the naive
    # FP32 fold, whose wrong bins at large tau f are what the precision study measures)
    opt = parity.oracle_options()
    for c in range(len(off) - 1 if phase != "fp32" else 0):
        a, e = int(off[c]), int(off[c + 1])
        gb = one.debug_bins(c, 0, len(freqs)).cpu().numpy()
        S_ref, S_abs, _ = parity.reference_for_curve(t[a:e], y[a:e], dy[a:e], freqs, M, opt, gpu_bins=gb,
                                                     exact_bins=phase == "fp64_listing")
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"curve {c} (n={e - a})")
    one.close()
    three.close()


@pytest.mark.parametrize("nf,M", [(1, 5), (2, 5), (65, 255), (130, 64)])
def test_fused_edge_cases(nf, M):
    """One and two frequencies, curves of one point, M at its maximum: fused pass against the oracle
    and the three-kernel pass."""
    _say(f"fused edge case nf={nf} M={M}")
    freqs = np.linspace(0.3, 5.0, nf)
    b = synth.random_batch(30 + nf, 4, 1, 40, freqs, M)
    k = min(3, nf)
    one, three = _both(b.offsets, b.t, b.y, b.dy, freqs, M, topk=k)
    S, idx, val = _same(one, three, True)
    parity.assert_topk_matches_rule(S, idx, val, k)
    opt = parity.oracle_options()
    for c in range(b.n_curves):
        t, y, dy = b.curve(c)
        gb = one.debug_bins(c, 0, nf).cpu().numpy()
        S_ref, S_abs, _ = parity.reference_for_curve(t, y, dy, freqs, M, opt, gpu_bins=gb)
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"curve {c}")
    one.close()
    three.close()


@pytest.mark.parametrize(
    "opts",
    [
        dict(center="mean"),
        dict(center="none", tref="first"),
        dict(tref="given", t_ref=-3.25),
        dict(stat_scale="listing_half", inv_alpha2=2.5),
    ],
    ids=lambda o: "-".join(f"{k}={v}" for k, v in o.items()),
)
def test_fused_options(opts):
    _say(f"fused options {opts}")
    freqs = np.linspace(0.05, 12.0, 700)
    off, t, y, dy = _ragged(41, freqs, 12)
    one, three = _both(off, t, y, dy, freqs, 12, topk=4, **opts)
    _same(one, three, True)
    one.close()
    three.close()


@pytest.mark.parametrize("chunk", [0, 100, 1000])
def test_forced_fused_on_a_larger_plan(chunk):
    """Forced on a plan above the default size (longer items, or the given chunk)."""
    _say(f"forced fused chunk={chunk}")
    freqs = np.linspace(0.05, 20.0, 3001)
    b = synth.random_batch(77, 400, 20, 300, freqs, 20)
    one, three = _both(b.offsets, b.t, b.y, b.dy, freqs, 20, topk=5, chunk_freqs=chunk)
    if chunk:
        assert one.info().chunk_freqs == ((chunk + 63) // 64) * 64
    else:
        assert one.info().chunk_freqs > 64  # the per-CU budget lengthens the items
    _same(one, three, True)
    one.close()
    three.close()


def test_fused_repeated_passes():
    """Repeated passes (use_graph on or off: the fused pass is launched directly either way) and
    S-only passes in between give the same S and peaks."""
    _say("fused repeated passes")
    freqs = np.linspace(0.05, 15.0, 1000)
    off, t, y, dy = _ragged(55, freqs, 16)
    ref = None
    for use_graph in (True, False):
        p = fpw.Plan(off, t, y, dy, freqs, 16, topk=6, use_graph=use_graph)
        assert p.info().fuse_prepare == 1
        for r in range(4):
            if r == 2:
                s_only = p.eval(topk=False)[0].cpu().numpy()
                np.testing.assert_array_equal(s_only, ref[0])
            out = [x.cpu().numpy() for x in p.eval()]
            torch.cuda.synchronize()
            if ref is None:
                ref = out
            for u, v in zip(out, ref):
                np.testing.assert_array_equal(u, v)
        p.close()


def test_default_size_rule():
    """Fused up to 4 items of 64 frequencies per CU, three kernels above, or when a shape is asked for."""
    _say("fused default size rule")
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    budget = 4 * n_cu
    n_curves = 16
    per_curve = budget // n_curves
    b = synth.random_batch(12, n_curves, 20, 100, np.linspace(0.1, 5.0, 10), 10)
    at = np.linspace(0.1, 5.0, per_curve * 64)
    above = np.linspace(0.1, 5.0, per_curve * 64 + 1)
    for freqs, expect in ((at, 1), (above, 0)):
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, freqs, 10, topk=2)
        assert p.info().fuse_prepare == expect, (len(freqs), n_cu)
        p.close()
    for opts in (dict(hist_share=1), dict(point_source="scalar"), dict(chunk_freqs=128), dict(derived_bins=(5,)),
                 dict(baseline_terms=1), dict(autotune=True)):
        p = fpw.Plan(b.offsets, b.t, b.y, b.dy, at, 10, topk=2, **opts)
        assert p.info().fuse_prepare == 0, opts
        p.close()


def test_fused_profile_timings():
    """prepare runs inside the fold kernel: its own time reads ~0, the merge is timed."""
    _say("fused timings")
    b = synth.single_curve()
    p = fpw.Plan.from_batch(b, topk=1, profile=True)
    p.eval()
    t = p.timings()
    assert t[1] > 0 and t[2] > 0 and t[0] < t[1]
    p.eval(topk=False)
    assert p.timings()[2] == 0.0
    p.close()
