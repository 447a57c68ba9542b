"""Shared helpers of the GPU parity tests (not collected by pytest).

Comparisons follow the tolerance protocol the design sets:
* bins: identical for every point farther than EPS_BIN bin widths from an
  edge (FP64 listing order: identical everywhere);
* S: the oracle is re-evaluated with the GPU's bins for the near-edge points
  only, then |S_gpu - S_ref| <= REL_TOL * S_ref + GUARD * S_abs, where
  S_abs = sum_m (sum_{j in m} |w_j x_j|)^2 / d_m bounds the cancellation a
  bin can suffer;
* peaks: the GPU's top-k over its own S equals the peak rule applied to that
  same S bit for bit, and agrees with the oracle's top-k up to near-ties.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import oracle
from oracle import OracleOptions

REL_TOL = 1e-5
GUARD = 1e-7
EPS_BIN = oracle.EPS_BIN
# Largest fraction of frequencies allowed to pass only through the
# cancellation guard (folds where every Y_m nearly cancels are rare).
MAX_GUARD_FRACTION = 1e-3


def on_exact_edge(tau, freqs, n_bins, near):
    """True where tau * f * M is exactly an integer in rational arithmetic.

    Only the points flagged ``near`` (FP64 edge distance below EPS_BIN) are
    examined; there floor() of the exact phase is the only correct bin, so a
    bin choice is excused only for near-edge points off the exact edge.
    """
    tau = np.asarray(tau, dtype=np.float64)
    freqs = np.asarray(freqs, dtype=np.float64)
    exact = np.zeros(near.shape, dtype=bool)
    # an exact edge has tau f = K / M with a dyadic K / M, which FP64 holds
    # exactly below 2^45 cycles, so phi * M is then an integer in FP64 too:
    # only those candidates need the rational check
    u = oracle.fold_phase(tau[None, :], freqs[:, None]) * float(n_bins)
    cand = near & (u == np.floor(u))
    for r, i in zip(*np.nonzero(cand)):
        x = Fraction(float(tau[i])) * Fraction(float(freqs[r])) * n_bins
        exact[r, i] = x.denominator == 1
    return exact


def oracle_options(**opts) -> OracleOptions:
    return OracleOptions(
        inv_alpha2=opts.get("inv_alpha2", 0.0),
        center=opts.get("center", "weighted"),
        tref=opts.get("tref", "zero"),
        t_ref=opts.get("t_ref", 0.0),
        stat_scale=opts.get("stat_scale", "eq1"),
    )


def reference_for_curve(t, y, dy, freqs, n_bins, opt, gpu_bins=None, exact_bins=False):
    """Oracle bins, S, S_abs and near-edge mask for one curve at the given frequencies.

    With ``gpu_bins`` ([n_freq, n]) the check of bins is done here and S is
    re-evaluated with the GPU's choice for near-edge points.
    """
    tau, w, x = oracle.prepare_curve(t, y, dy, opt)
    freqs = np.asarray(freqs, dtype=np.float64)
    ob = oracle.phase_bins(tau[None, :], freqs[:, None], n_bins)
    near = oracle.edge_distance(tau[None, :], freqs[:, None], n_bins) < EPS_BIN
    # a point exactly on an edge has one correct bin (floor): never excused
    if not exact_bins:
        near &= ~on_exact_edge(tau, freqs, n_bins, near)
    bins = ob
    if gpu_bins is not None:
        gb = np.asarray(gpu_bins, dtype=np.int64)
        mism = gb != ob
        if exact_bins:
            assert not mism.any(), f"{int(mism.sum())} bins differ (listing order must be exact)"
        else:
            bad = mism & ~near
            assert not bad.any(), f"{int(bad.sum())} off-edge or exact-edge bins differ"
        bins = np.where(near, gb, ob)
    S = np.empty(len(freqs))
    Sabs = np.empty(len(freqs))
    awx = np.abs(w * x)
    for r in range(len(freqs)):
        W, Y, _ = oracle.bin_sums(bins[r], w, x, n_bins)
        A = np.bincount(bins[r], weights=awx, minlength=n_bins)
        S[r] = oracle.statistic(W, Y, opt.inv_alpha2, opt.stat_scale)
        Sabs[r] = oracle.statistic(W, A, opt.inv_alpha2, opt.stat_scale)
    return S, Sabs, near


def assert_s_close(S_gpu, S_ref, S_abs, what="", max_guard=MAX_GUARD_FRACTION):
    """S within REL_TOL (or the cancellation guard); returns the fraction that needed the guard.

    That fraction is gated at ``max_guard`` of the values compared.
    """
    S_gpu = np.asarray(S_gpu, dtype=np.float64)
    err = np.abs(S_gpu - S_ref)
    lim = REL_TOL * np.abs(S_ref) + GUARD * S_abs
    bad = ~(err <= lim)
    if bad.any():
        i = int(np.argmax(np.where(bad, err / np.maximum(lim, 1e-300), 0)))
        raise AssertionError(
            f"{what}: {int(bad.sum())}/{bad.size} S values out of tolerance; worst at {i}: gpu {S_gpu.ravel()[i]!r} "
            f"ref {S_ref.ravel()[i]!r} abs {S_abs.ravel()[i]!r}"
        )
    # S that is zero in exact arithmetic (one point, one occupied bin with
    # the weighted mean removed) can only be checked through the guard; such
    # values are not counted as guard hits
    structural = np.abs(S_ref) <= 1e-9 * S_abs
    needs = (err > REL_TOL * np.abs(S_ref)) & ~structural
    guard = float(np.mean(needs)) if err.size else 0.0
    assert guard <= max_guard, f"{what}: {guard:.3g} of the S values needed the cancellation guard (> {max_guard})"
    return guard


def assert_topk_matches_rule(S_gpu_2d, idx, val, k):
    """The GPU's peaks equal the peak rule applied to the GPU's own S (bit for bit)."""
    S_gpu_2d = np.asarray(S_gpu_2d)
    for c in range(S_gpu_2d.shape[0]):
        ei, ev = oracle.topk(S_gpu_2d[c].astype(np.float32), k)
        np.testing.assert_array_equal(np.asarray(idx[c], dtype=np.int64), ei, err_msg=f"curve {c} indices")
        np.testing.assert_array_equal(np.asarray(val[c], dtype=np.float32), ev.astype(np.float32), err_msg=f"curve {c} values")


def assert_topk_near_oracle(S_ref, idx, val, k, rel=2e-5):
    """GPU peaks vs the oracle's: values agree in order; indices may differ only among near-ties."""
    oi, ov = oracle.topk(S_ref, k)
    gv = np.asarray(val, dtype=np.float64)
    gi = np.asarray(idx, dtype=np.int64)
    ok = np.isfinite(ov)
    assert np.array_equal(np.isfinite(gv), ok), (gi, oi)
    scale = np.maximum(np.abs(ov[ok]), 1e-30)
    assert np.all(np.abs(gv[ok] - ov[ok]) <= rel * scale + 1e-6 * np.max(np.abs(S_ref))), (gv, ov)
    for r in range(len(gi)):
        if gi[r] < 0 or gi[r] == oi[r]:
            continue
        # a different index must carry a value tied with the oracle's choice
        assert abs(S_ref[gi[r]] - ov[r]) <= rel * abs(ov[r]) + 1e-6 * np.max(np.abs(S_ref)), (r, gi, oi, gv, ov)


def reference_for_variant(t, y, dy, freqs, n_bins_max, n_bins, offset, opt, gpu_fine_bins):
    """Oracle S of an (M, offset) variant combined from M_max fine bins; near-edge fine bins follow the GPU."""
    tau, w, x = oracle.prepare_curve(t, y, dy, opt)
    freqs = np.asarray(freqs, dtype=np.float64)
    ob = oracle.phase_bins(tau[None, :], freqs[:, None], n_bins_max)
    near = oracle.edge_distance(tau[None, :], freqs[:, None], n_bins_max) < EPS_BIN
    gb = np.asarray(gpu_fine_bins, dtype=np.int64)
    assert not ((gb != ob) & ~near).any(), "off-edge fine bins differ"
    fine = np.where(near, gb, ob)
    S = np.empty(len(freqs))
    Sabs = np.empty(len(freqs))
    awx = np.abs(w * x)
    for r in range(len(freqs)):
        cb = oracle.combined_bins(fine[r], n_bins_max, n_bins, offset)
        W, Y, _ = oracle.bin_sums(cb, w, x, n_bins)
        A = np.bincount(cb, weights=awx, minlength=n_bins)
        S[r] = oracle.statistic(W, Y, opt.inv_alpha2, opt.stat_scale)
        Sabs[r] = oracle.statistic(W, A, opt.inv_alpha2, opt.stat_scale)
    return S, Sabs
