"""Plain FP64 CPU oracle for the Fast Periodicity Weighting (FPW) periodogram.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this module.  The GPU path
shares no code with it and never calls it.

It evaluates the paper's definitions literally, one trial frequency at a
time (vectorised over a block of frequencies with NumPy, which changes no
operation and no summation order):

* Fold and bin rule (App. A, the phase-bin index equation; Sec. 4 text and
  the App. D listing): the phase of an observation at offset tau = t - t_ref
  for trial frequency f is the fractional part of tau * f, and its bin is
  the integer part of M times that phase, zero-indexed.  The products are
  rounded in FP64 in the listing's order: p = fl(tau * f), phi = p - floor(p)
  (exact for p >= 0), b = floor(fl(phi * M)).
* Inverse variance (App. D listing, ``runFPW``): w = 1 / (dy * dy).
* Mean subtraction (Eq. 1 definitions; Sec. 3.5): x is the mean-subtracted
  flux.  Default: the inverse-variance-weighted mean (see ``center``).
* Per-bin sums (App. A, sparse form; App. D ``deltaChi2``):
  W_m = sum of w over points in bin m, Y_m = sum of w * x over those points.
* Statistic (Eq. 1): S = sum_m Y_m^2 / (W_m + 1/alpha^2).  Empty bins
  contribute zero.
* Peaks (Sec. 3.5 post-processing): local maxima of S over the frequency
  index, the k largest per curve.

Readings where the paper is silent or inconsistent (each is listed with its
reason in the design notes): the statistic carries no factor 1/2 by default
(Eq. 1 and App. A; the listing's ``1/(2 W)`` is available as
``stat_scale="listing_half"``); 1/alpha^2 defaults to 0 (App. A closing
paragraph: small and neglected); empty bins give 0 rather than the listing's
0 * inf; t_ref defaults to 0 (listing) and tau must be >= 0 so that the
listing's truncation and App. A's "mod 1" coincide; the weighted mean is the
default centring.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "OracleOptions",
    "validate",
    "weights",
    "center",
    "time_offsets",
    "fold_phase",
    "phase_bins",
    "edge_distance",
    "bin_sums",
    "statistic",
    "prepare_curve",
    "curve_periodogram",
    "shared_periodogram",
    "chebyshev_basis",
    "bm_statistic_dense",
    "bm_periodogram",
    "curve_bins",
    "periodogram",
    "peak_mask",
    "topk",
    "batch_topk",
    "combined_bins",
    "variant_periodogram",
    "phase_entropy",
    "entropy_expectation",
    "entropy_variance",
]

# Bins of a point closer than this many bin widths to a bin edge may
# legitimately differ between two correct FP64 evaluation orders.
EPS_BIN = 1e-6


class OracleOptions:
    """Options mirroring the library's plan options (same names and defaults)."""

    def __init__(
        self,
        inv_alpha2: float = 0.0,
        center: str = "weighted",
        tref: str = "zero",
        t_ref: float = 0.0,
        stat_scale: str = "eq1",
    ):
        if center not in ("weighted", "mean", "none"):
            raise ValueError(center)
        if tref not in ("zero", "first", "given"):
            raise ValueError(tref)
        if stat_scale not in ("eq1", "listing_half"):
            raise ValueError(stat_scale)
        self.inv_alpha2 = float(inv_alpha2)
        self.center = center
        self.tref = tref
        self.t_ref = float(t_ref)
        self.stat_scale = stat_scale


def validate(offsets, t, y, dy, freqs, n_bins, opt: OracleOptions | None = None):
    """Reject inputs outside the problem statement (raise ValueError)."""
    opt = opt or OracleOptions()
    offsets = np.asarray(offsets)
    if offsets.ndim != 1 or len(offsets) < 2:
        raise ValueError("need at least one curve")
    if offsets[0] != 0 or np.any(np.diff(offsets) < 1):
        raise ValueError("offsets must start at 0 and every curve needs >= 1 point")
    n = int(offsets[-1])
    for name, a in (("t", t), ("y", y), ("dy", dy)):
        a = np.asarray(a, dtype=np.float64)
        if a.shape != (n,):
            raise ValueError(f"{name} must have offsets[-1] elements")
        if not np.all(np.isfinite(a)):
            raise ValueError(f"{name} must be finite")
    if not np.all(np.asarray(dy) > 0):
        raise ValueError("dy must be > 0")
    freqs = np.asarray(freqs, dtype=np.float64)
    if freqs.ndim != 1 or len(freqs) < 1:
        raise ValueError("need at least one frequency")
    if not (np.all(np.isfinite(freqs)) and np.all(freqs > 0)):
        raise ValueError("frequencies must be finite and > 0")
    if int(n_bins) < 1:
        raise ValueError("n_bins must be >= 1")
    if not (math.isfinite(opt.inv_alpha2) and opt.inv_alpha2 >= 0):
        raise ValueError("inv_alpha2 must be finite and >= 0")
    for c in range(len(offsets) - 1):
        tc = np.asarray(t[offsets[c] : offsets[c + 1]], dtype=np.float64)
        tau = time_offsets(tc, opt)
        if np.any(tau < 0):
            raise ValueError("t - t_ref must be >= 0")


def weights(dy: np.ndarray) -> np.ndarray:
    """Inverse variance, formed as the listing does: 1 / (dy * dy)."""
    dy = np.asarray(dy, dtype=np.float64)
    return 1.0 / (dy * dy)


def center(y: np.ndarray, w: np.ndarray, mode: str = "weighted") -> np.ndarray:
    """Mean-subtracted flux x (Eq. 1 definitions, Sec. 3.5).

    ``weighted``: subtract sum(w y) / sum(w), the maximum-likelihood constant,
    which makes sum(w x) = 0 so that S is chi-square with M-1 degrees of
    freedom on pure noise.  ``mean``: subtract the plain average.
    ``none``: x = y.  Sums use exactly rounded ``math.fsum``.
    """
    y = np.asarray(y, dtype=np.float64)
    if mode == "none":
        return y.copy()
    if mode == "mean":
        mu = math.fsum(y) / len(y)
    elif mode == "weighted":
        mu = math.fsum(w * y) / math.fsum(w)
    else:
        raise ValueError(mode)
    return y - mu


def time_offsets(t: np.ndarray, opt: OracleOptions) -> np.ndarray:
    """tau = t - t_ref in FP64 (App. A): t_ref = 0, the first (minimum) time, or given."""
    t = np.asarray(t, dtype=np.float64)
    if opt.tref == "zero":
        return t.copy()
    if opt.tref == "first":
        return t - np.min(t)
    return t - opt.t_ref


def fold_phase(tau: np.ndarray, f) -> np.ndarray:
    """Phase in [0, 1): p = fl(tau * f), phi = p - floor(p) (App. A "mod 1")."""
    p = np.multiply(tau, f)
    return p - np.floor(p)


def phase_bins(tau: np.ndarray, f, n_bins: int) -> np.ndarray:
    """Zero-indexed bin floor(fl(phi * M)) (App. A bin-index equation).

    The final clamp to M-1 never changes a result for phi < 1 in
    round-to-nearest; it is kept as a guard.
    """
    phi = fold_phase(tau, f)
    b = np.floor(phi * float(n_bins)).astype(np.int64)
    return np.minimum(b, n_bins - 1)


def edge_distance(tau: np.ndarray, f, n_bins: int) -> np.ndarray:
    """Distance of phi * M to the nearest integer, in bin widths."""
    u = fold_phase(tau, f) * float(n_bins)
    return np.abs(u - np.round(u))


def bin_sums(bins: np.ndarray, w: np.ndarray, x: np.ndarray, n_bins: int):
    """Per-bin W_m = sum w, Y_m = sum w x and counts N_m, summed in point order."""
    bins = np.asarray(bins, dtype=np.int64)
    W = np.bincount(bins, weights=w, minlength=n_bins)
    Y = np.bincount(bins, weights=w * x, minlength=n_bins)
    N = np.bincount(bins, minlength=n_bins)
    return W, Y, N


def statistic(W: np.ndarray, Y: np.ndarray, inv_alpha2: float = 0.0, stat_scale: str = "eq1"):
    """Eq. 1: S = sum over bins with W_m + 1/alpha^2 > 0 of Y_m^2 / (W_m + 1/alpha^2).

    ``W`` and ``Y`` hold the bins on their last axis; one S per leading index.
    """
    d = np.asarray(W, dtype=np.float64) + inv_alpha2
    Y = np.asarray(Y, dtype=np.float64)
    terms = np.where(d > 0, Y * Y / np.where(d > 0, d, 1.0), 0.0)
    s = terms.sum(axis=-1)
    return 0.5 * s if stat_scale == "listing_half" else s


def prepare_curve(t, y, dy, opt: OracleOptions | None = None):
    """(tau, w, x) for one curve: time offsets, inverse variances, centred flux."""
    opt = opt or OracleOptions()
    w = weights(dy)
    x = center(y, w, opt.center)
    tau = time_offsets(t, opt)
    return tau, w, x


def curve_bins(t, freqs, n_bins, opt: OracleOptions | None = None) -> np.ndarray:
    """Bin index of every (frequency, point) pair: int64 [n_freq, n_points]."""
    opt = opt or OracleOptions()
    tau = time_offsets(t, opt)
    freqs = np.asarray(freqs, dtype=np.float64)
    return phase_bins(tau[None, :], freqs[:, None], n_bins)


def curve_periodogram(t, y, dy, freqs, n_bins, opt: OracleOptions | None = None, block: int = 256) -> np.ndarray:
    """S(f) for one curve, FP64, one frequency at a time (vectorised over a block)."""
    opt = opt or OracleOptions()
    tau, w, x = prepare_curve(t, y, dy, opt)
    wx = w * x
    freqs = np.asarray(freqs, dtype=np.float64)
    n = len(tau)
    out = np.empty(len(freqs))
    for a in range(0, len(freqs), block):
        fb = freqs[a : a + block]
        nb = len(fb)
        bins = phase_bins(tau[None, :], fb[:, None], n_bins)  # [nb, n]
        flat = (bins + n_bins * np.arange(nb)[:, None]).ravel()
        W = np.bincount(flat, weights=np.broadcast_to(w, (nb, n)).ravel(), minlength=nb * n_bins)
        Y = np.bincount(flat, weights=np.broadcast_to(wx, (nb, n)).ravel(), minlength=nb * n_bins)
        out[a : a + nb] = statistic(W.reshape(nb, n_bins), Y.reshape(nb, n_bins), opt.inv_alpha2, opt.stat_scale)
    return out


def periodogram(offsets, t, y, dy, freqs, n_bins, opt: OracleOptions | None = None, curves=None) -> np.ndarray:
    """S[c, f] for the selected curves (all by default), FP64."""
    offsets = np.asarray(offsets)
    if curves is None:
        curves = range(len(offsets) - 1)
    curves = list(curves)
    out = np.empty((len(curves), len(freqs)))
    for r, c in enumerate(curves):
        a, b = int(offsets[c]), int(offsets[c + 1])
        out[r] = curve_periodogram(t[a:b], y[a:b], dy[a:b], freqs, n_bins, opt)
    return out


def shared_periodogram(t, y, dy, freqs, n_bins, opt: OracleOptions | None = None) -> np.ndarray:
    """S[c, f] for curves observed at common times t (y, dy: [n_curves, n_points]), FP64.

    Sec. 4 (the batch function for curves sharing timestamps): the bins of
    the common times are computed once per frequency and reused for every
    curve; each curve keeps its own weights and centring.
    """
    opt = opt or OracleOptions()
    y = np.asarray(y, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    n_curves = y.shape[0]
    prepared = [prepare_curve(t, y[c], dy[c], opt) for c in range(n_curves)]
    tau = prepared[0][0]  # the same offsets for every curve
    freqs = np.asarray(freqs, dtype=np.float64)
    out = np.empty((n_curves, len(freqs)))
    for r, f in enumerate(freqs):
        bins = phase_bins(tau, f, n_bins)
        for c, (_, w, x) in enumerate(prepared):
            W, Y, _ = bin_sums(bins, w, x, n_bins)
            out[c, r] = statistic(W, Y, opt.inv_alpha2, opt.stat_scale)
    return out


def peak_mask(S: np.ndarray) -> np.ndarray:
    """Index k is a peak iff S[k] > S[k-1] and S[k] >= S[k+1], with S[-1] = S[n] = -inf."""
    S = np.asarray(S)
    left = np.concatenate(([-np.inf], S[:-1]))
    right = np.concatenate((S[1:], [-np.inf]))
    return (S > left) & (S >= right)


def topk(S: np.ndarray, k: int):
    """The k highest peaks: ordered by S descending, then by index ascending.

    Returns (idx int64 [k], val [k]); missing entries are idx -1, val -inf.
    """
    S = np.asarray(S)
    cand = np.nonzero(peak_mask(S))[0]
    order = np.lexsort((cand, -S[cand]))  # primary: -S, secondary: index
    sel = cand[order[:k]]
    idx = np.full(k, -1, dtype=np.int64)
    val = np.full(k, -np.inf)
    idx[: len(sel)] = sel
    val[: len(sel)] = S[sel]
    return idx, val


def batch_topk(S2d: np.ndarray, k: int):
    idx = np.empty((S2d.shape[0], k), dtype=np.int64)
    val = np.empty((S2d.shape[0], k))
    for r in range(S2d.shape[0]):
        idx[r], val[r] = topk(S2d[r], k)
    return idx, val


# ---------------------------------------------------------------- multiple M from M_max (Sec. 3.4)


def combined_bins(fine_bins: np.ndarray, n_bins_max: int, n_bins: int, offset: int) -> np.ndarray:
    """Coarse bin of each point when the fine bins of M_max are combined k = M_max / M at a time.

    Sec. 3.4: sums for M = M_max / k are formed by combining the M_max sums,
    with k choices of offset.  Coarse bin c of offset o holds fine bins
    o + c k, ..., o + c k + k - 1 (mod M_max).
    """
    if n_bins_max % n_bins:
        raise ValueError("M must divide M_max")
    k = n_bins_max // n_bins
    if not 0 <= offset < k:
        raise ValueError("offset must be in [0, M_max / M)")
    return ((np.asarray(fine_bins, dtype=np.int64) - offset) % n_bins_max) // k


def variant_periodogram(t, y, dy, freqs, n_bins_max, n_bins, offset, opt: OracleOptions | None = None) -> np.ndarray:
    """S(f) with M bins obtained from the M_max fine bins at the given offset (FP64)."""
    opt = opt or OracleOptions()
    tau, w, x = prepare_curve(t, y, dy, opt)
    freqs = np.asarray(freqs, dtype=np.float64)
    out = np.empty(len(freqs))
    for r, f in enumerate(freqs):
        b = combined_bins(phase_bins(tau, f, n_bins_max), n_bins_max, n_bins, offset)
        W, Y, _ = bin_sums(b, w, x, n_bins)
        out[r] = statistic(W, Y, opt.inv_alpha2, opt.stat_scale)
    return out


# ---------------------------------------------------------------- phase entropy (App. C)


def phase_entropy(tau: np.ndarray, f: float, n_bins: int) -> float:
    """H = -sum_m (N_m / N) log(N_m / N) over occupied bins (App. C), natural log.

    N_m counts the observations in phase bin m at trial frequency f.
    """
    counts = np.bincount(phase_bins(np.asarray(tau, dtype=np.float64), f, n_bins), minlength=n_bins)
    p = counts[counts > 0] / float(len(tau))
    return float(-np.sum(p * np.log(p)))


def entropy_expectation(n_bins: int, n_obs: int) -> float:
    """App. C (Hutcheson): E(H) for equiprobable bins, to order 1/N^2."""
    M, N = float(n_bins), float(n_obs)
    return math.log(M) - (M - 1.0) / (2.0 * N) - (M - 1.0) * (M + 1.0) / (12.0 * N * N)


def entropy_variance(n_bins: int, n_obs: int) -> float:
    """App. C (Hutcheson): Var(H) for equiprobable bins, to order 1/N^3."""
    M, N = float(n_bins), float(n_obs)
    return (M - 1.0) / (2.0 * N * N) + (M * M - 1.0) / (6.0 * N * N * N)


# ---------------------------------------------------------------- baseline-marginalised FPW (App. A, general case)


def chebyshev_basis(t, n_terms: int, scale: float = 1.0) -> np.ndarray:
    """Baseline basis B [N, K] of App. A: column k is scale * T_k(s) at s = 2 (t - t_min) / (t_max - t_min) - 1.

    App. A suggests a Chebyshev polynomial basis for the drift without fixing
    its domain or amplitude: the curve's own time span is mapped to [-1, 1]
    (s = 0 for a single epoch) and the prior covariance is C_B = B B^T, so
    each coefficient has prior standard deviation ``scale`` in flux units.
    """
    t = np.asarray(t, dtype=np.float64)
    span = float(np.max(t) - np.min(t)) if len(t) else 0.0
    s = 2.0 * (t - np.min(t)) / span - 1.0 if span > 0 else np.zeros_like(t)
    B = np.empty((len(t), n_terms))
    for k in range(n_terms):
        if k == 0:
            B[:, k] = 1.0
        elif k == 1:
            B[:, k] = s
        else:
            B[:, k] = 2.0 * s * B[:, k - 1] - B[:, k - 2]
    return scale * B


def bm_statistic_dense(x, w, bins, n_bins: int, B, inv_alpha2: float) -> float:
    """App. A definition with dense matrices (finite alpha):

    S = X^T (C_B + C_sigma)^-1 X - X^T (C_B + C_P + C_sigma)^-1 X,
    C_sigma = diag(1/w), C_B = B B^T, C_P = P P^T with P = alpha * one-hot(bins).
    (App. A writes the change of chi-square with the opposite sign; S is the
    non-negative decrease.)
    """
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    E = np.zeros((n, n_bins))
    E[np.arange(n), np.asarray(bins)] = 1.0
    C0 = np.diag(1.0 / np.asarray(w, dtype=np.float64)) + B @ B.T
    C1 = C0 + (1.0 / inv_alpha2) * (E @ E.T)
    return float(x @ np.linalg.solve(C0, x) - x @ np.linalg.solve(C1, x))


def bm_periodogram(t, y, dy, freqs, n_bins: int, n_terms: int, scale: float = 1.0,
                   opt: OracleOptions | None = None, bins=None) -> np.ndarray:
    """Baseline-marginalised S(f) for one curve (App. A, general case), FP64.

    Follows App. A's steps: the frequency-independent inverse
    C_Bsigma^-1 = (C_B + C_sigma)^-1 is formed once (Woodbury on the low-rank
    C_B), then for each frequency the products with the one-hot P reduce to
    bin sums: u = E^T C_Bsigma^-1 X (bin sums of C_Bsigma^-1 X) and
    G = E^T C_Bsigma^-1 E (block sums of C_Bsigma^-1), and
    S = u^T (alpha^-2 I + G)^-1 u over the occupied bins (an empty bin has
    u_m = 0 and a zero row of G, so it adds nothing for any alpha).
    ``n_terms = 0`` is the plain statistic of Eq. 1.  ``bins`` ([n_freq, N])
    replaces the fold's bins (a point within rounding of an edge may sit in
    either neighbour).
    """
    opt = opt or OracleOptions()
    tau, w, x = prepare_curve(t, y, dy, opt)
    n = len(x)
    D = np.diag(w)
    if n_terms > 0:
        B = chebyshev_basis(t, n_terms, scale)
        H = np.eye(n_terms) + B.T @ D @ B
        Cinv = D - D @ B @ np.linalg.solve(H, B.T @ D)
    else:
        Cinv = D
    CX = Cinv @ x
    freqs = np.asarray(freqs, dtype=np.float64)
    out = np.empty(len(freqs))
    for r, f in enumerate(freqs):
        b = phase_bins(tau, f, n_bins) if bins is None else np.asarray(bins[r], dtype=np.int64)
        occ = np.unique(b)
        idx = np.searchsorted(occ, b)
        no = len(occ)
        u = np.bincount(idx, weights=CX, minlength=no)
        G = np.bincount((idx[:, None] * no + idx[None, :]).ravel(), weights=Cinv.ravel(), minlength=no * no)
        G = G.reshape(no, no)
        A = G + opt.inv_alpha2 * np.eye(len(occ))
        val = float(u @ np.linalg.solve(A, u))
        out[r] = 0.5 * val if opt.stat_scale == "listing_half" else val
    return out
