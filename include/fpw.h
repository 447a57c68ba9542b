/*
 * fpw.h -- C ABI of libfpw, the FPW periodogram on AMD Instinct MI355X (gfx950).
 *
 * The Fast Periodicity Weighting statistic (Finkbeiner, Prince & Whitebook,
 * arXiv 2502.00243, Eq. 1) of one light curve at one trial frequency f is
 *
 *     S(f) = sum_m Y_m^2 / (W_m + 1/alpha^2),
 *     W_m  = sum over points i in phase bin m of w_i,      w_i = 1 / (dy_i * dy_i)
 *     Y_m  = sum over points i in phase bin m of w_i x_i,  x_i = y_i - mean,
 *
 * where point i falls in bin m_i = floor(M * frac((t_i - t_ref) * f)),
 * zero-indexed (App. A, phase-bin equation; App. D listing).  Bins whose
 * denominator is zero (empty, with 1/alpha^2 = 0) contribute 0.
 *
 * The library evaluates S for every (curve, frequency) pair of a batch of
 * irregularly sampled light curves, and selects the k highest peaks of each
 * curve's periodogram (Sec. 3.5 post-processing).  Inputs cross the ABI as
 * plain pointers and sizes: host arrays at plan time, device buffers for
 * outputs.  No C++ or torch type appears here.
 *
 * Errors: every entry point returns an fpw_status and never throws or aborts.
 * On failure fpw_last_error() gives a message (thread-local, valid until the
 * next call on the same thread).  All argument checks (FPW_EINVAL) run on
 * the host before any HIP call.  HIP failures return FPW_EHIP.
 *
 * Threading: calls on one plan must not overlap; separate plans are
 * independent.  Work is enqueued on the HIP stream passed as `stream`
 * (a hipStream_t; NULL is the null stream); outputs are ready when that
 * stream is synchronised.
 */
#ifndef FPW_H
#define FPW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpw_plan_s* fpw_plan_t; /* opaque; owned by the library */

typedef enum {
  FPW_OK = 0,
  FPW_EINVAL = -1,       /* bad argument (host-side check, no HIP call made) */
  FPW_ENOMEM = -2,       /* host or device allocation failed */
  FPW_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  FPW_ESTATE = -4,       /* call not valid in the plan's state */
  FPW_EUNSUPPORTED = -5  /* valid input beyond this build's limits */
} fpw_status;

/* Mean subtracted before folding (Eq. 1 defines x as mean-subtracted; Sec. 3.5). */
enum {
  FPW_CENTER_WEIGHTED = 0, /* sum(w y)/sum(w): makes sum(w x) = 0, S ~ chi2(M-1) on noise */
  FPW_CENTER_MEAN = 1,     /* plain average of y */
  FPW_CENTER_NONE = 2      /* x = y */
};

/* Reference time t_ref of the fold (App. A: often the first observation; listing: 0). */
enum {
  FPW_TREF_ZERO = 0,  /* t_ref = 0; every t must be >= 0 */
  FPW_TREF_FIRST = 1, /* t_ref = min(t) of each curve */
  FPW_TREF_GIVEN = 2  /* t_ref = fpw_options.t_ref; every t must be >= t_ref */
};

/* Arithmetic that forms the phase and the bin (the only step whose rounding decides bins). */
enum {
  FPW_PHASE_FP64 = 0,         /* FP64 fused form: phase = frac(fma(tau, f, -(1/(2M) - delta))),
                                 bin = round(M * phase) with bin M folded onto 0; delta (set per
                                 plan from its largest tau * f) makes a point exactly on an edge
                                 take the upper bin, as floor does.  Bins equal
                                 floor(M frac(tau f)) on and off the edges except for points less
                                 than 1e-7 bin widths below an edge.  Where the plan's fold range
                                 would widen that band, the plan folds in the listing order
                                 instead and fpw_get_plan_info reports FPW_PHASE_FP64_LISTING. */
  FPW_PHASE_FP64_LISTING = 1, /* FP64 in the listing's order: p = fl(tau f), phi = p - floor(p),
                                 bin = floor(fl(phi M)).  Bit-exact with a plain FP64 loop. */
  FPW_PHASE_DF32 = 2,         /* compensated FP32: tau and f split hi+lo, error-free product,
                                 compensated fraction and bin. */
  FPW_PHASE_FP32 = 3          /* naive FP32 product (precision study only; wrong bins at
                                 large tau f) */
};

/* Scale of the statistic. */
enum {
  FPW_STAT_EQ1 = 0,          /* Eq. 1 as printed */
  FPW_STAT_LISTING_HALF = 1  /* times 1/2, as the App. D listing computes it */
};

#define FPW_MAX_BINS 255      /* largest M (phase-bin histograms live in LDS) */
#define FPW_MAX_DERIVED 4     /* derived bin counts per plan (multi-M reuse) */
#define FPW_MAX_VARIANTS 8    /* periodograms per pass: (M, offset) variants */
#define FPW_MAX_TOPK 16       /* largest k for peak selection */
#define FPW_MAX_CURVE_POINTS (1 << 24)
#define FPW_MAX_BASELINE_TERMS 3  /* Chebyshev terms of the marginalised baseline */
#define FPW_MAX_BASELINE_BINS 64  /* largest M with a marginalised baseline (LDS) */
#define FPW_MAX_WIDE_BINS 156     /* largest M for curves whose bin sums take the wide format (LDS) */

typedef struct {
  int32_t n_bins;      /* M >= 1; > FPW_MAX_BINS -> FPW_EUNSUPPORTED.  Default 10. */
  int32_t center;      /* FPW_CENTER_*; default WEIGHTED */
  int32_t tref_mode;   /* FPW_TREF_*; default ZERO */
  int32_t phase;       /* FPW_PHASE_*; default FP64 */
  int32_t stat_scale;  /* FPW_STAT_*; default EQ1 */
  int32_t topk;        /* k of the fused peak selection in fpw_eval_batch; 0 = none;
                          <= FPW_MAX_TOPK */
  double inv_alpha2;   /* 1/alpha^2 >= 0, finite (Eq. 1 prior); default 0 (alpha -> inf) */
  double t_ref;        /* used iff tref_mode == FPW_TREF_GIVEN */
  int32_t autotune;    /* 1: time candidate launch shapes at plan time and keep the fastest */
  int32_t use_graph;   /* 1 (default): replay fpw_eval_batch as one captured hipGraph (not
                          for the fused pass of small plans, see fuse_prepare).  0: launch
                          the pass's kernels directly, which costs the host about half as
                          much per call and measured 4-5 us less per pass back to back */
  int32_t freqs_per_lane; /* launch shape override, 0 = default: frequencies per lane (1, 2) */
  int32_t waves_per_group;/* launch shape override, 0 = default: waves per workgroup (1, 2, 4) */
  int32_t chunk_freqs;    /* launch shape override, 0 = default: frequencies per work item
                             (rounded up to a whole sweep of the wave).  The default
                             aims at ~12 items per persistent wave or group, raised
                             so an item carries >= 1.2e5 observation x frequency
                             evaluations per wave while every wave still gets an
                             item, within [one sweep, 16384]. */
  const char* tune_cache; /* path of a text cache of autotune results; NULL = none */
  int32_t point_source;   /* launch shape override: how a wave fetches observations.
                             0 = default (by M and the kind of plan; scalar loads for
                             the baseline kernel),
                             1 = scalar loads, 2 = vector loads + DPP broadcast (one
                             frequency per lane) */
  int32_t derived_bins[FPW_MAX_DERIVED];
                          /* multi-M reuse (Sec. 3.4): further bin counts M' < n_bins that
                             divide n_bins, 0-terminated.  Their sums are combined from the
                             n_bins fine sums of the same pass: coarse bin c of offset o
                             covers fine bins o + c*k .. o + c*k + k-1 (mod n_bins),
                             k = n_bins / M'.  Default: none. */
  int32_t all_offsets;    /* 1: every offset o = 0..k-1 of each derived M'; 0: offset 0 only */
  int32_t profile;        /* 1: record HIP events around each kernel of fpw_eval_batch
                             (read them with fpw_pass_timings); the pass is then
                             launched kernel by kernel instead of as a graph */
  int32_t shared_kernel;  /* plans made by fpw_plan_shared: FPW_SHARED_* (ignored otherwise) */
  int32_t baseline_terms; /* App. A general case: marginalise a baseline drift of K Chebyshev
                             terms T_0..T_{K-1} of the curve's time span mapped to [-1, 1],
                             0 <= K <= FPW_MAX_BASELINE_TERMS; 0 (default) = Eq. 1.  The
                             statistic becomes S = X^T C^-1 P (I + P^T C^-1 P)^-1 P^T C^-1 X
                             with C = C_B + C_sigma, C_B = B B^T (columns of B: baseline_scale
                             * T_k), C_sigma = diag(dy^2), P = alpha * one-hot(bins); empty
                             bins add nothing.  K > 0 needs the FP64 phase modes, n_bins <=
                             FPW_MAX_BASELINE_BINS and no derived bin counts. */
  double baseline_scale;  /* prior standard deviation of each baseline coefficient, in flux
                             units (> 0, finite; default 1) */
  int32_t hist_share;     /* launch shape override: waves that share one LDS histogram.
                             0 = default: by M (1 below 16 bins, 2 up to 31, 4 from 32;
                             4 also from 16 for one variant when n_points x n_freq is
                             below 1.5e8 per CU) when freqs_per_lane and waves_per_group
                             are 0 (and, with derived
                             bin counts, the phase mode is FP64), else 1.  1 = one private
                             histogram per wave.  2 or 4 = a workgroup of that many waves folds
                             disjoint slices of each curve's observations into one histogram
                             (waves_per_group must be 0 or equal; one frequency per lane;
                             derived bin counts only with the FP64 phase modes).  S is
                             summed in one fixed order for every launch shape, so results are
                             bit-identical to private histograms.  With baseline_terms > 0 it
                             sets the baseline kernel's sharing instead; 0 = by histogram size
                             per wave (1 below 8704 bytes, 2 below 12288, else 4). */
  int32_t fuse_prepare;   /* fused pass for small plans: the fold kernel prepares its curve
                             itself (each work item's workgroup of four waves reduces the
                             curve's constants and forms its records in registers), then
                             one workgroup per curve merges the peaks: two launches instead
                             of three, launched directly rather than as a graph (a graph
                             replay costs the host more than they do).  S and peaks are
                             bit-identical to the three-kernel pass.
                             0 = default: for plans of one periodogram variant and no
                             baseline terms with at most 4 items of 64 frequencies per CU
                             (n_curves * ceil(n_freq / 64) <= 4 * CUs), when no launch shape
                             override and no autotune is set.  -1 = never.  1 = always (FPW_EUNSUPPORTED with
                             derived bin counts, baseline terms, or a shape override other
                             than chunk_freqs and four waves per group). */
  int32_t sum_format;     /* FPW_SUMS_*: fixed-point format of the per-bin sums, see below.
                             Default AUTO. */
} fpw_options;

/*
 * Per-bin sums.  The bin sums W_m and Y_m are accumulated exactly as
 * integers after each point's w and w x are rounded once to a per-curve
 * fixed-point unit; the unit is Sum(w) / 2^B of weight and Sum|w x| / 2^(B-1)
 * of residual, so a light point's value carries a relative rounding error of
 * up to unit / (2 w).  fpw_plan measures, per curve,
 *   e_w   = W unit / (2 min w): the largest relative error of any bin's W,
 *   e_dup = W unit / (2 w) for the smallest weight w that at least
 *           max(2, N / (4 M)) points share (up to a quarter unit): such points
 *           round alike, so a bin filled with them keeps that error without
 *           averaging,
 *   e_y   = sqrt(Sum(1/w) (Sum(w) + M/alpha^2)) / 2^B: the rounding of the
 *           residual sums against the cancellation guard sum|w x|^2 / W,
 * and gives each curve one of two formats:
 *   narrow: one 64-bit word per bin, B = 32 (weight) / 31 (residual), when
 *           e_w <= 1e-4, e_dup <= 5e-6 and e_y <= 4e-6.  The W bound is a
 *           worst case reached only by a bin holding nothing but the lightest
 *           points with same-signed rounding; where weights differ the
 *           rounding errors are independent and S stays within ~1e-6.
 *   wide:   two 64-bit words per bin, B = 64 / 63 (scales 2^-11 below the
 *           limits), when e_w <= 1e-6 and e_y <= 1e-6 there: every bin within
 *           1e-6 of its exact sum.  About twice the LDS atomics per
 *           evaluation; FP64 phase modes, one periodogram variant.
 * A curve that fits neither (or a plan that needs the narrow format for every
 * curve: derived bin counts, baseline terms, the FPW_PHASE_DF32/FP32 modes,
 * the fused pass) makes fpw_plan return FPW_EUNSUPPORTED; so does a dy whose
 * 1/dy^2 is not a finite normal double.  fpw_get_plan_info reports how many
 * curves took the wide format.
 */
enum {
  FPW_SUMS_AUTO = 0,  /* per curve, as above */
  FPW_SUMS_WIDE = 1   /* every curve in the wide format */
};

/* Kernel of a shared-timestamp plan (fpw_plan_shared). */
enum {
  FPW_SHARED_AUTO = 0,    /* the matrix-core kernel where it applies (n_bins <= 64, phase FP64
                             or FP64_LISTING, no derived bin counts), else the general one */
  FPW_SHARED_GENERAL = 1, /* the general batched kernel, as for fpw_plan */
  FPW_SHARED_MATRIX = 2   /* the matrix-core kernel; FPW_EUNSUPPORTED where it does not apply */
};

/* Fills *opt with the defaults listed above. */
void fpw_options_default(fpw_options* opt);

/*
 * Creates a plan for a batch of light curves (Sec. 4: "individual light
 * curves as well as batches").  All arrays are HOST memory owned by the
 * caller; the plan copies what it needs to the device, so they may be freed
 * on return.
 *   n_curves   >= 1
 *   offsets    int64 [n_curves + 1]; curve c is points offsets[c] .. offsets[c+1]-1;
 *              offsets[0] = 0, every curve has >= 1 point (<= FPW_MAX_CURVE_POINTS)
 *   t, y, dy   float64 [offsets[n_curves]]: times (days), fluxes, flux errors;
 *              all finite, dy > 0, t - t_ref >= 0
 *   n_freq     >= 1, < 2^31
 *   freqs      float64 [n_freq], finite, > 0, any order and spacing (Sec. 1: any grid)
 *   opt        NULL = defaults
 *   stream     hipStream_t used for the uploads and any autotune launches
 * On success *out receives the plan (release with fpw_plan_destroy).
 */
fpw_status fpw_plan(fpw_plan_t* out, int64_t n_curves, const int64_t* offsets, const double* t,
                    const double* y, const double* dy, int64_t n_freq, const double* freqs,
                    const fpw_options* opt, void* stream);

/*
 * Creates a plan for curves that share their observation times (Sec. 4: the
 * batch function for light curves with common timestamps; App. C: every
 * source of one image field).  The phase bins of a time at a frequency are
 * then the same for all curves, so one fold serves the whole batch and the
 * per-bin sums of all curves at a frequency form one matrix product over the
 * observations: sums[curve][bin] = sum_p value[curve][p] * [bin(f, p) == bin].
 * The default kernel evaluates that product exactly on the int8 matrix cores
 * (fixed-point values split into base-256 digits, int32 accumulation); see
 * opt.shared_kernel.  Results have the same definition, layout and tolerance
 * as for fpw_plan on the equivalent CSR batch (every curve with the same t),
 * and every other entry point (fpw_eval_fp64, fpw_debug_bins,
 * fpw_phase_entropy, fpw_topk) accepts the plan as such a batch.
 *   n_curves   >= 1
 *   n_points   >= 1 (<= FPW_MAX_CURVE_POINTS): observations per curve
 *   t          float64 [n_points], HOST: the common times
 *   y, dy      float64 [n_curves * n_points], HOST, curve-major: fluxes and errors
 *   n_freq, freqs, opt, stream: as for fpw_plan
 * The plan holds the equivalent CSR batch as well (about 64 bytes of device
 * memory per curve and point) for the general kernel and the other entry
 * points.  With the matrix-core kernel it also owns a float32 periodogram
 * buffer [n_curves * n_freq] used when fpw_eval_batch gets S_dev = NULL.
 */
fpw_status fpw_plan_shared(fpw_plan_t* out, int64_t n_curves, int64_t n_points, const double* t, const double* y,
                           const double* dy, int64_t n_freq, const double* freqs, const fpw_options* opt,
                           void* stream);

/*
 * One pass of the periodogram over the plan's batch (Eq. 1 for every curve and
 * frequency): prepares weights, centred fluxes and time offsets on the device,
 * folds, bins, accumulates and reduces, and selects peaks.  A plan has
 * n_variants periodograms per curve (1 without derived bin counts; see
 * fpw_variant): variant 0 is n_bins at offset 0, then each derived M' with its
 * offsets in order.
 *   S_dev     DEVICE float32 [n_variants * n_curves * n_freq], row-major (variant,
 *             curve, frequency), or NULL to not store the periodogram.
 *   topk_idx  DEVICE int32 [n_variants * n_curves * opt.topk]: frequency indices of
 *             the highest peaks, best first (ties: lower index first); -1 where a
 *             curve has fewer.
 *   topk_val  DEVICE float32 [n_variants * n_curves * opt.topk]: their S values
 *             (-inf where idx = -1).
 *             Both NULL, or both non-NULL with opt.topk > 0 (else FPW_EINVAL).
 * Peak rule: index k is a peak iff S[k] > S[k-1] and S[k] >= S[k+1], with
 * S[-1] = S[n_freq] = -inf.
 * A plan owns its prepared records, queue counter and peak scratch, and every
 * pass rewrites them: passes of one plan must not overlap (enqueue them on one
 * stream, or synchronise between the streams used).
 */
fpw_status fpw_eval_batch(fpw_plan_t plan, float* S_dev, int32_t* topk_idx, float* topk_val,
                          void* stream);

/*
 * Peak selection over a periodogram already in device memory (Sec. 3.5):
 *   S_dev     DEVICE float32 [n_curves * n_freq] (the plan's shape), read only
 *   k         1 <= k <= min(FPW_MAX_TOPK, n_freq)
 *   idx_dev   DEVICE int32 [n_curves * k]; val_dev DEVICE float32 [n_curves * k]
 * Same peak rule and ordering as fpw_eval_batch's fused selection.
 */
fpw_status fpw_topk(fpw_plan_t plan, const float* S_dev, int32_t k, int32_t* idx_dev,
                    float* val_dev, void* stream);

/*
 * The plain per-curve FP64 comparator: one launch per curve, listing-order FP64
 * fold, FP64 per-bin sums and FP64 statistic (App. D "runFPW", re-designed as a
 * GPU kernel).  S_dev: DEVICE float64 [n_curves * n_freq].  Eq. 1 only:
 * FPW_EUNSUPPORTED for plans with baseline terms.
 */
fpw_status fpw_eval_fp64(fpw_plan_t plan, double* S_dev, void* stream);

/*
 * Parity hook: the bin index of every point of one curve at frequencies
 * f_begin .. f_end-1, computed by the same device code as the main kernels
 * for the given FPW_PHASE_* mode.
 *   bins_dev  DEVICE int32 [(f_end - f_begin) * N_curve], row-major by frequency.
 */
fpw_status fpw_debug_bins(fpw_plan_t plan, int32_t phase, int64_t curve, int64_t f_begin,
                          int64_t f_end, int32_t* bins_dev, void* stream);

/*
 * Kernel durations of the most recent fpw_eval_batch of a plan made with
 * opt.profile = 1, in milliseconds, measured with HIP events recorded on the
 * stream the kernels ran on: ms[0] prepare, ms[1] fold/bin/accumulate/reduce
 * (+ fused peaks), ms[2] peak merge (0 if not run).  In the fused pass of a
 * small plan (fuse_prepare) the fold kernel prepares its curves itself:
 * ms[0] is then ~0 and ms[1] includes the preparation.  Waits for that pass to
 * finish.  FPW_ESTATE if profiling is off or no pass has run.
 */
fpw_status fpw_pass_timings(fpw_plan_t plan, float ms[3]);

/*
 * The part of ms[1] of fpw_pass_timings spent in the wide-format fold kernel
 * (curves whose bin sums take the wide format, see FPW_SUMS_*), in
 * milliseconds, from a HIP event recorded between the two fold kernels: ms[1]
 * minus it is the batched kernel alone.  0 when the pass launched no wide
 * kernel.  Same conditions as fpw_pass_timings.
 */
fpw_status fpw_pass_wide_ms(fpw_plan_t plan, float* ms);

/*
 * Phase entropy of each curve's observation times at given trial frequencies
 * (App. C): H = -sum_m (N_m/N) log(N_m/N) over the plan's n_bins phase bins
 * (N_m observations of the curve in bin m, natural log), with the expectation
 * E and variance V of H for equiprobable bins (Hutcheson, as quoted in
 * App. C: E = log M - (M-1)/(2N) - (M^2-1)/(12N^2), V = (M-1)/(2N^2) +
 * (M^2-1)/(6N^3)).  A peak whose H lies far below E comes from regularities
 * of the sampling rather than from the source.  Bins follow the plan's phase
 * mode, as in fpw_eval_batch.
 *   freq_idx_dev  DEVICE int32 [n_curves * k]: frequency index for each (curve, slot),
 *                 e.g. fpw_eval_batch's top-k output; slots whose index is outside
 *                 [0, n_freq) are skipped
 *   H_dev, E_dev, V_dev  DEVICE float32 [n_curves * k]; NaN in skipped slots
 *   k             1 <= k <= n_freq
 */
fpw_status fpw_phase_entropy(fpw_plan_t plan, const int32_t* freq_idx_dev, int32_t k, float* H_dev,
                             float* E_dev, float* V_dev, void* stream);

/* Bin count and offset of periodogram variant v (0 <= v < n_variants). */
fpw_status fpw_variant(fpw_plan_t plan, int32_t v, int32_t* n_bins, int32_t* offset);

/* What a plan holds and the launch shape it chose. */
typedef struct {
  int64_t n_curves, n_freq, n_points;
  int64_t evals;          /* n_points * n_freq: observation x frequency evaluations per pass */
  int32_t n_bins, topk, phase;
  int32_t freqs_per_lane, waves_per_group, chunk_freqs;
  int32_t grid_groups;    /* persistent workgroups launched */
  int32_t work_items;     /* (curve, frequency chunk) items in the queue */
  int32_t lds_bytes;      /* LDS per workgroup */
  int32_t tuned;          /* 1 if the launch shape came from the autotuner or its cache */
  int32_t point_source;   /* 1 scalar loads, 2 vector loads + DPP broadcast, 3 records formed
                             in the lanes + readlane broadcast (fused pass) */
  int32_t n_variants;     /* periodograms per curve and pass */
  int32_t kernel;         /* 0 general batched kernel, 1 shared-timestamp matrix-core kernel,
                             2 baseline-marginalised kernel */
  int32_t hist_share;     /* waves per LDS histogram (1, 2, 4) of the general batched kernel
                             or of the baseline kernel; 0 for the matrix-core kernel */
  int32_t fuse_prepare;   /* 1 if the plan runs the fused pass (see fpw_options) */
  int32_t n_wide_curves;  /* curves whose bin sums take the wide format (see FPW_SUMS_*) */
  int64_t n_wide_points;  /* their observations (the wide kernel folds n_wide_points * n_freq) */
} fpw_plan_info;

fpw_status fpw_get_plan_info(fpw_plan_t plan, fpw_plan_info* info);

/*
 * One periodogram pass with no plan and no allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Inputs and outputs are the caller's
 * DEVICE buffers, with the layouts of fpw_plan and fpw_eval_batch:
 *   offsets      int64 [n_curves + 1]; t, y, dy float64 [n_points]; freqs float64 [n_freq]
 *   S_dev        float32 [n_curves * n_freq] or NULL
 *   topk_idx, topk_val  int32 / float32 [n_curves * opt.topk] or both NULL
 * Every other buffer the pass needs lives in one static device array of 16 MiB
 * per GPU (kept until the process ends): with topk k it must hold about
 * 32 n_points + 44 n_curves + (36 + 8k) n_items bytes (n_items = n_curves *
 * chunks per curve, about one per workgroup the GPU holds at once; 256-byte
 * alignment of each region on top), else FPW_EUNSUPPORTED.
 * The sums take the wide format (see FPW_SUMS_*) and the phase is folded in
 * the listing order (FPW_PHASE_FP64 and FPW_PHASE_FP64_LISTING give the same
 * exact-floor bins here), so S has the plan's definition and tolerance; a curve
 * whose weights exceed the wide format's bound gets S = NaN and no peaks.
 * Options: n_bins <= FPW_MAX_WIDE_BINS, center, tref_mode, t_ref, inv_alpha2,
 * stat_scale, topk; FPW_EUNSUPPORTED for the FP32-based phase modes, derived
 * bin counts, baseline terms, autotune and launch-shape overrides.
 * The argument checks cover sizes, pointers and options only (FPW_EINVAL,
 * before any HIP call): the values on the device are not read on the host,
 * so they must meet fpw_plan's conditions for S to be meaningful (no device
 * access leaves the buffers whatever they hold).  Calls that overlap on one
 * GPU race on the static array: serialise them (one stream, or synchronise).
 */
fpw_status fpw_eval_static(int64_t n_curves, const int64_t* offsets, int64_t n_points, const double* t,
                           const double* y, const double* dy, int64_t n_freq, const double* freqs,
                           const fpw_options* opt, float* S_dev, int32_t* topk_idx, float* topk_val,
                           void* stream);

/* Releases the plan and its device memory.  NULL is a no-op. */
void fpw_plan_destroy(fpw_plan_t plan);

/* Message for the last failure on this thread ("" if none). */
const char* fpw_last_error(void);

/* Library version, e.g. "fpw 0.1.0 gfx950". */
const char* fpw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FPW_H */
