// Host runtime of libfpw: argument checks, plan construction, work queue,
// launch-shape selection (defaults, autotuner and its cache), hipGraph
// capture and the C ABI declared in include/fpw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fpw.h"
#include "fpw_internal.h"

namespace {

thread_local std::string g_err;

fpw_status fail(fpw_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

fpw_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? FPW_ENOMEM : FPW_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define FPW_HIP(call, what)                     \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Device buffer owned by a plan.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = n;
    return n ? hipMalloc(&p, n) : hipSuccess;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

}  // namespace

struct fpw_plan_s {
  fpw_options opt{};
  int64_t n_curves = 0, n_freq = 0, n_points = 0;
  int device = 0;
  int n_cu = 0;
  std::vector<int64_t> h_offsets;
  std::vector<fpw::Item> h_items_nat;  // natural order (curve, chunk)
  // device inputs and prepared data
  DevBuf t, y, dy, offsets, freqs, rec, cc, tau64, w64, wx64;
  // work queue and peak-selection scratch
  DevBuf items, queue, cand_val, cand_idx, edge, slot_k0, curve_slot;
  fpw::Shape shape{1, 1, 4096, 0, 1};
  fpw::Variants var{};        // periodogram variants (multi-M reuse); var.n >= 1
  // per-bin sum formats (fpw.h, "Per-bin sums"): fpw::FMT_* per curve, the
  // first wide record of each curve, the wide queue and its launch shape
  std::vector<uint8_t> h_fmt;
  std::vector<int64_t> h_offw;
  int64_t n_wide = 0;
  DevBuf fmt, offw, recw, wc, items_w;
  int n_items_w = 0;
  int wide_share = 1, wide_grid = 0;
  // shift of the fused FP64 fold (see fused_fold_shift); fused_fold is false
  // when the plan's fold range made it fold in the listing order instead
  double fold_nh = 0.0;
  bool fused_fold = true;
  std::vector<int32_t> var_bins;  // bin count of each variant
  int grid_groups = 0;
  size_t lds_bytes = 0;
  int n_items = 0;
  bool tuned = false;
  // graph of one eval pass
  // Captured passes, one per set of output pointers (a few kept, least
  // recently used dropped): callers that alternate between output buffers,
  // as a caching allocator does, replay without re-capturing.
  struct Graph {
    float* S;
    int32_t* idx;
    float* val;
    hipGraph_t g;
    hipGraphExec_t x;
    uint64_t used;
  };
  static constexpr size_t kMaxGraphs = 4;
  std::vector<Graph> graphs;
  uint64_t graph_clock = 0;
  hipStream_t cap_stream = nullptr;
  bool graph_ok = true;
  void drop_graphs() {
    for (Graph& e : graphs) {
      if (e.x) (void)hipGraphExecDestroy(e.x);
      if (e.g) (void)hipGraphDestroy(e.g);
    }
    graphs.clear();
  }
  // shared-timestamp plans on the matrix cores
  bool mfma = false;
  int32_t sh_points = 0, sh_kblocks = 0, sh_chunk = 0, sh_fw = 0, sh_nb = 2, sh_rounds = 0, sh_priv = 0;
  int sh_grid_x = 0, sh_grid_y = 0;
  size_t sh_lds = 0;
  DevBuf sh_tau, sh_vals, sh_cc, sh_S;
  // marginalised baseline (App. A general case)
  bool bm = false;
  int bm_grid = 0;
  int bm_share = 1;   // waves per histogram of the baseline kernel
  int bm_source = 0;  // its point source: 0 scalar loads, 1 vector loads + DPP broadcast
  DevBuf bm_rec, bm_z, bm_const, bm_S;
  // fused pass (small plans): prepare fused into the fold kernel, then the merge
  bool fused = false;
  // profiling events: before prepare, after prepare, after the fold kernels, after merge, and between
  // the batched and the wide-format fold kernels
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool ev_recorded = false;
  bool ev_merge = false;
  bool ev_wide = false;
  ~fpw_plan_s() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

const int kWave = 64;
// Smallest M for which, by default, two waves share one histogram (and four
// from kShare4MinBins): a private histogram of M+1 slots per wave would
// leave room for too few waves per CU (measured on 1000 ZTF-like curves:
// M = 20 +10 % with two waves, M = 50 +73 % with four, M = 10 even).
const int kShare2MinBins = 16;
const int kShare4MinBins = 32;
// Below this many evaluations (n_points x n_freq) per CU, one variant with
// 16 <= M < 32 takes four waves per histogram instead of two: fewer, longer
// items even out the tail of a short pass (measured with N ~ U(100, 1000),
// M = 20: 7-15 % faster up to 1.6e10 evaluations on 256 CUs, even at 5e10,
// two waves 1 % faster on the 5.5e10 of 1000 ZTF-like curves).
const double kShare4SmallPlanEvalsPerCu = 1.5e8;
// Smallest M for which the default point source is the DPP broadcast, with
// private histograms (or more than four variants) and with shared histograms
// and up to four variants (their extra waves hide the scalar loads' waits up
// to M ~ 100).
const int kDppMinBins = 32;
const int kDppMinBinsShared = 128;
// Largest plan that runs the fused pass by default, in items of 64
// frequencies per CU (measured with N ~ U(100, 1000), M = 20, 4-64 curves:
// the fused pass is 1.05-1.2x faster at 3-4 items per CU, 0.9x at 5 and
// 0.8-0.9x at 6-7; beyond ~100 the persistent kernel is up to 2.3x faster).
const int kFusedItemsPerCu = 4;
// Smallest work item of the persistent kernel, in evaluations per wave: a
// pop of the queue's one counter costs ~20 ns serialised, so with ~3300
// waves popping an item has to keep its wave busy ~70 us (~1.2e5
// evaluations) for the counter to stay off the critical path (measured on
// mid-size plans: 3e4, 6e4, 1.2e5, 2.4e5 -> 1.2e5 best or within noise).
const double kMinItemEvalsPerWave = 1.2e5;

bool finite(double v) { return std::isfinite(v); }

// The fused FP64 fold forms phase' = frac(fma(tau, f, nh)) and takes
// round(M phase') as the bin.  nh = -(1/(2M) - delta): with delta = 2^(e-52),
// where 2^e exceeds every |tau f| of the plan, delta is at least four times
// the rounding error of that fma, so a point exactly on a bin edge lies above
// the rounding midpoint and takes the upper bin, as floor() does (App. A
// phase-bin equation), rather than following round-half-to-even.  The cost:
// points less than ~1.375 M delta bin widths below an edge move up too.  The
// fused fold is used while that band stays under 1e-7 bin widths (a tenth of
// the near-edge tolerance); *ok is false beyond, and the plan then folds in
// the listing order.
double fused_fold_shift(int M, double max_cycles, bool* ok) {
  int ex = 0;
  (void)std::frexp(std::max(max_cycles, 1.0), &ex);  // 2^ex > max_cycles
  const double delta = std::ldexp(1.0, ex - 52);
  *ok = 1.375 * (double)M * delta <= 1e-7;
  return -(0.5 / (double)M - delta);
}

// ---------------------------------------------------------------- per-bin sum formats
// The bin sums are exact integers of values rounded once to a per-curve unit
// (fpw.h, "Per-bin sums").  For one curve and a field capacity cap_w
// (weights) / cap_y (residuals), with u = Sum(w) / cap_w:
//   e_w   = u / (2 min w): the worst relative error of any bin's W (a bin's
//           error over its weight is at most the largest error over weight
//           of its points);
//   e_dup = u / (2 w) for the smallest w of a run of at least
//           max(2, ceil(N / (4 M))) weights (in sorted order) each closer
//           than u / 4 to the next: points of (nearly) equal weight round
//           alike, so a bin filled with them keeps that error instead of
//           averaging it (a few such points are no worse than one point,
//           which e_w covers);
//   e_y   = sqrt(Sum(1/w) (Sum(w) + M/alpha^2)) / (2 cap_y): with |E_m| the
//           rounding of a bin's residual sum, Sum_m E_m^2 / W_m <= Sum_i
//           e_i^2 / w_i <= (v/2)^2 Sum(1/w), v = Sum|w x| / cap_y, against the
//           guard scale S_abs >= Sum|w x|^2 / (Sum(w) + M/alpha^2).
constexpr double kNarrowMaxW = 1e-4, kNarrowMaxDup = 5e-6, kNarrowMaxY = 4e-6;
constexpr double kWideMax = 1e-6;
constexpr double kWideCapW = 18446744073709551616.0 * (1.0 - 1.0 / 2048.0);  // as the prepare kernel's scales
constexpr double kWideCapY = 9223372036854775808.0 * (1.0 - 1.0 / 2048.0);

struct SumBounds {
  double e_w = 0, e_dup = 0, e_y = 0;
};

// Per-curve quantities the bounds need: N, Sum(w), min w, Sum(1/w), Sum|w x|
// and the weights in ascending order.
struct CurveWeights {
  int64_t n = 0;
  double sw = 0, wmin = 0, h = 0, a = 0;
  std::vector<double> w;  // sorted
};

void curve_weights(const double* y, const double* dy, int64_t n, int center, CurveWeights* cw) {
  cw->n = n;
  cw->w.resize((size_t)n);
  double sw = 0, swy = 0, sy = 0, h = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double w = 1.0 / (dy[i] * dy[i]);
    cw->w[(size_t)i] = w;
    sw += w;
    swy += w * y[i];
    sy += y[i];
    h += dy[i] * dy[i];
  }
  const double mu = center == FPW_CENTER_WEIGHTED ? swy / sw : (center == FPW_CENTER_MEAN ? sy / (double)n : 0.0);
  double a = 0;
  for (int64_t i = 0; i < n; ++i) a += std::fabs(cw->w[(size_t)i] * (y[i] - mu));
  std::sort(cw->w.begin(), cw->w.end());
  cw->sw = sw;
  cw->wmin = cw->w[0];
  cw->h = h;
  cw->a = a;
}

SumBounds sum_bounds(const CurveWeights& cw, double cap_w, double cap_y, int M, double ia2, bool dup) {
  SumBounds b;
  const double u = cw.sw / cap_w;
  b.e_w = u / (2.0 * cw.wmin);
  b.e_y = std::sqrt(cw.h * (cw.sw + M * ia2)) / (2.0 * cap_y);
  if (dup) {
    const size_t k_min = (size_t)std::max<int64_t>(2, (cw.n + 4 * (int64_t)M - 1) / (4 * (int64_t)M));
    for (size_t i = 0; i < cw.w.size();) {
      size_t j = i + 1;
      while (j < cw.w.size() && cw.w[j] - cw.w[j - 1] < 0.25 * u) ++j;
      if (j - i >= k_min) {
        b.e_dup = u / (2.0 * cw.w[i]);
        break;
      }
      i = j;
    }
  }
  return b;
}

bool narrow_fits(const CurveWeights& cw, int M, double ia2, double cap_w, double cap_y, SumBounds* b) {
  *b = sum_bounds(cw, cap_w, cap_y, M, ia2, true);
  return b->e_w <= kNarrowMaxW && b->e_dup <= kNarrowMaxDup && b->e_y <= kNarrowMaxY;
}

// The format of every curve (fpw::FMT_*): narrow where it fits, else wide
// where that fits, else FPW_EUNSUPPORTED (also where the plan needs the
// narrow format for every curve).  `cap_shift` 0 for the general kernels;
// the baseline kernel's Z sums have 31-bit fields.  Curves are split over
// host threads.
fpw_status choose_formats(int64_t n_curves, const int64_t* offsets, const double* y, const double* dy,
                          const fpw_options& o, int n_var, std::vector<uint8_t>* fmt, int64_t* n_wide) {
  fmt->assign((size_t)n_curves, (uint8_t)fpw::FMT_NARROW);
  const bool bm = o.baseline_terms > 0;
  std::vector<int64_t> bad((size_t)n_curves, 0);  // 1 narrow impossible here, 2 no format fits
  std::vector<SumBounds> why((size_t)n_curves);
  const int64_t pts = offsets[n_curves];
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::max(1u, std::thread::hardware_concurrency()),
                                                               (int64_t)16, 1 + pts / 200000}));
  auto work = [&](int tid) {
    CurveWeights cw;
    for (int64_t c = tid; c < n_curves; c += nt) {
      const int64_t a = offsets[c], n = offsets[c + 1] - offsets[c];
      curve_weights(y + a, dy + a, n, o.center, &cw);
      if (!std::isfinite(cw.sw) || !std::isfinite(cw.a)) {
        bad[(size_t)c] = 3;
        continue;
      }
      SumBounds b;
      const double nd = (double)n;
      const double cap_w = (bm ? 2147483648.0 - 2.0 - nd : 4294967296.0 - 2.0 - 2.0 * nd);
      const double cap_y = 2147483648.0 - 2.0 - nd;
      if (o.sum_format != FPW_SUMS_WIDE && narrow_fits(cw, o.n_bins, o.inv_alpha2, cap_w, cap_y, &b)) continue;
      if (o.sum_format == FPW_SUMS_WIDE) b = sum_bounds(cw, cap_w, cap_y, o.n_bins, o.inv_alpha2, true);
      why[(size_t)c] = b;
      if (bm) {
        bad[(size_t)c] = 1;
        continue;
      }
      const SumBounds wb = sum_bounds(cw, kWideCapW, kWideCapY, o.n_bins, o.inv_alpha2, false);
      if (std::max(wb.e_w, 0x1p-53) <= kWideMax && wb.e_y <= kWideMax) {
        (*fmt)[(size_t)c] = (uint8_t)fpw::FMT_WIDE;
      } else {
        bad[(size_t)c] = 2;
        why[(size_t)c] = wb;
      }
    }
  };
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work, i);
  work(0);
  for (std::thread& t : th) t.join();
  *n_wide = 0;
  for (int64_t c = 0; c < n_curves; ++c) {
    const SumBounds& b = why[(size_t)c];
    if (bad[(size_t)c] == 3)
      return fail(FPW_EUNSUPPORTED, "curve %lld: sum of 1/dy^2 or of |w x| overflows", (long long)c);
    if (bad[(size_t)c] == 1)
      return fail(FPW_EUNSUPPORTED,
                  "curve %lld: its weights span too wide a range for the baseline kernel's 32-bit sums "
                  "(e_w %.3g, e_dup %.3g, e_y %.3g; limits %g, %g, %g)",
                  (long long)c, b.e_w, b.e_dup, b.e_y, kNarrowMaxW, kNarrowMaxDup, kNarrowMaxY);
    if (bad[(size_t)c] == 2)
      return fail(FPW_EUNSUPPORTED,
                  "curve %lld: its weights span too wide a range even for the wide bin sums (e_w %.3g, e_y %.3g; "
                  "limit %g)",
                  (long long)c, b.e_w, b.e_y, kWideMax);
    *n_wide += (*fmt)[(size_t)c] == fpw::FMT_WIDE;
  }
  if (*n_wide > 0) {
    const char* why_narrow = n_var > 1 ? "derived bin counts"
                             : (o.phase >= FPW_PHASE_DF32 ? "the FP32-based phase modes"
                                                          : (o.fuse_prepare == 1 ? "the fused pass" : nullptr));
    if (why_narrow)
      return fail(FPW_EUNSUPPORTED, "%lld curve(s) need the wide bin sums, which %s do not support", (long long)*n_wide,
                  why_narrow);
    if (o.n_bins > FPW_MAX_WIDE_BINS)
      return fail(FPW_EUNSUPPORTED, "%lld curve(s) need the wide bin sums, built for n_bins <= %d", (long long)*n_wide,
                  FPW_MAX_WIDE_BINS);
  }
  return FPW_OK;
}

fpw_status check_options(const fpw_options& o) {
  if (o.n_bins < 1) return fail(FPW_EINVAL, "n_bins must be >= 1 (got %d)", o.n_bins);
  if (o.n_bins > FPW_MAX_BINS) return fail(FPW_EUNSUPPORTED, "n_bins %d exceeds FPW_MAX_BINS=%d", o.n_bins, FPW_MAX_BINS);
  if (o.center < 0 || o.center > 2) return fail(FPW_EINVAL, "bad center mode %d", o.center);
  if (o.tref_mode < 0 || o.tref_mode > 2) return fail(FPW_EINVAL, "bad tref_mode %d", o.tref_mode);
  if (o.phase < 0 || o.phase > 3) return fail(FPW_EINVAL, "bad phase mode %d", o.phase);
  if (o.stat_scale < 0 || o.stat_scale > 1) return fail(FPW_EINVAL, "bad stat_scale %d", o.stat_scale);
  if (o.topk < 0) return fail(FPW_EINVAL, "topk must be >= 0");
  if (o.topk > FPW_MAX_TOPK) return fail(FPW_EUNSUPPORTED, "topk %d exceeds FPW_MAX_TOPK=%d", o.topk, FPW_MAX_TOPK);
  if (!finite(o.inv_alpha2) || o.inv_alpha2 < 0) return fail(FPW_EINVAL, "inv_alpha2 must be finite and >= 0");
  if (o.tref_mode == FPW_TREF_GIVEN && !finite(o.t_ref)) return fail(FPW_EINVAL, "t_ref must be finite");
  if (o.freqs_per_lane < 0 || o.freqs_per_lane > 2) return fail(FPW_EINVAL, "freqs_per_lane must be 0, 1 or 2");
  if (o.freqs_per_lane == 2 && o.phase >= FPW_PHASE_DF32)
    return fail(FPW_EUNSUPPORTED, "freqs_per_lane 2 is built for the FP64 phase modes only");
  if (!(o.waves_per_group == 0 || o.waves_per_group == 1 || o.waves_per_group == 2 || o.waves_per_group == 4))
    return fail(FPW_EINVAL, "waves_per_group must be 0, 1, 2 or 4");
  if (o.chunk_freqs < 0) return fail(FPW_EINVAL, "chunk_freqs must be >= 0");
  if (o.point_source < 0 || o.point_source > 2) return fail(FPW_EINVAL, "point_source must be 0, 1 or 2");
  if (o.point_source == 2 && o.freqs_per_lane == 2)
    return fail(FPW_EUNSUPPORTED, "DPP point broadcast is built for one frequency per lane");
  if (!(o.hist_share == 0 || o.hist_share == 1 || o.hist_share == 2 || o.hist_share == 4))
    return fail(FPW_EINVAL, "hist_share must be 0, 1, 2 or 4");
  if (o.hist_share > 1) {
    if (o.freqs_per_lane == 2) return fail(FPW_EUNSUPPORTED, "a shared histogram is built for one frequency per lane");
    if (o.waves_per_group != 0 && o.waves_per_group != o.hist_share)
      return fail(FPW_EINVAL, "with hist_share %d the workgroup has %d waves (waves_per_group 0 or %d)", o.hist_share,
                  o.hist_share, o.hist_share);
  }
  int nvar = 1;
  for (int d = 0; d < FPW_MAX_DERIVED && o.derived_bins[d] != 0; ++d) {
    const int m = o.derived_bins[d];
    if (m < 1 || m >= o.n_bins || o.n_bins % m != 0)
      return fail(FPW_EINVAL, "derived bin count %d must divide n_bins %d and be smaller", m, o.n_bins);
    for (int e = 0; e < d; ++e)
      if (o.derived_bins[e] == m) return fail(FPW_EINVAL, "derived bin count %d listed twice", m);
    nvar += o.all_offsets ? o.n_bins / m : 1;
  }
  if (nvar > FPW_MAX_VARIANTS)
    return fail(FPW_EUNSUPPORTED, "%d periodogram variants exceed FPW_MAX_VARIANTS=%d", nvar, FPW_MAX_VARIANTS);
  if (nvar > 1 && o.freqs_per_lane == 2)
    return fail(FPW_EUNSUPPORTED, "derived bin counts are built for one frequency per lane");
  if (nvar > 1 && o.hist_share > 1 && o.phase >= FPW_PHASE_DF32)
    return fail(FPW_EUNSUPPORTED, "derived bin counts with a shared histogram are built for the FP64 phase modes");
  if (o.shared_kernel < 0 || o.shared_kernel > 2) return fail(FPW_EINVAL, "shared_kernel must be 0, 1 or 2");
  if (o.fuse_prepare < -1 || o.fuse_prepare > 1) return fail(FPW_EINVAL, "fuse_prepare must be -1, 0 or 1");
  if (o.sum_format != FPW_SUMS_AUTO && o.sum_format != FPW_SUMS_WIDE)
    return fail(FPW_EINVAL, "sum_format must be FPW_SUMS_AUTO or FPW_SUMS_WIDE");
  if (o.sum_format == FPW_SUMS_WIDE && o.baseline_terms > 0)
    return fail(FPW_EUNSUPPORTED, "the baseline kernel keeps its sums in the narrow format");
  if (o.fuse_prepare == 1 && (nvar > 1 || o.baseline_terms != 0))
    return fail(FPW_EUNSUPPORTED, "the fused pass serves plans with one periodogram variant and no baseline terms");
  if (o.fuse_prepare == 1 && (o.freqs_per_lane == 2 || o.point_source != 0 || o.waves_per_group == 1 ||
                              o.waves_per_group == 2 || o.hist_share == 1 || o.hist_share == 2))
    return fail(FPW_EUNSUPPORTED, "the fused pass runs four waves per histogram and its own point source");
  if (o.baseline_terms < 0) return fail(FPW_EINVAL, "baseline_terms must be >= 0");
  if (o.baseline_terms > FPW_MAX_BASELINE_TERMS)
    return fail(FPW_EUNSUPPORTED, "baseline_terms %d exceeds FPW_MAX_BASELINE_TERMS=%d", o.baseline_terms, FPW_MAX_BASELINE_TERMS);
  if (o.baseline_terms > 0) {
    if (!finite(o.baseline_scale) || !(o.baseline_scale > 0))
      return fail(FPW_EINVAL, "baseline_scale must be finite and > 0");
    if (o.phase != FPW_PHASE_FP64 && o.phase != FPW_PHASE_FP64_LISTING)
      return fail(FPW_EUNSUPPORTED, "a marginalised baseline is built for the FP64 phase modes");
    if (o.n_bins > FPW_MAX_BASELINE_BINS)
      return fail(FPW_EUNSUPPORTED, "n_bins %d exceeds FPW_MAX_BASELINE_BINS=%d", o.n_bins, FPW_MAX_BASELINE_BINS);
    if (nvar > 1) return fail(FPW_EUNSUPPORTED, "derived bin counts are not built with a marginalised baseline");
  }
  return FPW_OK;
}

fpw_status validate(int64_t n_curves, const int64_t* offsets, const double* t, const double* y, const double* dy,
                    int64_t n_freq, const double* freqs, const fpw_options& o, double* max_tau, double* max_f) {
  if (n_curves < 1) return fail(FPW_EINVAL, "n_curves must be >= 1");
  if (n_curves > INT32_MAX - 1) return fail(FPW_EUNSUPPORTED, "n_curves too large");
  if (!offsets || !t || !y || !dy || !freqs) return fail(FPW_EINVAL, "null input pointer");
  if (n_freq < 1) return fail(FPW_EINVAL, "n_freq must be >= 1");
  if (n_freq >= INT32_MAX) return fail(FPW_EUNSUPPORTED, "n_freq must be < 2^31");
  if (offsets[0] != 0) return fail(FPW_EINVAL, "offsets[0] must be 0");
  for (int64_t c = 0; c < n_curves; ++c) {
    const int64_t n = offsets[c + 1] - offsets[c];
    if (n < 1) return fail(FPW_EINVAL, "curve %lld has no points (offsets must increase)", (long long)c);
    if (n > FPW_MAX_CURVE_POINTS)
      return fail(FPW_EUNSUPPORTED, "curve %lld has %lld points (> %d)", (long long)c, (long long)n, FPW_MAX_CURVE_POINTS);
  }
  *max_tau = 0.0;
  for (int64_t c = 0; c < n_curves; ++c) {
    double tmin = INFINITY, tmax = -INFINITY;
    for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i) {
      if (!finite(t[i]) || !finite(y[i]) || !finite(dy[i]))
        return fail(FPW_EINVAL, "non-finite t, y or dy at point %lld", (long long)i);
      if (!(dy[i] > 0)) return fail(FPW_EINVAL, "dy must be > 0 (point %lld)", (long long)i);
      const double w = 1.0 / (dy[i] * dy[i]);
      if (!(w >= DBL_MIN && w <= DBL_MAX))
        return fail(FPW_EUNSUPPORTED, "1/dy^2 of point %lld (dy = %g) is not a finite normal double", (long long)i,
                    dy[i]);
      tmin = std::min(tmin, t[i]);
      tmax = std::max(tmax, t[i]);
    }
    const double tref = o.tref_mode == FPW_TREF_ZERO ? 0.0 : (o.tref_mode == FPW_TREF_FIRST ? tmin : o.t_ref);
    if (tmin - tref < 0)
      return fail(FPW_EINVAL, "t - t_ref must be >= 0 (curve %lld starts at %g, t_ref %g)", (long long)c, tmin, tref);
    *max_tau = std::max(*max_tau, tmax - tref);
  }
  *max_f = 0.0;
  for (int64_t k = 0; k < n_freq; ++k) {
    if (!finite(freqs[k]) || !(freqs[k] > 0)) return fail(FPW_EINVAL, "frequency %lld must be finite and > 0", (long long)k);
    *max_f = std::max(*max_f, freqs[k]);
  }
  if (o.topk > n_freq) return fail(FPW_EINVAL, "topk %d exceeds n_freq %lld", o.topk, (long long)n_freq);
  // Range of the fold for each phase encoding (the fused FP64 fold hands over
  // to the listing order itself where its range would blur the edges).
  const double cycles = *max_tau * *max_f;
  if (!finite(cycles)) return fail(FPW_EUNSUPPORTED, "tau*f overflows (max tau %g, max f %g)", *max_tau, *max_f);
  if ((o.phase == FPW_PHASE_DF32 || o.phase == FPW_PHASE_FP32) && cycles >= 4194304.0)
    return fail(FPW_EUNSUPPORTED, "tau*f = %g cycles too large for the FP32 phase encodings (< 2^22)", cycles);
  return FPW_OK;
}

}  // namespace

namespace {

// ---------------------------------------------------------------- work queue
// Frequencies of every curve are cut into chunks of `chunk` (a multiple of the
// frequencies a wave covers per sweep).  A trailing chunk of one frequency is
// merged into its predecessor so every chunk of a multi-frequency grid has at
// least two frequencies, which the cross-chunk peak test relies on.
void build_items(fpw_plan_s* p, int chunk, std::vector<fpw::Item>* nat, std::vector<int32_t>* slot_k0,
                 std::vector<int32_t>* curve_slot) {
  nat->clear();
  slot_k0->clear();
  curve_slot->assign(p->n_curves + 1, 0);
  const int64_t nf = p->n_freq;
  for (int64_t c = 0; c < p->n_curves; ++c) {
    (*curve_slot)[c] = (int32_t)nat->size();
    for (int64_t k0 = 0; k0 < nf;) {
      int64_t k1 = std::min(k0 + chunk, nf);
      if (nf - k1 == 1) k1 = nf;
      fpw::Item it;
      it.curve = (int32_t)c;
      it.k0 = (int32_t)k0;
      it.k1 = (int32_t)k1;
      it.slot = (int32_t)nat->size();
      nat->push_back(it);
      slot_k0->push_back((int32_t)k0);
      k0 = k1;
    }
  }
  (*curve_slot)[p->n_curves] = (int32_t)nat->size();
}

// Queue order: longest curves first (their items take longest), then by curve
// and frequency so neighbouring pops share a curve in cache.
std::vector<fpw::Item> queue_order(const fpw_plan_s* p, const std::vector<fpw::Item>& nat) {
  std::vector<fpw::Item> q = nat;
  const std::vector<int64_t>& off = p->h_offsets;
  std::stable_sort(q.begin(), q.end(), [&](const fpw::Item& a, const fpw::Item& b) {
    const int64_t na = off[a.curve + 1] - off[a.curve], nb = off[b.curve + 1] - off[b.curve];
    if (na != nb) return na > nb;
    if (a.curve != b.curve) return a.curve < b.curve;
    return a.k0 < b.k0;
  });
  return q;
}

int round_up(int64_t v, int64_t m) { return (int)(((v + m - 1) / m) * m); }

// Default chunk: about twelve work items per persistent wave (enough for the
// queue to even out the tail), at least one sweep of the wave, at most 16384
// frequencies.  On mid-size plans that rule makes items so small that the
// queue's atomics (one per item, serialised on one counter) bind instead of
// the folding, so an item also gets at least kMinItemEvalsPerWave,
// unless that would leave consumers without an item.
int default_chunk(const fpw_plan_s* p, const fpw::Shape& s, int total_waves) {
  const int sweep = s.freqs_per_lane * kWave;
  const double per_curve_items = std::max(1.0, 12.0 * total_waves / (double)p->n_curves);
  int64_t chunk = (int64_t)std::ceil((double)p->n_freq / per_curve_items);
  const double points_per_wave = std::max(1.0, (double)p->n_points / p->n_curves / std::max(1, s.share));
  const int64_t pop_floor = (int64_t)std::ceil(kMinItemEvalsPerWave / points_per_wave);
  const int64_t fill_cap = (int64_t)std::ceil((double)p->n_freq * p->n_curves / total_waves);
  chunk = std::max<int64_t>(chunk, std::min(pop_floor, fill_cap));
  chunk = std::max<int64_t>(chunk, sweep);
  chunk = std::min<int64_t>(chunk, 16384);
  return round_up(chunk, sweep);
}

fpw_status configure_shape(fpw_plan_s* p, fpw::Shape s) {
  if (!fpw::batched_shape_built(s, p->opt.phase, p->var.n))
    return fail(FPW_EUNSUPPORTED, "no batched kernel is built for this launch shape");
  const size_t lds = fpw::batched_lds_bytes(s, p->opt.n_bins, p->var.n);
  if (lds > 160 * 1024) return fail(FPW_EUNSUPPORTED, "LDS %zu bytes per workgroup exceeds 160 KiB", lds);
  int per_cu = 0;
  FPW_HIP(fpw::batched_groups_per_cu(s, p->opt.phase, p->opt.topk, p->var.n, lds, &per_cu), "occupancy query");
  if (per_cu < 1) return fail(FPW_EUNSUPPORTED, "batched kernel does not fit on a CU with %zu bytes of LDS", lds);
  p->shape = s;
  p->lds_bytes = lds;
  p->grid_groups = per_cu * p->n_cu;
  // a group of waves sharing a histogram takes one item at a time
  const int consumers = p->grid_groups * (s.share > 1 ? 1 : s.waves_per_group);
  if (s.chunk_freqs <= 0) p->shape.chunk_freqs = default_chunk(p, s, consumers);
  p->shape.chunk_freqs = round_up(p->shape.chunk_freqs, s.freqs_per_lane * kWave);
  return FPW_OK;
}

fpw_status upload_items(fpw_plan_s* p) {
  const int64_t per_curve = (p->n_freq + p->shape.chunk_freqs - 1) / p->shape.chunk_freqs;
  if (per_curve * p->n_curves > (int64_t)INT32_MAX)
    return fail(FPW_EUNSUPPORTED, "%lld work items exceed the 32-bit item index (raise chunk_freqs)",
                (long long)(per_curve * p->n_curves));
  std::vector<fpw::Item> nat;
  std::vector<int32_t> slot_k0, curve_slot;
  build_items(p, p->shape.chunk_freqs, &nat, &slot_k0, &curve_slot);
  // one queue per sum format, each longest curves first
  std::vector<fpw::Item> q, qw;
  for (const fpw::Item& it : queue_order(p, nat))
    (p->n_wide > 0 && p->h_fmt[it.curve] == fpw::FMT_WIDE ? qw : q).push_back(it);
  p->n_items = (int)q.size();
  p->n_items_w = (int)qw.size();
  p->h_items_nat = nat;
  FPW_HIP(p->items.alloc(q.size() * sizeof(fpw::Item)), "alloc items");
  if (!q.empty())
    FPW_HIP(hipMemcpy(p->items.p, q.data(), q.size() * sizeof(fpw::Item), hipMemcpyHostToDevice), "upload items");
  FPW_HIP(p->items_w.alloc(qw.size() * sizeof(fpw::Item)), "alloc wide items");
  if (!qw.empty())
    FPW_HIP(hipMemcpy(p->items_w.p, qw.data(), qw.size() * sizeof(fpw::Item), hipMemcpyHostToDevice),
            "upload wide items");
  FPW_HIP(p->slot_k0.alloc(slot_k0.size() * sizeof(int32_t)), "alloc slot_k0");
  FPW_HIP(hipMemcpy(p->slot_k0.p, slot_k0.data(), slot_k0.size() * sizeof(int32_t), hipMemcpyHostToDevice), "upload slot_k0");
  FPW_HIP(p->curve_slot.alloc(curve_slot.size() * sizeof(int32_t)), "alloc curve_slot");
  FPW_HIP(hipMemcpy(p->curve_slot.p, curve_slot.data(), curve_slot.size() * sizeof(int32_t), hipMemcpyHostToDevice),
          "upload curve_slot");
  if (p->opt.topk > 0) {
    const size_t ns = nat.size() * (size_t)p->var.n;
    FPW_HIP(p->cand_val.alloc(ns * p->opt.topk * sizeof(float)), "alloc cand_val");
    FPW_HIP(p->cand_idx.alloc(ns * p->opt.topk * sizeof(int32_t)), "alloc cand_idx");
    FPW_HIP(p->edge.alloc(ns * 4 * sizeof(float)), "alloc edge");
  }
  // captured passes hold the old buffers: drop them
  p->drop_graphs();
  return FPW_OK;
}

// Persistent workgroups actually launched: never more than the items can keep busy.
int launch_groups(const fpw_plan_s* p, int n_items) {
  const int wpg = p->shape.share > 1 ? 1 : p->shape.waves_per_group;
  const int need = (n_items + wpg - 1) / wpg;
  return std::max(1, std::min(p->grid_groups, need));
}

fpw::BatchArgs batch_args(const fpw_plan_s* p, float* S, const DevBuf& items, int n_items) {
  fpw::BatchArgs a{};
  a.rec = p->rec.as<fpw::Rec>();
  a.offsets = p->offsets.as<int64_t>();
  a.cc = p->cc.as<fpw::CurveConst>();
  a.freqs = p->freqs.as<double>();
  a.items = items.as<fpw::Item>();
  a.n_items = n_items;
  a.n_freq = (int32_t)p->n_freq;
  a.n_bins = p->opt.n_bins;
  a.topk = p->opt.topk;
  a.n_curves = (int32_t)p->n_curves;
  a.var = p->var;
  a.fold_nh = p->fold_nh;
  a.S = S;
  a.cand_val = p->cand_val.as<float>();
  a.cand_idx = p->cand_idx.as<int32_t>();
  a.edge = p->edge.as<float>();
  a.queue = p->queue.as<uint32_t>();
  return a;
}

fpw::PrepArgs prep_args(const fpw_plan_s* p) {
  fpw::PrepArgs a{};
  a.t = p->t.as<double>();
  a.y = p->y.as<double>();
  a.dy = p->dy.as<double>();
  a.offsets = p->offsets.as<int64_t>();
  a.n_curves = p->n_curves;
  a.center = p->opt.center;
  a.tref_mode = p->opt.tref_mode;
  a.phase = p->opt.phase;
  a.t_ref = p->opt.t_ref;
  a.inv_alpha2 = p->opt.inv_alpha2;
  a.stat_scale = p->opt.stat_scale == FPW_STAT_LISTING_HALF ? 0.5f : 1.0f;
  a.rec = p->rec.as<fpw::Rec>();
  a.cc = p->cc.as<fpw::CurveConst>();
  a.tau64 = p->tau64.as<double>();
  a.w64 = p->w64.as<double>();
  a.wx64 = p->wx64.as<double>();
  a.queue = p->queue.as<uint32_t>();
  a.n_queues = p->n_wide > 0 ? 2 : 1;
  if (p->n_wide > 0) {
    a.fmt = p->fmt.as<uint8_t>();
    a.offw = p->offw.as<int64_t>();
    a.recw = p->recw.as<fpw::WRec>();
    a.wc = p->wc.as<fpw::WideConst>();
  }
  return a;
}

// Arguments of the wide-format fold kernel: its own queue and counter.
fpw::BatchArgs wide_args(const fpw_plan_s* p, float* S) {
  fpw::BatchArgs a = batch_args(p, S, p->items_w, p->n_items_w);
  a.queue = p->queue.as<uint32_t>() + 1;
  a.recw = p->recw.as<fpw::WRec>();
  a.offw = p->offw.as<int64_t>();
  a.wc = p->wc.as<fpw::WideConst>();
  return a;
}

fpw::MergeArgs merge_args(const fpw_plan_s* p, int32_t* idx, float* val) {
  fpw::MergeArgs m{};
  m.cand_val = p->cand_val.as<float>();
  m.cand_idx = p->cand_idx.as<int32_t>();
  m.edge = p->edge.as<float>();
  m.slot_k0 = p->slot_k0.as<int32_t>();
  m.curve_slot = p->curve_slot.as<int32_t>();
  m.n_curves = (int32_t)p->n_curves;
  m.n_freq = (int32_t)p->n_freq;
  m.topk = p->opt.topk;
  m.n_var = p->var.n;
  m.out_idx = idx;
  m.out_val = val;
  return m;
}

fpw::SharedPrepArgs shared_prep_args(const fpw_plan_s* p) {
  fpw::SharedPrepArgs a{};
  a.y = p->y.as<double>();
  a.dy = p->dy.as<double>();
  a.n_curves = (int32_t)p->n_curves;
  a.n_points = p->sh_points;
  a.n_kblocks = p->sh_kblocks;
  a.center = p->opt.center;
  a.inv_alpha2 = p->opt.inv_alpha2;
  a.stat_scale = p->opt.stat_scale == FPW_STAT_LISTING_HALF ? 0.5f : 1.0f;
  a.vals = p->sh_vals.as<int8_t>();
  a.cc = p->sh_cc.as<fpw::CurveConst>();
  return a;
}

fpw::SharedArgs shared_args(const fpw_plan_s* p, float* S) {
  fpw::SharedArgs a{};
  a.tau = p->sh_tau.as<double>();
  a.vals = p->sh_vals.as<int8_t>();
  a.cc = p->sh_cc.as<fpw::CurveConst>();
  a.freqs = p->freqs.as<double>();
  a.n_curves = (int32_t)p->n_curves;
  a.n_freq = (int32_t)p->n_freq;
  a.n_bins = p->opt.n_bins;
  a.n_kblocks = p->sh_kblocks;
  a.chunk_kblocks = p->sh_chunk;
  a.fw = p->sh_fw;
  a.rounds = p->sh_rounds;
  a.priv_bytes = p->sh_priv;
  a.fold_nh = p->fold_nh;
  a.S = S;
  return a;
}

// A pass of a shared-timestamp plan on the matrix cores: digits, products,
// then peaks over the stored periodogram.
fpw_status enqueue_shared_pass(fpw_plan_s* p, float* S, int32_t* idx, float* val, hipStream_t s) {
  const bool prof = p->opt.profile != 0;
  float* Sd = S ? S : p->sh_S.as<float>();
  if (prof) FPW_HIP(hipEventRecord(p->ev[0], s), "event record");
  FPW_HIP(fpw::launch_prepare_shared(shared_prep_args(p), s), "shared prepare kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[1], s), "event record");
  FPW_HIP(fpw::launch_shared(shared_args(p, Sd), p->opt.phase, 4, p->sh_nb, p->sh_grid_x, p->sh_grid_y, p->sh_lds, s),
          "shared kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[2], s), "event record");
  if (idx != nullptr) {
    fpw::TopkArgs a{};
    a.S = Sd;
    a.n_curves = (int32_t)p->n_curves;
    a.n_freq = (int32_t)p->n_freq;
    a.k = p->opt.topk;
    a.out_idx = idx;
    a.out_val = val;
    FPW_HIP(fpw::launch_topk(a, s), "top-k kernel");
  }
  if (prof) FPW_HIP(hipEventRecord(p->ev[3], s), "event record");
  p->ev_merge = idx != nullptr;
  return FPW_OK;
}

// A pass with a marginalised baseline: records and constants, the two-sum
// kernel with its FP64 epilogue, then peaks over the stored periodogram.
fpw_status enqueue_bm_pass(fpw_plan_s* p, float* S, int32_t* idx, float* val, hipStream_t s) {
  const bool prof = p->opt.profile != 0;
  float* Sd = S ? S : p->bm_S.as<float>();
  if (prof) FPW_HIP(hipEventRecord(p->ev[0], s), "event record");
  fpw::BmPrepArgs pa{};
  pa.t = p->t.as<double>();
  pa.y = p->y.as<double>();
  pa.dy = p->dy.as<double>();
  pa.offsets = p->offsets.as<int64_t>();
  pa.n_curves = p->n_curves;
  pa.center = p->opt.center;
  pa.tref_mode = p->opt.tref_mode;
  pa.n_terms = p->opt.baseline_terms;
  pa.t_ref = p->opt.t_ref;
  pa.inv_alpha2 = p->opt.inv_alpha2;
  pa.beta = p->opt.baseline_scale;
  pa.stat_scale = p->opt.stat_scale == FPW_STAT_LISTING_HALF ? 0.5 : 1.0;
  pa.rec = p->bm_rec.as<fpw::Rec>();
  pa.z64 = p->bm_z.as<uint64_t>();
  pa.z32 = p->bm_z.as<uint32_t>();
  pa.bc = p->bm_const.as<fpw::BaseConst>();
  pa.queue = p->queue.as<uint32_t>();
  FPW_HIP(fpw::launch_bm_prepare(pa, s), "baseline prepare kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[1], s), "event record");
  fpw::BmArgs a{};
  a.rec = p->bm_rec.as<fpw::Rec>();
  a.z = p->bm_z.p;
  a.offsets = p->offsets.as<int64_t>();
  a.bc = p->bm_const.as<fpw::BaseConst>();
  a.freqs = p->freqs.as<double>();
  a.items = p->items.as<fpw::Item>();
  a.n_items = p->n_items;
  a.n_freq = (int32_t)p->n_freq;
  a.n_bins = p->opt.n_bins;
  a.n_terms = p->opt.baseline_terms;
  a.share = p->bm_share;
  a.source = p->bm_source;
  a.fold_nh = p->fold_nh;
  a.S = Sd;
  a.queue = p->queue.as<uint32_t>();
  FPW_HIP(fpw::launch_bm(a, p->opt.phase, p->bm_grid, s), "baseline kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[2], s), "event record");
  if (idx != nullptr) {
    fpw::TopkArgs t{};
    t.S = Sd;
    t.n_curves = (int32_t)p->n_curves;
    t.n_freq = (int32_t)p->n_freq;
    t.k = p->opt.topk;
    t.out_idx = idx;
    t.out_val = val;
    FPW_HIP(fpw::launch_topk(t, s), "top-k kernel");
  }
  if (prof) FPW_HIP(hipEventRecord(p->ev[3], s), "event record");
  p->ev_merge = idx != nullptr;
  return FPW_OK;
}

fpw::FusedArgs fused_args(const fpw_plan_s* p) {
  fpw::FusedArgs o{};
  o.t = p->t.as<double>();
  o.y = p->y.as<double>();
  o.dy = p->dy.as<double>();
  o.center = p->opt.center;
  o.tref_mode = p->opt.tref_mode;
  o.t_ref = p->opt.t_ref;
  o.inv_alpha2 = p->opt.inv_alpha2;
  o.stat_scale = p->opt.stat_scale == FPW_STAT_LISTING_HALF ? 0.5f : 1.0f;
  return o;
}

// One full pass: prepare, fold/bin/accumulate/reduce (+ fused peaks), merge.
fpw_status enqueue_pass(fpw_plan_s* p, float* S, int32_t* idx, float* val, hipStream_t s) {
  p->ev_wide = false;
  if (p->mfma) return enqueue_shared_pass(p, S, idx, val, s);
  if (p->bm) return enqueue_bm_pass(p, S, idx, val, s);
  const bool prof = p->opt.profile != 0;
  if (p->fused) {
    // prepare runs inside the fold kernel: its time is reported as the batched kernel's
    if (prof) FPW_HIP(hipEventRecord(p->ev[0], s), "event record");
    if (prof) FPW_HIP(hipEventRecord(p->ev[1], s), "event record");
    FPW_HIP(fpw::launch_fused(batch_args(p, S, p->items, p->n_items), fused_args(p), p->opt.phase, s), "fused kernel");
    if (prof) FPW_HIP(hipEventRecord(p->ev[2], s), "event record");
    if (idx != nullptr) FPW_HIP(fpw::launch_merge(merge_args(p, idx, val), s, true), "merge kernel");
    if (prof) FPW_HIP(hipEventRecord(p->ev[3], s), "event record");
    p->ev_merge = idx != nullptr;
    return FPW_OK;
  }
  if (prof) FPW_HIP(hipEventRecord(p->ev[0], s), "event record");
  FPW_HIP(fpw::launch_prepare(prep_args(p), s), "prepare kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[1], s), "event record");
  if (p->n_items > 0)
    FPW_HIP(fpw::launch_batched(batch_args(p, S, p->items, p->n_items), p->shape, p->opt.phase,
                                launch_groups(p, p->n_items), p->lds_bytes, s),
            "batched kernel");
  p->ev_wide = prof && p->n_items_w > 0;
  if (p->ev_wide) FPW_HIP(hipEventRecord(p->ev[4], s), "event record");
  if (p->n_items_w > 0)
    FPW_HIP(fpw::launch_wide(wide_args(p, S), p->opt.phase, p->wide_share, p->wide_grid, s), "wide kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[2], s), "event record");
  // Few periodograms leave most CUs idle during the merge: a workgroup of four
  // waves per periodogram then shortens it (16 curves: 1-2 us less per pass),
  // while from 64 curves on one wave per periodogram is the faster form.
  const bool group_merge = p->n_curves * p->var.n * 8 <= p->n_cu;
  if (idx != nullptr) FPW_HIP(fpw::launch_merge(merge_args(p, idx, val), s, group_merge), "merge kernel");
  if (prof) FPW_HIP(hipEventRecord(p->ev[3], s), "event record");
  p->ev_merge = idx != nullptr;
  return FPW_OK;
}

// ---------------------------------------------------------------- autotuner
std::string tune_key(const fpw_plan_s* p) {
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  const double mean_n = (double)p->n_points / (double)p->n_curves;
  const int nb = (int)std::floor(std::log2(std::max(1.0, mean_n)));
  std::ostringstream k;
  k << arch << "|M=" << p->opt.n_bins << "|phase=" << p->opt.phase << "|topk=" << fpw::topk_capacity(p->opt.topk)
    << "|log2N=" << nb;
  return k.str();
}

// Cache file: one line per key, "key fl waves chunk source share" (a line
// without the share field means private histograms).
bool cache_lookup(const char* path, const std::string& key, fpw::Shape* s) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string k;
    int fl, w, ch, src, sh = 1;
    if (!(in >> k >> fl >> w >> ch >> src) || k != key) continue;
    if (!(in >> sh)) sh = 1;
    s->freqs_per_lane = fl;
    s->waves_per_group = w;
    s->chunk_freqs = ch;
    s->point_source = src;
    s->share = sh;
    return true;
  }
  return false;
}

void cache_store(const char* path, const std::string& key, const fpw::Shape& s) {
  if (!path) return;
  std::map<std::string, std::string> lines;
  {
    std::ifstream f(path);
    std::string k, rest;
    while (f >> k && std::getline(f, rest)) lines[k] = rest;
  }
  std::ostringstream v;
  v << " " << s.freqs_per_lane << " " << s.waves_per_group << " " << s.chunk_freqs << " " << s.point_source << " "
    << s.share;
  lines[key] = v.str();
  std::ofstream f(path, std::ios::trunc);
  for (auto& kv : lines) f << kv.first << kv.second << "\n";
}

// Times each candidate shape on a calibration slice (every stride-th curve)
// and keeps the fastest.
fpw_status autotune(fpw_plan_s* p, hipStream_t s) {
  const std::string key = tune_key(p);
  fpw::Shape best{};
  if (cache_lookup(p->opt.tune_cache, key, &best)) {
    fpw_status st = configure_shape(p, best);
    if (st == FPW_OK) {
      p->tuned = true;
      return FPW_OK;
    }
  }
  std::vector<fpw::Shape> cands;
  const int fls = (p->opt.phase <= FPW_PHASE_FP64_LISTING && p->var.n == 1) ? 2 : 1;
  for (int src = 0; src <= 1; ++src)
    for (int fl = 1; fl <= (src == 1 ? 1 : fls); ++fl)
      for (int w : {1, 2})
        for (int cm : {1, 4}) cands.push_back(fpw::Shape{fl, w, -cm, src, 1});
  // histograms shared by 2 or 4 waves (with the FP32-based folds: one variant)
  if (p->opt.phase <= FPW_PHASE_FP64_LISTING || p->var.n == 1)
    for (int src = 0; src <= 1; ++src)
      for (int sh : {2, 4}) cands.push_back(fpw::Shape{1, sh, -1, src, sh});
  // calibration slice: about 2e9 evaluations
  const double target = 2e9;
  const double per_curve = (double)p->n_points / p->n_curves * (double)p->n_freq;
  const int64_t want = std::max<int64_t>(1, (int64_t)(target / std::max(1.0, per_curve)));
  const int64_t stride = std::max<int64_t>(1, p->n_curves / want);
  hipEvent_t e0, e1;
  FPW_HIP(hipEventCreate(&e0), "event");
  FPW_HIP(hipEventCreate(&e1), "event");
  double best_t = INFINITY;
  fpw::Shape best_s = p->shape;
  for (const fpw::Shape& c0 : cands) {
    fpw::Shape c = c0;
    c.chunk_freqs = 0;
    if (configure_shape(p, c) != FPW_OK) continue;
    if (c0.chunk_freqs == -4) p->shape.chunk_freqs = round_up(std::min<int64_t>(p->n_freq, 4 * (int64_t)p->shape.chunk_freqs), c.freqs_per_lane * kWave);
    std::vector<fpw::Item> nat;
    std::vector<int32_t> sk, cs;
    build_items(p, p->shape.chunk_freqs, &nat, &sk, &cs);
    std::vector<fpw::Item> q;
    for (const fpw::Item& it : queue_order(p, nat))
      if (it.curve % stride == 0 && (p->n_wide == 0 || p->h_fmt[it.curve] == fpw::FMT_NARROW)) q.push_back(it);
    if (q.empty()) continue;
    DevBuf items;
    FPW_HIP(items.alloc(q.size() * sizeof(fpw::Item)), "alloc tune items");
    FPW_HIP(hipMemcpy(items.p, q.data(), q.size() * sizeof(fpw::Item), hipMemcpyHostToDevice), "upload tune items");
    // candidate scratch sized for this chunking
    DevBuf cv, ci, ed;
    fpw::BatchArgs a = batch_args(p, nullptr, items, (int)q.size());
    if (p->opt.topk > 0) {
      const size_t ns = nat.size() * (size_t)p->var.n;
      FPW_HIP(cv.alloc(ns * p->opt.topk * sizeof(float)), "alloc");
      FPW_HIP(ci.alloc(ns * p->opt.topk * sizeof(int32_t)), "alloc");
      FPW_HIP(ed.alloc(ns * 4 * sizeof(float)), "alloc");
      a.cand_val = cv.as<float>();
      a.cand_idx = ci.as<int32_t>();
      a.edge = ed.as<float>();
    }
    double tmin = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {
      FPW_HIP(hipMemsetAsync(p->queue.p, 0, sizeof(uint32_t), s), "clear queue");  // (no prepare kernel runs here)
      FPW_HIP(hipEventRecord(e0, s), "event");
      FPW_HIP(fpw::launch_batched(a, p->shape, p->opt.phase, launch_groups(p, (int)q.size()), p->lds_bytes, s),
              "tune launch");
      FPW_HIP(hipEventRecord(e1, s), "event");
      FPW_HIP(hipEventSynchronize(e1), "event sync");
      float ms = 0;
      FPW_HIP(hipEventElapsedTime(&ms, e0, e1), "event time");
      if (rep > 0) tmin = std::min(tmin, (double)ms);
    }
    if (tmin < best_t) {
      best_t = tmin;
      best_s = p->shape;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  fpw_status st = configure_shape(p, best_s);
  if (st != FPW_OK) return st;
  p->tuned = true;
  cache_store(p->opt.tune_cache, key, p->shape);
  return FPW_OK;
}

// Which wave of a histogram shared by 2 or 4 waves computes (and keeps the
// S and peaks of) each derived variant: of all assignments of variants
// 1..n-1 to the waves, at most as many per wave as the kernel has register
// slots for (ceil((NV - 1) / SH) for its NV = 4 or 8), the one whose busiest
// wave has the least work, counted as the variant's coarse bins plus a
// fixed cost for its set-up, store and peak step; wave 0 also stores and
// keeps variant 0.  At most 4^7 assignments: exhaustive search.  False if
// no assignment fits the slots (not reachable with at most kMaxVariants
// variants, but checked rather than assumed).
bool assign_variant_waves(fpw::Variants& var, int M) {
  constexpr int kPerVariant = 5, kLeadExtra = 5;
  std::memset(var.own, 0, sizeof(var.own));
  const int nd = var.n - 1;
  if (nd <= 0) return true;
  const int nv_inst = var.n <= 4 ? 4 : fpw::kMaxVariants;
  for (int s = 0; s < 2; ++s) {
    const int sh = s == 0 ? 2 : 4;
    const int cap = (nv_inst - 1 + sh - 1) / sh;
    int n_assign = 1;
    for (int d = 0; d < nd; ++d) n_assign *= sh;
    int best = -1, best_cost = INT_MAX;
    for (int code = 0; code < n_assign; ++code) {
      int load[4] = {kLeadExtra, 0, 0, 0}, count[4] = {0, 0, 0, 0};
      bool ok = true;
      for (int d = 0, c = code; d < nd; ++d, c /= sh) {
        const int w = c % sh;
        load[w] += M / var.k[d + 1] + kPerVariant;
        ok = ok && ++count[w] <= cap;
      }
      if (!ok) continue;
      const int cost = *std::max_element(load, load + sh);
      if (cost < best_cost) {
        best_cost = cost;
        best = code;
      }
    }
    if (best < 0) return false;
    int count[4] = {0, 0, 0, 0};
    for (int d = 0, c = best; d < nd; ++d, c /= sh) {
      const int w = c % sh;
      var.own[s][w][count[w]++] = (int8_t)(d + 1);
    }
  }
  return true;
}

template <class T>
fpw_status upload(DevBuf& b, const T* src, size_t n, hipStream_t s, const char* what) {
  FPW_HIP(b.alloc(n * sizeof(T)), what);
  if (n) FPW_HIP(hipMemcpyAsync(b.p, src, n * sizeof(T), hipMemcpyHostToDevice, s), what);
  return FPW_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

void fpw_options_default(fpw_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n_bins = 10;
  o->center = FPW_CENTER_WEIGHTED;
  o->tref_mode = FPW_TREF_ZERO;
  o->phase = FPW_PHASE_FP64;
  o->stat_scale = FPW_STAT_EQ1;
  o->topk = 0;
  o->inv_alpha2 = 0.0;
  o->t_ref = 0.0;
  o->autotune = 0;
  o->use_graph = 1;
  o->tune_cache = nullptr;
  o->baseline_terms = 0;
  o->baseline_scale = 1.0;
}

const char* fpw_last_error(void) { return g_err.c_str(); }

const char* fpw_version(void) { return "fpw 0.1.0 gfx950"; }

fpw_status fpw_plan(fpw_plan_t* out, int64_t n_curves, const int64_t* offsets, const double* t, const double* y,
                    const double* dy, int64_t n_freq, const double* freqs, const fpw_options* opt, void* stream) {
  g_err.clear();
  if (!out) return fail(FPW_EINVAL, "out is NULL");
  *out = nullptr;
  fpw_options o;
  fpw_options_default(&o);
  if (opt) o = *opt;
  fpw_status st = check_options(o);
  if (st != FPW_OK) return st;
  double max_tau = 0, max_f = 0;
  st = validate(n_curves, offsets, t, y, dy, n_freq, freqs, o, &max_tau, &max_f);
  if (st != FPW_OK) return st;
  bool fused_fold = true;
  const double fold_nh = fused_fold_shift(o.n_bins, max_tau * max_f, &fused_fold);
  if (o.phase == FPW_PHASE_FP64 && !fused_fold) o.phase = FPW_PHASE_FP64_LISTING;
  int n_var = 1;
  for (int d = 0; d < FPW_MAX_DERIVED && o.derived_bins[d] != 0; ++d) n_var += o.all_offsets ? o.n_bins / o.derived_bins[d] : 1;
  std::vector<uint8_t> fmt;
  int64_t n_wide = 0;
  try {
    st = choose_formats(n_curves, offsets, y, dy, o, n_var, &fmt, &n_wide);
  } catch (const std::bad_alloc&) {
    return fail(FPW_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(FPW_EHIP, "unexpected exception");
  }
  if (st != FPW_OK) return st;
  // ---- all checks passed: from here on HIP calls are made
  try {
    fpw_plan_s* p = new fpw_plan_s();
    std::unique_ptr<fpw_plan_s> guard(p);
    p->opt = o;
    p->fold_nh = fold_nh;
    p->fused_fold = fused_fold;
    p->h_fmt.swap(fmt);
    p->n_wide = n_wide;
    p->n_curves = n_curves;
    p->n_freq = n_freq;
    p->n_points = offsets[n_curves];
    p->h_offsets.assign(offsets, offsets + n_curves + 1);
    // variant 0: the fine binning; then each derived M' with its offsets
    p->var.n = 1;
    p->var.k[0] = 1;
    p->var.o[0] = 0;
    p->var_bins.assign(1, o.n_bins);
    for (int d = 0; d < FPW_MAX_DERIVED && o.derived_bins[d] != 0; ++d) {
      const int k = o.n_bins / o.derived_bins[d];
      for (int off = 0; off < (o.all_offsets ? k : 1); ++off) {
        p->var.k[p->var.n] = k;
        p->var.o[p->var.n] = off;
        p->var_bins.push_back(o.derived_bins[d]);
        ++p->var.n;
      }
    }
    // prefix slots the derived variants read: window ends x - 1 (and o - 1)
    for (int v = 1; v < p->var.n; ++v) {
      const int k = p->var.k[v], off = p->var.o[v], M = o.n_bins;
      for (int c = 0; c < M / k; ++c) {
        const int e = off + (c + 1) * k;
        const int slot = (e > M ? e - M : e) - 1;
        p->var.need[slot >> 5] |= 1u << (slot & 31);
      }
    }
    if (!assign_variant_waves(p->var, o.n_bins))
      return fail(FPW_EUNSUPPORTED, "%d periodogram variants do not fit the kernels' register slots", p->var.n);
    hipStream_t s = (hipStream_t)stream;
    FPW_HIP(hipGetDevice(&p->device), "hipGetDevice");
    FPW_HIP(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device), "CU count");
    const size_t np = (size_t)p->n_points;
    st = upload(p->t, t, np, s, "upload t");
    if (st == FPW_OK) st = upload(p->y, y, np, s, "upload y");
    if (st == FPW_OK) st = upload(p->dy, dy, np, s, "upload dy");
    if (st == FPW_OK) st = upload(p->offsets, offsets, (size_t)n_curves + 1, s, "upload offsets");
    if (st == FPW_OK) st = upload(p->freqs, freqs, (size_t)n_freq, s, "upload freqs");
    if (st != FPW_OK) return st;
    FPW_HIP(p->rec.alloc(np * sizeof(fpw::Rec)), "alloc records");
    FPW_HIP(p->cc.alloc((size_t)n_curves * sizeof(fpw::CurveConst)), "alloc curve constants");
    FPW_HIP(p->tau64.alloc(np * sizeof(double)), "alloc tau64");
    FPW_HIP(p->w64.alloc(np * sizeof(double)), "alloc w64");
    FPW_HIP(p->wx64.alloc(np * sizeof(double)), "alloc wx64");
    if (o.profile)
      for (hipEvent_t& e : p->ev) FPW_HIP(hipEventCreate(&e), "event create");
    // one counter per fold kernel: the batched one, then the wide-format one
    FPW_HIP(p->queue.alloc(2 * sizeof(uint32_t)), "alloc queue");
    FPW_HIP(hipMemsetAsync(p->queue.p, 0, 2 * sizeof(uint32_t), s), "clear queue");
    if (p->n_wide > 0) {
      // wide records: the wide curves' points, packed in curve order
      p->h_offw.assign((size_t)n_curves + 1, 0);
      for (int64_t c = 0; c < n_curves; ++c)
        p->h_offw[(size_t)c + 1] = p->h_offw[(size_t)c] + (p->h_fmt[(size_t)c] == fpw::FMT_WIDE ? offsets[c + 1] - offsets[c] : 0);
      st = upload(p->fmt, p->h_fmt.data(), p->h_fmt.size(), s, "upload formats");
      if (st == FPW_OK) st = upload(p->offw, p->h_offw.data(), p->h_offw.size(), s, "upload wide offsets");
      if (st != FPW_OK) return st;
      FPW_HIP(p->recw.alloc((size_t)p->h_offw[(size_t)n_curves] * sizeof(fpw::WRec)), "alloc wide records");
      FPW_HIP(p->wc.alloc((size_t)n_curves * sizeof(fpw::WideConst)), "alloc wide constants");
    }
    // prepared records are needed by autotune, fpw_eval_fp64 and fpw_debug_bins
    FPW_HIP(fpw::launch_prepare(prep_args(p), s), "prepare kernel");
    // Large M leaves room for few waves per CU; their scalar-load waits then
    // stall the LDS atomics, so the DPP broadcast source is the default there.
    int share = o.hist_share;
    if (share == 0) {  // by M, where a shared histogram is built and no other group shape was asked for
      const bool can = (o.phase <= FPW_PHASE_FP64_LISTING || p->var.n == 1) && o.freqs_per_lane != 2 &&
                       o.waves_per_group == 0;
      share = !can ? 1 : (o.n_bins >= kShare4MinBins ? 4 : (o.n_bins >= kShare2MinBins ? 2 : 1));
      if (share == 2 && p->var.n == 1 && (double)np * (double)n_freq < kShare4SmallPlanEvalsPerCu * p->n_cu) share = 4;
    }
    // with more than four variants (the 8-variant kernel) the DPP broadcast wins even with
    // shared histograms (M = 40 -> 20, 10 at every offset, four waves per histogram: 2.90
    // against 2.95 s on the uneven batch, a tie on the ZTF-like one); with up to four the
    // scalar source does (offset 0 only: 2.35 against 2.37 s, 14.0 against 14.6 ms)
    const int dpp_from = share > 1 && p->var.n <= 4 ? kDppMinBinsShared : kDppMinBins;
    const int src = o.point_source ? o.point_source - 1 : (o.n_bins >= dpp_from ? 1 : 0);
    const int fl = (src == 1 || p->var.n > 1 || share > 1) ? 1 : (o.freqs_per_lane ? o.freqs_per_lane : 1);
    const int wpg = share > 1 ? share : (o.waves_per_group ? o.waves_per_group : 1);
    fpw::Shape sh{fl, wpg, o.chunk_freqs, src, share};
    // The fused pass for small plans (at most kFusedItemsPerCu items of 64
    // frequencies per CU) unless a launch shape or its tuning was asked for.
    const int64_t items64 = n_curves * ((n_freq + kWave - 1) / kWave);
    const bool overrides = o.freqs_per_lane || o.waves_per_group || o.chunk_freqs || o.point_source || o.hist_share;
    const bool fused_ok = p->var.n == 1 && o.baseline_terms == 0 && p->n_wide == 0 &&
                          fpw::fused_lds_bytes(o.n_bins) + 1024 <= (size_t)160 * 1024;
    p->fused = fused_ok && (o.fuse_prepare == 1 || (o.fuse_prepare == 0 && !overrides && !o.autotune &&
                                                    items64 <= (int64_t)kFusedItemsPerCu * p->n_cu));
    if (p->fused) {
      // items of 64 frequencies, or longer ones where a forced plan would exceed the per-CU budget
      const int64_t budget = (int64_t)kFusedItemsPerCu * p->n_cu;
      const int64_t per_curve = std::max<int64_t>(1, budget / n_curves);
      int64_t chunk = o.chunk_freqs ? o.chunk_freqs : (n_freq + per_curve - 1) / per_curve;
      chunk = std::min<int64_t>(std::max<int64_t>(chunk, kWave), std::max<int64_t>(n_freq, kWave));
      p->shape = fpw::Shape{1, fpw::fused_waves(), round_up(chunk, kWave), 0, fpw::fused_waves()};
      p->lds_bytes = fpw::fused_lds_bytes(o.n_bins);
      st = FPW_OK;
    } else if (o.autotune && !overrides) {
      st = autotune(p, s);
    } else {
      st = configure_shape(p, sh);
    }
    if (st != FPW_OK) return st;
    st = upload_items(p);
    if (st != FPW_OK) return st;
    if (p->fused) p->grid_groups = p->n_items;
    if (p->n_items_w > 0) {
      // wide histograms take 16 bytes per bin and lane: shared by two waves
      // from 8 bins, by four from 16
      const int M = o.n_bins;
      p->wide_share = M < 8 ? 1 : (M < 16 ? 2 : 4);
      int per_cu = 0;
      FPW_HIP(fpw::wide_groups_per_cu(o.phase, o.topk, M, p->wide_share, &per_cu), "wide kernel occupancy");
      p->wide_grid = std::max(1, std::min(std::max(1, per_cu) * p->n_cu, p->n_items_w));
    }
    if (o.baseline_terms > 0) {
      p->bm = true;
      FPW_HIP(p->bm_rec.alloc(np * sizeof(fpw::Rec)), "alloc baseline records");
      const size_t zb = o.baseline_terms >= 3 ? sizeof(uint64_t) : (o.baseline_terms == 2 ? sizeof(uint32_t) : 0);
      FPW_HIP(p->bm_z.alloc(std::max<size_t>(np * zb, 8)), "alloc baseline sums");
      FPW_HIP(p->bm_const.alloc((size_t)n_curves * sizeof(fpw::BaseConst)), "alloc baseline constants");
      FPW_HIP(p->bm_S.alloc((size_t)n_curves * (size_t)n_freq * sizeof(float)), "alloc baseline periodogram");
      int per_cu = 0;
      // histograms of ~8.5 KiB or more per wave are shared by two waves, from 12 KiB by four (measured
      // at M = 20: K = 1, 10.5 KiB, two waves 2 % faster than four; K = 2, 3, 16 and 21 KiB, four
      // waves faster than two by 2 and 6 %; private ones slowest every time); scalar point loads
      // unless asked otherwise
      const size_t hb = fpw::bm_lds_bytes(o.n_bins, o.baseline_terms, 1);
      p->bm_share = o.hist_share ? o.hist_share : (hb >= 12288 ? 4 : (hb >= 8704 ? 2 : 1));
      p->bm_source = o.point_source == 2 ? 1 : 0;
      FPW_HIP(fpw::bm_groups_per_cu(o.phase, o.n_bins, o.baseline_terms, p->bm_share, p->bm_source, &per_cu),
              "baseline kernel occupancy");
      p->bm_grid = std::max(1, std::min(std::max(1, per_cu) * p->n_cu, p->n_items));
    }
    FPW_HIP(hipStreamSynchronize(s), "plan sync");
    *out = guard.release();
    return FPW_OK;
  } catch (const std::bad_alloc&) {
    return fail(FPW_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(FPW_EHIP, "unexpected exception");
  }
}

fpw_status fpw_plan_shared(fpw_plan_t* out, int64_t n_curves, int64_t n_points, const double* t, const double* y,
                           const double* dy, int64_t n_freq, const double* freqs, const fpw_options* opt,
                           void* stream) {
  g_err.clear();
  if (!out) return fail(FPW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!t || !y || !dy || !freqs) return fail(FPW_EINVAL, "null input pointer");
  if (n_curves < 1) return fail(FPW_EINVAL, "n_curves must be >= 1");
  if (n_points < 1) return fail(FPW_EINVAL, "n_points must be >= 1");
  if (n_points > FPW_MAX_CURVE_POINTS) return fail(FPW_EUNSUPPORTED, "n_points %lld > %d", (long long)n_points, FPW_MAX_CURVE_POINTS);
  if (n_curves > (int64_t)INT32_MAX / n_points) return fail(FPW_EUNSUPPORTED, "n_curves * n_points too large");
  fpw_options o;
  fpw_options_default(&o);
  if (opt) o = *opt;
  fpw_status st = check_options(o);
  if (st != FPW_OK) return st;
  const bool fits = o.n_bins <= fpw::kSharedMaxBins && (o.phase == FPW_PHASE_FP64 || o.phase == FPW_PHASE_FP64_LISTING) &&
                    o.derived_bins[0] == 0 && o.baseline_terms == 0 && (n_curves + 15) / 16 <= 65535 &&
                    n_points <= fpw::kSharedMaxPoints;
  if (o.shared_kernel == FPW_SHARED_MATRIX && !fits)
    return fail(FPW_EUNSUPPORTED, "the matrix-core kernel needs n_bins <= %d, phase FP64 or FP64_LISTING, no derived bin "
                "counts, no baseline terms, at most 1048560 curves and %d points", fpw::kSharedMaxBins, fpw::kSharedMaxPoints);
  // the matrix-core kernel's sums have 30-bit fields: every curve must fit the
  // narrow bounds there (else the general kernel takes the plan, or, when the
  // matrix-core kernel was asked for, the plan is refused)
  bool digits_fit = o.sum_format == FPW_SUMS_AUTO;
  if (fits && digits_fit && o.shared_kernel != FPW_SHARED_GENERAL) {
    bool finite_ok = true;
    for (int64_t i = 0; i < n_curves * n_points && finite_ok; ++i)
      finite_ok = std::isfinite(y[i]) && std::isfinite(dy[i]) && dy[i] > 0 && 1.0 / (dy[i] * dy[i]) >= DBL_MIN &&
                  1.0 / (dy[i] * dy[i]) <= DBL_MAX;
    if (finite_ok) {  // (otherwise fpw_plan below reports the input)
      try {
        CurveWeights cw;
        const double nd = (double)n_points;
        for (int64_t c = 0; c < n_curves && digits_fit; ++c) {
          SumBounds b;
          curve_weights(y + c * n_points, dy + c * n_points, n_points, o.center, &cw);
          digits_fit = std::isfinite(cw.sw) && std::isfinite(cw.a) &&
                       narrow_fits(cw, o.n_bins, o.inv_alpha2, 1073741824.0 - 2.0 - 2.0 * nd, 1073741824.0 - 2.0 - nd, &b);
        }
      } catch (const std::bad_alloc&) {
        return fail(FPW_ENOMEM, "host allocation failed");
      }
    }
  }
  if (o.shared_kernel == FPW_SHARED_MATRIX && !digits_fit)
    return fail(FPW_EUNSUPPORTED, "a curve's weights span too wide a range for the matrix-core kernel's 30-bit sums "
                "(or sum_format asks for the wide format)");
  const bool mfma = fits && digits_fit && o.shared_kernel != FPW_SHARED_GENERAL;
  try {
    // the equivalent CSR batch: every curve holds the common times
    std::vector<int64_t> offs((size_t)n_curves + 1);
    for (int64_t c = 0; c <= n_curves; ++c) offs[(size_t)c] = c * n_points;
    std::vector<double> tt((size_t)(n_curves * n_points));
    for (int64_t c = 0; c < n_curves; ++c) std::memcpy(&tt[(size_t)(c * n_points)], t, (size_t)n_points * sizeof(double));
    fpw_plan_t raw = nullptr;
    st = fpw_plan(&raw, n_curves, offs.data(), tt.data(), y, dy, n_freq, freqs, &o, stream);
    if (st != FPW_OK) return st;
    std::unique_ptr<fpw_plan_s> guard(raw);
    fpw_plan_s* p = raw;
    if (mfma) {
      hipStream_t s = (hipStream_t)stream;
      const int M = o.n_bins;
      p->mfma = true;
      p->sh_points = (int32_t)n_points;
      p->sh_kblocks = (int32_t)((n_points + 31) / 32);
      p->sh_chunk = std::min(p->sh_kblocks, 16);
      fpw::shared_shape(M, &p->sh_nb, &p->sh_fw);
      const int term_bytes = 4 * 4 * (32 * p->sh_nb + 1) * (int)sizeof(float);
      p->sh_priv = round_up(std::max(p->sh_fw * p->sh_chunk * 32, term_bytes), 16);
      p->sh_lds = (size_t)4 * p->sh_chunk * fpw::kSharedTileBytes + (size_t)fpw::kSharedWaves * p->sh_priv;
      const int64_t nfb = (n_freq + p->sh_fw - 1) / p->sh_fw;        // frequency blocks
      const int64_t wrounds = (nfb + fpw::kSharedWaves - 1) / fpw::kSharedWaves;
      p->sh_grid_y = (int)((n_curves + 15) / 16);
      p->sh_rounds = (int)std::max<int64_t>(1, std::min<int64_t>(32, (int64_t)p->sh_grid_y * wrounds / 2048));
      p->sh_grid_x = (int)((wrounds + p->sh_rounds - 1) / p->sh_rounds);
      const int64_t groups = (int64_t)p->sh_grid_y * 4;
      // the common time offsets, formed once in FP64 as for every curve
      double tmin = t[0];
      for (int64_t i = 1; i < n_points; ++i) tmin = std::min(tmin, t[i]);
      const double tref = o.tref_mode == FPW_TREF_ZERO ? 0.0 : (o.tref_mode == FPW_TREF_FIRST ? tmin : o.t_ref);
      std::vector<double> tau((size_t)p->sh_kblocks * 32, 0.0);
      for (int64_t i = 0; i < n_points; ++i) tau[(size_t)i] = t[i] - tref;
      st = upload(p->sh_tau, tau.data(), tau.size(), s, "upload shared tau");
      if (st != FPW_OK) return st;
      const size_t vbytes = (size_t)groups * p->sh_kblocks * fpw::kSharedTileBytes;
      FPW_HIP(p->sh_vals.alloc(vbytes), "alloc digit tiles");
      FPW_HIP(hipMemsetAsync(p->sh_vals.p, 0, vbytes, s), "clear digit tiles");
      FPW_HIP(p->sh_cc.alloc((size_t)groups * 4 * sizeof(fpw::CurveConst)), "alloc shared constants");
      FPW_HIP(hipMemsetAsync(p->sh_cc.p, 0, p->sh_cc.bytes, s), "clear shared constants");
      FPW_HIP(p->sh_S.alloc((size_t)n_curves * (size_t)n_freq * sizeof(float)), "alloc shared periodogram");
      FPW_HIP(hipStreamSynchronize(s), "shared plan sync");
    }
    *out = guard.release();
    return FPW_OK;
  } catch (const std::bad_alloc&) {
    return fail(FPW_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(FPW_EHIP, "unexpected exception");
  }
}

fpw_status fpw_eval_batch(fpw_plan_t p, float* S_dev, int32_t* topk_idx, float* topk_val, void* stream) {
  g_err.clear();
  if (!p) return fail(FPW_EINVAL, "plan is NULL");
  if ((topk_idx == nullptr) != (topk_val == nullptr)) return fail(FPW_EINVAL, "topk_idx and topk_val must both be set or both NULL");
  if (topk_idx && p->opt.topk <= 0) return fail(FPW_EINVAL, "plan was made with topk = 0");
  hipStream_t s = (hipStream_t)stream;
  try {
    // Profiling records plain stream events, so a profiled pass is launched
    // directly rather than replayed from the graph.
    if (p->opt.use_graph && p->graph_ok && !p->opt.profile && !p->fused) {
      fpw_plan_s::Graph* hit = nullptr;
      for (fpw_plan_s::Graph& e : p->graphs)
        if (e.S == S_dev && e.idx == topk_idx && e.val == topk_val) hit = &e;
      if (!hit) {
        if (p->graphs.size() >= fpw_plan_s::kMaxGraphs) {
          auto lru = p->graphs.begin();
          for (auto it = p->graphs.begin(); it != p->graphs.end(); ++it)
            if (it->used < lru->used) lru = it;
          (void)hipGraphExecDestroy(lru->x);
          (void)hipGraphDestroy(lru->g);
          p->graphs.erase(lru);
        }
        if (!p->cap_stream) FPW_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capture stream");
        bool ok = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        fpw_status st = FPW_OK;
        if (ok) st = enqueue_pass(p, S_dev, topk_idx, topk_val, p->cap_stream);
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        const bool ended = ok && hipStreamEndCapture(p->cap_stream, &g) == hipSuccess && g != nullptr;
        if (ended && st == FPW_OK && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) {
          p->graphs.push_back({S_dev, topk_idx, topk_val, g, x, 0});
          hit = &p->graphs.back();
        } else {
          if (g) (void)hipGraphDestroy(g);
          p->graph_ok = false;  // fall back to direct launches from now on
          (void)hipGetLastError();
        }
      }
      if (hit) {
        hit->used = ++p->graph_clock;
        FPW_HIP(hipGraphLaunch(hit->x, s), "graph launch");
        p->ev_recorded = false;
        return FPW_OK;
      }
    }
    fpw_status st = enqueue_pass(p, S_dev, topk_idx, topk_val, s);
    p->ev_recorded = st == FPW_OK && p->opt.profile != 0;
    return st;
  } catch (...) {
    return fail(FPW_EHIP, "unexpected exception");
  }
}

fpw_status fpw_topk(fpw_plan_t p, const float* S_dev, int32_t k, int32_t* idx_dev, float* val_dev, void* stream) {
  g_err.clear();
  if (!p) return fail(FPW_EINVAL, "plan is NULL");
  if (!S_dev || !idx_dev || !val_dev) return fail(FPW_EINVAL, "null device pointer");
  if (k < 1 || k > p->n_freq) return fail(FPW_EINVAL, "k must be in [1, n_freq]");
  if (k > FPW_MAX_TOPK) return fail(FPW_EUNSUPPORTED, "k %d exceeds FPW_MAX_TOPK=%d", k, FPW_MAX_TOPK);
  fpw::TopkArgs a{};
  a.S = S_dev;
  a.n_curves = (int32_t)p->n_curves;
  a.n_freq = (int32_t)p->n_freq;
  a.k = k;
  a.out_idx = idx_dev;
  a.out_val = val_dev;
  FPW_HIP(fpw::launch_topk(a, (hipStream_t)stream), "top-k kernel");
  return FPW_OK;
}

fpw_status fpw_eval_fp64(fpw_plan_t p, double* S_dev, void* stream) {
  g_err.clear();
  if (!p) return fail(FPW_EINVAL, "plan is NULL");
  if (!S_dev) return fail(FPW_EINVAL, "S_dev is NULL");
  if (p->bm) return fail(FPW_EUNSUPPORTED, "the FP64 comparator evaluates Eq. 1 only (the plan has baseline terms)");
  if ((size_t)2 * p->opt.n_bins * kWave * sizeof(double) > 160 * 1024)
    return fail(FPW_EUNSUPPORTED, "the FP64 comparator holds 2*M doubles per lane in LDS: M <= 160");
  hipStream_t s = (hipStream_t)stream;
  FPW_HIP(fpw::launch_prepare(prep_args(p), s), "prepare kernel");
  for (int64_t c = 0; c < p->n_curves; ++c) {
    fpw::Fp64Args a{};
    a.tau = p->tau64.as<double>();
    a.w = p->w64.as<double>();
    a.wx = p->wx64.as<double>();
    a.freqs = p->freqs.as<double>();
    a.p0 = p->h_offsets[c];
    a.n = (int32_t)(p->h_offsets[c + 1] - p->h_offsets[c]);
    a.n_freq = (int32_t)p->n_freq;
    a.n_bins = p->opt.n_bins;
    a.inv_alpha2 = p->opt.inv_alpha2;
    a.scale = p->opt.stat_scale == FPW_STAT_LISTING_HALF ? 0.5 : 1.0;
    a.S = S_dev + c * p->n_freq;
    FPW_HIP(fpw::launch_fp64(a, s), "fp64 kernel");
  }
  return FPW_OK;
}

fpw_status fpw_debug_bins(fpw_plan_t p, int32_t phase, int64_t curve, int64_t f_begin, int64_t f_end, int32_t* bins_dev,
                          void* stream) {
  g_err.clear();
  if (!p) return fail(FPW_EINVAL, "plan is NULL");
  if (!bins_dev) return fail(FPW_EINVAL, "bins_dev is NULL");
  if (phase < 0 || phase > 3) return fail(FPW_EINVAL, "bad phase mode %d", phase);
  if (curve < 0 || curve >= p->n_curves) return fail(FPW_EINVAL, "curve out of range");
  if (f_begin < 0 || f_end > p->n_freq || f_begin >= f_end) return fail(FPW_EINVAL, "bad frequency range");
  fpw::BinsArgs a{};
  a.rec = p->rec.as<fpw::Rec>();
  a.tau64 = p->tau64.as<double>();
  a.freqs = p->freqs.as<double>();
  a.p0 = p->h_offsets[curve];
  a.n = (int32_t)(p->h_offsets[curve + 1] - p->h_offsets[curve]);
  a.f_begin = (int32_t)f_begin;
  a.f_end = (int32_t)f_end;
  a.n_bins = p->opt.n_bins;
  // FP64 on a plan whose fold range made it fold in the listing order
  a.phase = phase == FPW_PHASE_FP64 && !p->fused_fold ? FPW_PHASE_FP64_LISTING : phase;
  a.fold_nh = p->fold_nh;
  a.out = bins_dev;
  FPW_HIP(fpw::launch_bins(a, (hipStream_t)stream), "bins kernel");
  return FPW_OK;
}

fpw_status fpw_pass_timings(fpw_plan_t p, float ms[3]) {
  g_err.clear();
  if (!p || !ms) return fail(FPW_EINVAL, "NULL argument");
  if (!p->opt.profile) return fail(FPW_ESTATE, "plan was made with profile = 0");
  if (!p->ev_recorded) return fail(FPW_ESTATE, "no fpw_eval_batch has run on this plan");
  FPW_HIP(hipEventSynchronize(p->ev[3]), "event sync");
  FPW_HIP(hipEventElapsedTime(&ms[0], p->ev[0], p->ev[1]), "event time");
  FPW_HIP(hipEventElapsedTime(&ms[1], p->ev[1], p->ev[2]), "event time");
  if (p->ev_merge) {
    FPW_HIP(hipEventElapsedTime(&ms[2], p->ev[2], p->ev[3]), "event time");
  } else {
    ms[2] = 0.f;
  }
  return FPW_OK;
}

fpw_status fpw_pass_wide_ms(fpw_plan_t p, float* ms) {
  g_err.clear();
  if (!p || !ms) return fail(FPW_EINVAL, "NULL argument");
  if (!p->opt.profile) return fail(FPW_ESTATE, "plan was made with profile = 0");
  if (!p->ev_recorded) return fail(FPW_ESTATE, "no fpw_eval_batch has run on this plan");
  *ms = 0.f;
  if (!p->ev_wide) return FPW_OK;
  FPW_HIP(hipEventSynchronize(p->ev[2]), "event sync");
  FPW_HIP(hipEventElapsedTime(ms, p->ev[4], p->ev[2]), "event time");
  return FPW_OK;
}

fpw_status fpw_phase_entropy(fpw_plan_t p, const int32_t* freq_idx_dev, int32_t k, float* H_dev, float* E_dev,
                             float* V_dev, void* stream) {
  g_err.clear();
  if (!p) return fail(FPW_EINVAL, "plan is NULL");
  if (!freq_idx_dev || !H_dev || !E_dev || !V_dev) return fail(FPW_EINVAL, "null device pointer");
  if (k < 1 || k > p->n_freq) return fail(FPW_EINVAL, "k must be in [1, n_freq]");
  if ((int64_t)p->n_curves * k > INT32_MAX) return fail(FPW_EUNSUPPORTED, "n_curves * k too large");
  fpw::EntropyArgs a{};
  a.tau64 = p->tau64.as<double>();
  a.offsets = p->offsets.as<int64_t>();
  a.freqs = p->freqs.as<double>();
  a.freq_idx = freq_idx_dev;
  a.n_curves = (int32_t)p->n_curves;
  a.k = k;
  a.n_freq = (int32_t)p->n_freq;
  a.n_bins = p->opt.n_bins;
  a.phase = p->opt.phase;
  a.fold_nh = p->fold_nh;
  a.H = H_dev;
  a.E = E_dev;
  a.V = V_dev;
  FPW_HIP(fpw::launch_entropy(a, (hipStream_t)stream), "entropy kernel");
  return FPW_OK;
}

fpw_status fpw_variant(fpw_plan_t p, int32_t v, int32_t* n_bins, int32_t* offset) {
  g_err.clear();
  if (!p || !n_bins || !offset) return fail(FPW_EINVAL, "NULL argument");
  if (v < 0 || v >= p->var.n) return fail(FPW_EINVAL, "variant %d out of range [0, %d)", v, p->var.n);
  *n_bins = p->var_bins[v];
  *offset = p->var.o[v];
  return FPW_OK;
}

fpw_status fpw_get_plan_info(fpw_plan_t p, fpw_plan_info* info) {
  g_err.clear();
  if (!p || !info) return fail(FPW_EINVAL, "NULL argument");
  info->n_curves = p->n_curves;
  info->n_freq = p->n_freq;
  info->n_points = p->n_points;
  info->evals = p->n_points * p->n_freq;
  info->n_bins = p->opt.n_bins;
  info->topk = p->opt.topk;
  info->phase = p->opt.phase;
  info->freqs_per_lane = p->shape.freqs_per_lane;
  info->waves_per_group = p->shape.waves_per_group;
  info->chunk_freqs = p->shape.chunk_freqs;
  info->grid_groups = p->grid_groups;
  info->work_items = p->n_items + p->n_items_w;
  info->n_wide_curves = (int32_t)p->n_wide;
  info->n_wide_points = p->n_wide > 0 ? p->h_offw[(size_t)p->n_curves] : 0;
  info->lds_bytes = (int32_t)p->lds_bytes;
  info->tuned = p->tuned ? 1 : 0;
  info->point_source = p->shape.point_source + 1;
  info->n_variants = p->var.n;
  info->kernel = p->mfma ? 1 : (p->bm ? 2 : 0);
  info->hist_share = p->shape.share;
  info->fuse_prepare = p->fused && !p->mfma ? 1 : 0;
  if (info->fuse_prepare) info->point_source = 3;
  if (p->bm) {
    info->grid_groups = p->bm_grid;
    info->waves_per_group = p->bm_share;
    info->freqs_per_lane = 1;
    info->point_source = p->bm_source + 1;
    info->hist_share = p->bm_share;
    info->lds_bytes = (int32_t)fpw::bm_lds_bytes(p->opt.n_bins, p->opt.baseline_terms, p->bm_share);
  }
  if (p->mfma) {
    info->grid_groups = p->sh_grid_x * p->sh_grid_y;
    info->work_items = p->sh_grid_x * p->sh_grid_y * p->sh_rounds * fpw::kSharedWaves;
    info->lds_bytes = (int32_t)p->sh_lds;
    info->chunk_freqs = p->sh_fw;
    info->waves_per_group = fpw::kSharedWaves;
    info->freqs_per_lane = 0;
    info->point_source = 0;
    info->hist_share = 0;
  }
  return FPW_OK;
}

fpw_status fpw_eval_static(int64_t n_curves, const int64_t* offsets, int64_t n_points, const double* t,
                           const double* y, const double* dy, int64_t n_freq, const double* freqs,
                           const fpw_options* opt, float* S_dev, int32_t* topk_idx, float* topk_val, void* stream) {
  g_err.clear();
  fpw_options o;
  fpw_options_default(&o);
  if (opt) o = *opt;
  fpw_status st = check_options(o);
  if (st != FPW_OK) return st;
  if (!offsets || !t || !y || !dy || !freqs) return fail(FPW_EINVAL, "null input pointer");
  if (n_curves < 1) return fail(FPW_EINVAL, "n_curves must be >= 1");
  if (n_curves > INT32_MAX - 1) return fail(FPW_EUNSUPPORTED, "n_curves too large");
  if (n_points < n_curves) return fail(FPW_EINVAL, "n_points must be >= n_curves (every curve has a point)");
  if (n_freq < 1) return fail(FPW_EINVAL, "n_freq must be >= 1");
  if (n_freq >= INT32_MAX) return fail(FPW_EUNSUPPORTED, "n_freq must be < 2^31");
  if ((topk_idx == nullptr) != (topk_val == nullptr))
    return fail(FPW_EINVAL, "topk_idx and topk_val must both be set or both NULL");
  if (topk_idx && o.topk <= 0) return fail(FPW_EINVAL, "peaks asked for with topk = 0");
  if (!topk_idx && !S_dev) return fail(FPW_EINVAL, "no output: S_dev and topk_idx are NULL");
  if (o.topk > n_freq) return fail(FPW_EINVAL, "topk %d exceeds n_freq %lld", o.topk, (long long)n_freq);
  if (o.phase != FPW_PHASE_FP64 && o.phase != FPW_PHASE_FP64_LISTING)
    return fail(FPW_EUNSUPPORTED, "fpw_eval_static folds in FP64 (listing order)");
  if (o.derived_bins[0] != 0 || o.baseline_terms != 0 || o.autotune || o.freqs_per_lane || o.waves_per_group ||
      o.chunk_freqs || o.point_source || o.hist_share || o.fuse_prepare == 1)
    return fail(FPW_EUNSUPPORTED, "fpw_eval_static takes no derived bin counts, baseline terms, autotune or "
                "launch-shape overrides");
  if (o.n_bins > FPW_MAX_WIDE_BINS)
    return fail(FPW_EUNSUPPORTED, "fpw_eval_static: n_bins %d > FPW_MAX_WIDE_BINS = %d", o.n_bins, FPW_MAX_WIDE_BINS);
  const int topk = topk_idx ? o.topk : 0;
  // ---- checks done: from here on HIP queries (none allocates)
  int dev = 0, n_cu = 0, per_cu = 0;
  FPW_HIP(hipGetDevice(&dev), "hipGetDevice");
  FPW_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  const int M = o.n_bins;
  const int share = M < 8 ? 1 : (M < 16 ? 2 : 4);
  FPW_HIP(fpw::wide_groups_per_cu(FPW_PHASE_FP64_LISTING, topk, M, share, &per_cu), "wide kernel occupancy");
  const int64_t consumers = (int64_t)std::max(1, per_cu) * n_cu;
  // about one item per workgroup, in whole sweeps of 64 frequencies
  int64_t chunk = (n_freq * n_curves + consumers - 1) / consumers;
  chunk = std::max<int64_t>(kWave, ((chunk + kWave - 1) / kWave) * kWave);
  chunk = std::min<int64_t>(chunk, std::max<int64_t>(kWave, ((n_freq + kWave - 1) / kWave) * kWave));
  int64_t per_curve = (n_freq + chunk - 1) / chunk;
  if (per_curve > 1 && n_freq - (per_curve - 1) * chunk == 1) --per_curve;  // a lone trailing frequency joins
  const int64_t n_items = per_curve * n_curves;
  fpw::StaticLayout lay;
  if (n_items > INT32_MAX || !fpw::static_layout(n_curves, n_points, n_items, topk, &lay))
    return fail(FPW_EUNSUPPORTED,
                "fpw_eval_static: %lld curves, %lld points and %lld work items need %zu bytes of its %zu-byte static "
                "scratch", (long long)n_curves, (long long)n_points, (long long)n_items, lay.total,
                fpw::kStaticScratchBytes);
  fpw::StaticPass sp{};
  sp.offsets = offsets;
  sp.t = t;
  sp.y = y;
  sp.dy = dy;
  sp.freqs = freqs;
  sp.n_curves = n_curves;
  sp.n_points = n_points;
  sp.n_items = n_items;
  sp.center = o.center;
  sp.tref_mode = o.tref_mode;
  sp.t_ref = o.t_ref;
  sp.inv_alpha2 = o.inv_alpha2;
  sp.stat_scale = o.stat_scale == FPW_STAT_LISTING_HALF ? 0.5 : 1.0;
  sp.n_freq = (int32_t)n_freq;
  sp.n_bins = M;
  sp.topk = topk;
  sp.chunk = (int32_t)chunk;
  sp.per_curve = (int32_t)per_curve;
  sp.share = share;
  sp.grid = (int)std::min<int64_t>(consumers, n_items);
  sp.S = S_dev;
  sp.idx = topk_idx;
  sp.val = topk_val;
  FPW_HIP(fpw::launch_static_pass(sp, (hipStream_t)stream), "static pass");
  return FPW_OK;
}

void fpw_plan_destroy(fpw_plan_t p) { delete p; }

}  // extern "C"
