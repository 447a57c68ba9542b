// Internal interface between the host runtime (fpw_host.cpp) and the HIP
// kernels (fpw_batched.hip, fpw_aux.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpw {

// One prepared observation, 16 bytes.  `tau` holds the time offset in the
// encoding of the plan's phase mode (FP64, or two FP32 words hi/lo, or one
// FP32).  `pk` packs the fixed-point weight (high 32 bits, unsigned) and the
// fixed-point weighted residual (low 32 bits, two's complement) so that one
// 64-bit integer add accumulates both per-bin sums exactly.
struct alignas(16) Rec {
  uint64_t tau_bits;
  uint64_t pk;
};

// One prepared observation of a curve whose sums take the wide format, 32
// bytes: the time offset as in Rec, then the fixed-point weight (unsigned 64
// bits) and weighted residual (two's complement 64 bits), each added by its
// own 64-bit LDS atomic.
struct alignas(16) WRec {
  uint64_t tau_bits;
  uint64_t wq;
  uint64_t yq;
  uint64_t pad;
};

// Per-bin sum formats of a curve: one packed 64-bit word of 32-bit fields, or
// two 64-bit words (fpw_plan chooses per curve from its weights).
enum { FMT_NARROW = 0, FMT_WIDE = 1 };

// Per-curve constants of a wide-format curve (FP64 epilogue).
struct alignas(16) WideConst {
  double inv_sw;  // data units of one weight unit
  double inv_sy;  // data units of one weighted-residual unit
  double ia2;     // 1 / alpha^2
  double scale;   // 0.5 for the listing's half scale, else 1
};

// Per-curve constants produced by the prepare kernel.
struct alignas(16) CurveConst {
  float kc;     // s_w / s_y^2: converts sum Y_q^2 / W_q back to data units
  float ia2q;   // inv_alpha2 * s_w: the prior term in fixed-point weight units
  float scale;  // 0.5 for the listing's half scale, else 1
  float pad;
};

struct PrepArgs {
  const double* t;
  const double* y;
  const double* dy;
  const int64_t* offsets;
  int64_t n_curves;
  int center;       // FPW_CENTER_*
  int tref_mode;    // FPW_TREF_*
  int phase;        // FPW_PHASE_*
  double t_ref;
  double inv_alpha2;
  float stat_scale;
  Rec* rec;              // [n_points]
  CurveConst* cc;        // [n_curves]
  double* tau64;         // [n_points] FP64 arrays for the plain comparator
  double* w64;
  double* wx64;
  uint32_t* queue;       // work-queue counters of the pass's fold kernels, zeroed here (or null)
  int n_queues;          // counters at queue (1, or 2 with wide-format curves)
  const uint8_t* fmt;    // [n_curves] FMT_*, or null: every curve narrow
  const int64_t* offw;   // [n_curves + 1]: first wide record of each curve (wide curves only)
  WRec* recw;            // wide records
  WideConst* wc;         // [n_curves] (wide curves only)
};

// Work item: curve, frequency range [k0, k1), output slot (natural order).
struct alignas(16) Item {
  int32_t curve, k0, k1, slot;
};

// Periodogram variants of one pass (multi-M reuse): variant v combines k[v]
// fine bins per coarse bin, starting at fine bin o[v].  Variant 0 is always
// the fine binning itself (k = 1, o = 0).
constexpr int kMaxVariants = 8;
struct Variants {
  int32_t n;
  int32_t k[kMaxVariants];
  int32_t o[kMaxVariants];
  // bit m of need: slot m must hold the prefix sum F(0) + ... + F(m) because
  // a derived variant reads it (the last slot of one of its windows, or the
  // slot before its first window)
  uint32_t need[8];
  // With a histogram shared by 2 (own[0]) or 4 (own[1]) waves: the derived
  // variants that wave w computes and keeps (S and peaks), own[.][w][j], 0
  // for none; chosen on the host so that the waves' epilogues take about
  // equal time.
  int8_t own[2][4][4];
};

struct BatchArgs {
  const Rec* rec;
  const int64_t* offsets;
  const CurveConst* cc;
  const double* freqs;
  const Item* items;      // in queue order (longest curves first)
  int32_t n_items;
  int32_t n_freq;
  int32_t n_bins;
  int32_t topk;           // 0 = no peak selection
  int32_t n_curves;
  Variants var;
  double fold_nh;         // shift of the fused FP64 fold: -(1/(2M) - delta), set per plan
  float* S;               // [n_var * n_curves * n_freq] or null
  float* cand_val;        // [(n_slots * n_var) * topk]
  int32_t* cand_idx;      // [(n_slots * n_var) * topk]
  float* edge;            // [(n_slots * n_var) * 4]: S at k0, k0+1, k1-2, k1-1 (-inf if absent)
  uint32_t* queue;        // [1]: the work-queue counter; zeroed by the prepare kernel
  // wide-format launch only: its records, offsets into them and constants
  const WRec* recw;
  const int64_t* offw;
  const WideConst* wc;
};

// Raw inputs of the fused pass, whose fold kernel prepares every curve itself.
struct FusedArgs {
  const double* t;
  const double* y;
  const double* dy;
  int center;        // FPW_CENTER_*
  int tref_mode;     // FPW_TREF_*
  double t_ref;
  double inv_alpha2;
  float stat_scale;
};

struct MergeArgs {
  const float* cand_val;
  const int32_t* cand_idx;
  const float* edge;
  const int32_t* slot_k0;     // [n_slots + n_curves]: k0 of each slot in natural order
  const int32_t* curve_slot;  // [n_curves + 1]: first slot of each curve
  int32_t n_curves;
  int32_t n_freq;
  int32_t topk;
  int32_t n_var;
  int32_t* out_idx;           // [n_var * n_curves * topk]
  float* out_val;
};

struct TopkArgs {
  const float* S;
  int32_t n_curves;
  int32_t n_freq;
  int32_t k;
  int32_t* out_idx;
  float* out_val;
};

struct Fp64Args {
  const double* tau;
  const double* w;
  const double* wx;
  const double* freqs;
  int64_t p0;          // first point of the curve
  int32_t n;           // points in the curve
  int32_t n_freq;
  int32_t n_bins;
  double inv_alpha2;
  double scale;
  double* S;           // row of the curve: [n_freq]
};

struct BinsArgs {
  const Rec* rec;
  const double* tau64;
  const double* freqs;
  int64_t p0;
  int32_t n;
  int32_t f_begin, f_end;
  int32_t n_bins;
  int32_t phase;
  double fold_nh;   // as in BatchArgs
  int32_t* out;
};

struct EntropyArgs {
  const double* tau64;
  const int64_t* offsets;
  const double* freqs;
  const int32_t* freq_idx;  // [n_curves * k]
  int32_t n_curves, k, n_freq, n_bins, phase;
  double fold_nh;   // as in BatchArgs
  float* H;
  float* E;
  float* V;
};

// Shared-timestamp batches (every curve observed at the same times).  Per
// curve and point, the fixed-point weight and weighted residual (30-bit
// ranges) are split into four signed base-256 digits each; the digits sit in
// 1 KB tiles laid out as the A operand of the 32x32x32 int8 matrix product:
// tile (group g of 4 curves, K-block kb of 32 points), lane l = 32h + r reads
// bytes [16 l, 16 l + 16), byte j is point 32 kb + 16 h + j.  Row
// r = 8 (2 u + q) + 4 v + i holds digit i of quantity q (0 weight, 1
// residual) of curve 4g + 2u + v, so that the product's lanes of half v
// receive both quantities of curves 4g + v and 4g + 2 + v.
constexpr int kSharedGroupCurves = 4;   // curves per A tile
constexpr int kSharedTileBytes = 1024;  // one tile: 32 rows x 32 points
constexpr int kSharedMaxBins = 64;      // largest M of the matrix-core kernel
constexpr int kSharedMaxFw = 12;        // frequencies per wave and round, at most
// points per curve: the products accumulate 64 x (digit sums), |64 * 128 * N| < 2^31
constexpr int kSharedMaxPoints = 262112;
constexpr int kSharedWaves = 8;         // waves per workgroup of the shared kernel

struct SharedPrepArgs {
  const double* y;         // [n_curves * n_points], curve-major
  const double* dy;
  int32_t n_curves, n_points, n_kblocks;
  int center;              // FPW_CENTER_*
  double inv_alpha2;
  float stat_scale;
  int8_t* vals;            // [n_groups * n_kblocks * 1024]; padding stays zero
  CurveConst* cc;          // [n_curves padded]
};

struct SharedArgs {
  const double* tau;       // [n_kblocks * 32] shared time offsets, zero-padded
  const int8_t* vals;      // digit tiles, see above
  const CurveConst* cc;    // [n_curves padded]
  const double* freqs;     // [n_freq]
  int32_t n_curves, n_freq, n_bins;
  int32_t n_kblocks;       // K-blocks of 32 points
  int32_t chunk_kblocks;   // K-blocks staged in LDS at a time
  int32_t fw;              // frequencies per wave per round (fw * n_bins <= 32 * B tiles)
  int32_t rounds;          // rounds per workgroup (8 waves x fw frequencies each)
  int32_t priv_bytes;      // LDS bytes private to each wave
  double fold_nh;          // as in BatchArgs
  float* S;                // [n_curves * n_freq]
};

// Baseline-marginalised statistic (App. A, general case).  Every quantity
// the statistic needs is a per-bin sum of fixed-point integers, so the bin
// sums are exact; the per-curve constants are formed from the same rounded
// per-point values, which keeps S = v^T L^-1 v + r^T Q^-1 r consistent with
// one exactly solved (rounded) problem.
// Baseline sums of an observation (the records themselves are Rec): with
// K = 3 terms the pair (w T_1, w T_2) in fixed point, T_2 * 2^32 + T_1 (two's
// complement), one 64-bit word; with K = 2 the word w T_1 alone (32 bits).

struct BaseConst {
  double g[3];      // H^-1 z: the best-fitting baseline coefficients
  double H[6];      // I + B^T C_sigma^-1 B, upper triangle 00 01 02 11 12 22
  double inv_sw, inv_sy, inv_sz;  // fixed-point units of weight, residual and w T_k
  double beta;      // baseline prior scale
  double ia2;       // 1 / alpha^2
  double scale;     // 0.5 for the listing's half scale, else 1
};

struct BmPrepArgs {
  const double* t;
  const double* y;
  const double* dy;
  const int64_t* offsets;
  int64_t n_curves;
  int center, tref_mode, n_terms;
  double t_ref, inv_alpha2, beta, stat_scale;
  Rec* rec;         // [n_points]: tau and (weight, weighted residual), as for the batched kernel
  uint64_t* z64;    // [n_points] when n_terms == 3
  uint32_t* z32;    // [n_points] when n_terms == 2
  BaseConst* bc;    // [n_curves]
  uint32_t* queue;  // work-queue counter of the pass's baseline kernel, zeroed here (or null)
};

struct BmArgs {
  const Rec* rec;
  const void* z;     // baseline sums per observation: uint64_t (K = 3), uint32_t (K = 2), unused (K = 1)
  const int64_t* offsets;
  const BaseConst* bc;
  const double* freqs;
  const Item* items;
  int32_t n_items, n_freq, n_bins;
  int32_t n_terms;   // baseline terms K (1..3); K = 1 needs no second sum
  int32_t share;     // waves per histogram (1, 2, 4): the workgroup size in waves
  int32_t source;    // observations: 0 scalar loads, 1 vector loads + DPP broadcast
  double fold_nh;    // as in BatchArgs
  float* S;          // [n_curves * n_freq]
  uint32_t* queue;   // [1], zeroed by the baseline prepare kernel, as for the batched kernel
};

hipError_t launch_bm_prepare(const BmPrepArgs& a, hipStream_t s);
hipError_t launch_bm(const BmArgs& a, int phase, int grid, hipStream_t s);
hipError_t bm_groups_per_cu(int phase, int n_bins, int n_terms, int share, int source, int* out);
size_t bm_lds_bytes(int n_bins, int n_terms, int share);

// The pass that allocates nothing (fpw_eval_static): its scratch is one
// file-scope device array of kStaticScratchBytes per GPU.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;

// Byte offsets of one call's regions in that array.
struct StaticLayout {
  size_t offs, recw, wc, items, slot_k0, curve_slot, cand_val, cand_idx, edge, queue, total;
};

struct StaticPass {
  const int64_t* offsets;  // caller's device arrays
  const double* t;
  const double* y;
  const double* dy;
  const double* freqs;
  int64_t n_curves, n_points, n_items;
  int center, tref_mode;
  double t_ref, inv_alpha2, stat_scale;
  int32_t n_freq, n_bins, topk;
  int32_t chunk, per_curve;  // frequencies per work item, items per curve
  int share, grid;           // wide-kernel waves per histogram and workgroups
  float* S;                  // outputs (device), S may be null, idx/val null when topk == 0
  int32_t* idx;
  float* val;
};

// False when the regions of a call do not fit the array.
bool static_layout(int64_t n_curves, int64_t n_points, int64_t n_items, int topk, StaticLayout* l);
// Prepare, wide-format fold and peak merge, with every buffer beyond the
// caller's in the static array (hipGetSymbolAddress once per device).
hipError_t launch_static_pass(const StaticPass& s, hipStream_t st);

// Launch shapes of the batched kernel.
struct Shape {
  int freqs_per_lane;   // 1 or 2
  int waves_per_group;  // 1, 2 or 4
  int chunk_freqs;      // frequencies per work item
  int point_source;     // 0: scalar loads, 1: vector loads + DPP broadcast (one frequency per lane)
  int share;            // waves per histogram: 1 (private), or 2 / 4 = waves_per_group (one item per group)
};

// Launchers; each returns the hipError_t of its launch.
hipError_t launch_prepare(const PrepArgs& a, hipStream_t s);
hipError_t launch_batched(const BatchArgs& a, const Shape& shape, int phase, int grid_groups,
                          size_t lds_bytes, hipStream_t s);  // n_var > 1 needs one frequency per lane
// The wide-format fold kernel over a.items (curves whose sums need two 64-bit
// words), with `share` waves per histogram (1, 2 or 4), one frequency per lane
// and scalar point loads; one periodogram variant.
hipError_t launch_wide(const BatchArgs& a, int phase, int share, int grid_groups, hipStream_t s);
size_t wide_lds_bytes(int n_bins, int share);
hipError_t wide_groups_per_cu(int phase, int topk, int n_bins, int share, int* out);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s, bool group = false);
// Fused pass of a small plan: prepare + fold/bin/accumulate/reduce + peaks
// in workgroups of fused_waves() waves, one per item of a.items (a.n_items
// of them); then launch_merge with `group` set merges each curve's peaks
// with one workgroup of four waves.
hipError_t launch_fused(const BatchArgs& a, const FusedArgs& o, int phase, hipStream_t s);
size_t fused_lds_bytes(int n_bins);
int fused_waves();
hipError_t launch_topk(const TopkArgs& a, hipStream_t s);
hipError_t launch_fp64(const Fp64Args& a, hipStream_t s);
hipError_t launch_bins(const BinsArgs& a, hipStream_t s);
hipError_t launch_entropy(const EntropyArgs& a, hipStream_t s);
hipError_t launch_prepare_shared(const SharedPrepArgs& a, hipStream_t s);
// curve_groups: A tiles (of 4 curves) per workgroup, 4 is the one built;
// nb: one-hot B tiles (32 columns) per wave, 2 or 3
hipError_t launch_shared(const SharedArgs& a, int phase, int curve_groups, int nb, int grid_x, int grid_y,
                         size_t lds_bytes, hipStream_t s);
// B tiles and frequencies per wave for M bins: the choice with the best column use
void shared_shape(int n_bins, int* nb, int* fw);

// LDS bytes the batched kernel needs per workgroup (n_var periodogram variants).
size_t batched_lds_bytes(const Shape& shape, int n_bins, int n_var);
// Whether the batched kernel is built for this shape, phase mode and variant count.
bool batched_shape_built(const Shape& shape, int phase, int n_var);
// Persistent workgroups per CU the batched kernel reaches for this shape.
hipError_t batched_groups_per_cu(const Shape& shape, int phase, int topk, int n_var, size_t lds_bytes, int* out);
// Top-k list length the kernels are instantiated for (8 or 16; 0 without peaks).
int topk_capacity(int k);

}  // namespace fpw
