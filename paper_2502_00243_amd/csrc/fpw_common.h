// Device code shared by every kernel of libfpw: the fold/bin variants,
// the LDS histogram helpers and the top-k lists.  The main batched kernel,
// the parity hook and the FP64 comparator all bin through these same
// functions.
#pragma once

#include <float.h>
#include <math.h>

#include <type_traits>

#include "fpw_internal.h"

namespace fpw {
namespace dev {

constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52: fma(x, M, kMagic) rounds to an integer in the low word
constexpr int kBatch = 8;                       // observations per scalar-load batch
constexpr int kWave = 64;

enum { PH_FP64 = 0, PH_LISTING = 1, PH_DF32 = 2, PH_FP32 = 3 };

__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }

// Time-offset encodings stored in a record for each phase mode.
__device__ __forceinline__ uint64_t encode_tau(double tau, int phase) {
  if (phase == PH_DF32) {
    const float th = (float)tau;
    const float tl = (float)(tau - (double)th);
    return ((uint64_t)__float_as_uint(tl) << 32) | (uint64_t)__float_as_uint(th);
  }
  if (phase == PH_FP32) return (uint64_t)__float_as_uint((float)tau);
  return (uint64_t)__double_as_longlong(tau);
}

// ---------------------------------------------------------------- fold + bin
// Folder<PH>::bin(tau) returns the bin of one observation at the lane's
// frequency.  All results lie in [0, M]; only PH_FP64 produces M, which
// stands for bin 0 (see below) and is folded onto it when the bins are read.
template <int PH>
struct Folder;

// FP64, fused: the fold is shifted by just under half a bin,
// phase' = frac(fma(tau, f, nh)) with nh = -(1/(2M) - delta), and
// round(M phase') (one fma into the magic constant) is the bin.  Off the
// edges that equals floor(M frac(tau f)).  delta (set per plan, at least
// twice the largest rounding error of the first fma over the plan's fold
// range) makes a point exactly on an edge land above the rounding midpoint,
// so it takes the upper bin, as floor does, instead of following
// round-half-to-even; the price is that points within ~1.4 M delta bin
// widths below an edge also move up (the plan keeps that under 1e-7 bin
// widths, else it folds in the listing order).  phase' just below 1 rounds
// to M, which is bin 0.
template <>
struct Folder<PH_FP64> {
  double f, nh, md;
  __device__ __forceinline__ void init(double freq, int M, double shift) {
    f = freq;
    md = (double)M;
    nh = shift;
    // tau comes from an SGPR, so the fma's other uniform operand must sit in
    // a VGPR; held there once, it is not copied in again for every batch
    asm volatile("" : "+v"(nh));
  }
  __device__ __forceinline__ int bin(uint64_t tb) const {
    const double tau = __longlong_as_double((long long)tb);
    const double ph = __builtin_amdgcn_fract(__builtin_fma(tau, f, nh));
    return (int)lo32((uint64_t)__double_as_longlong(__builtin_fma(ph, md, kMagic)));
  }
};

// FP64 in the order of the paper's listing: p = fl(tau f); phi = p - floor(p)
// (exact for p >= 0); bin = trunc(fl(phi M)).  Identical to a plain FP64 loop.
template <>
struct Folder<PH_LISTING> {
  double f, md;
  __device__ __forceinline__ void init(double freq, int M, double) {
    f = freq;
    md = (double)M;
  }
  __device__ __forceinline__ int bin(uint64_t tb) const {
    const double tau = __longlong_as_double((long long)tb);
    const double p = tau * f;
    const double ph = __builtin_amdgcn_fract(p);
    return (int)(ph * md);
  }
};

// Compensated FP32 ("double-float"): tau = th + tl and f = fh + fl.  The
// product th*fh is split exactly (fma), the cross terms are added to the low
// part, the fraction is taken from the exact high part, and the bin is the
// floor of M*(fraction + low part) formed with an exact product and one
// final correction step.
template <>
struct Folder<PH_DF32> {
  float fh, fl, mf;
  int m;
  __device__ __forceinline__ void init(double freq, int M, double) {
    fh = (float)freq;
    fl = (float)(freq - (double)fh);
    mf = (float)M;
    m = M;
  }
  __device__ __forceinline__ int bin(uint64_t tb) const {
    const float th = __uint_as_float(lo32(tb));
    const float tl = __uint_as_float(hi32(tb));
    const float ph = th * fh;
    float pl = __builtin_fmaf(th, fh, -ph);
    pl = __builtin_fmaf(th, fl, pl);
    pl = __builtin_fmaf(tl, fh, pl);
    const float fr = __builtin_amdgcn_fractf(ph);  // ph - floor(ph), exact: 0 <= ph < 2^23
    const float uh = mf * fr;
    const float ul = __builtin_fmaf(mf, fr, -uh);  // uh + ul = M*fr exactly
    const float c = __builtin_fmaf(mf, pl, ul);
    const float b0 = floorf(uh);
    const float r = (uh - b0) + c;           // uh - b0 exact
    // b = floor(M (fr + pl)) with fr in [0, 1) and |pl| < 3/4 (the plan
    // keeps tau f below 2^22 cycles, so ulp(ph) <= 1/2 and each cross term
    // is below 1/4): b lies in [-M, 2M - 1] and one compare each way folds
    // it into [0, M) instead of an integer remainder
    const int b = (int)(b0 + floorf(r));  // a sum of small integers: exact
    return b >= m ? b - m : (b < 0 ? b + m : b);
  }
};

// Naive FP32 product, for the precision study only.
template <>
struct Folder<PH_FP32> {
  float f, mf;
  int m;
  __device__ __forceinline__ void init(double freq, int M, double) {
    f = (float)freq;
    mf = (float)M;
    m = M;
  }
  __device__ __forceinline__ int bin(uint64_t tb) const {
    const float p = __uint_as_float(lo32(tb)) * f;
    const float fr = p - floorf(p);
    const int b = (int)(fr * mf);
    return b < m - 1 ? b : m - 1;
  }
};

// ---------------------------------------------------------------- DPP helpers
// Lane Q of each row of 16 lanes, broadcast to its row (64-bit DPP
// row_newbcast).  Every lane reads an existing lane, so the "old" operand is
// never used.
template <int Q>
__device__ __forceinline__ uint64_t row_bcast(uint64_t v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x150 + Q, 0xf, 0xf, true);
}

// f(integral_constant<int, q>) for q = Q .. N-1: DPP controls must be constants.
template <int Q, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (Q < N) {
    f(std::integral_constant<int, Q>{});
    static_for<Q + 1, N>(f);
  }
}

// ---------------------------------------------------------------- LDS histograms
__device__ __forceinline__ void lds_add(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t lds_take(uint64_t* p) {
  return __hip_atomic_exchange(p, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds the Eq. 1 term of one bin, Y_q^2 / (W_q + ia2q), from its packed
// fixed-point word.  Every non-empty bin has W_q >= 1 (weights are clamped to
// at least one unit) and an empty bin has Y_q = 0; ia2q is at least
// kMinPrior (make_curve_const), which leaves fl(W_q + ia2q) unchanged for
// W_q >= 1 and keeps an empty bin's denominator positive, so it adds 0
// without a branch or a clamp.
constexpr float kMinPrior = 0x1p-100f;
__device__ __forceinline__ float add_bin_term(float acc, uint64_t v, float ia2q) {
  const uint32_t l = lo32(v);
  const int32_t yq = (int32_t)l;
  const uint32_t wq = hi32(v) + (l >> 31);  // undo the borrow of a negative low word
  const float d = (float)wq + ia2q;
  const float yf = (float)yq;
  return __builtin_fmaf(yf, yf * __builtin_amdgcn_rcpf(d), acc);
}

// Slots are read (and cleared) eight at a time so that the LDS round trips
// overlap; slot indices past M are clamped to slot M, which is empty by then.
constexpr int kReduceBlock = 8;

// The FP64 fused fold files phases just below 1 in slot M; they belong to bin 0.
template <int PH>
__device__ __forceinline__ uint64_t take_wrap_slot(uint64_t* h, int M) {
  return PH == PH_FP64 ? lds_take(h + M * kWave) : (uint64_t)0;
}

template <int PH>
__device__ __forceinline__ void take_block(uint64_t* h, int M, int m0, uint64_t (&f)[kReduceBlock]) {
#pragma unroll
  for (int q = 0; q < kReduceBlock; ++q) f[q] = lds_take(h + min(m0 + q, M) * kWave);
}

// S is summed in one fixed order whatever the launch shape: the read blocks
// of 8 bins are split into kSumParts consecutive parts (part p = blocks
// [p nb / 4, (p+1) nb / 4) of nb), each part's terms are added in bin order
// from zero, and the part sums are added in part order.  A histogram shared
// by 2 or 4 waves gives each wave whole parts, so private and shared
// histograms (and the multi-M reduction) produce bit-identical S.
constexpr int kSumParts = 4;
__device__ __forceinline__ int part_block(int p, int n_blocks) { return p * n_blocks / kSumParts; }

// Reads and clears one lane's histogram (slot m at h + 64 m) and returns
// sum_m Y_m^2 / (W_m + 1/alpha^2) in fixed-point units, in the order above.
template <int PH>
__device__ __forceinline__ float reduce_hist(uint64_t* h, int M, float ia2q) {
  const uint64_t wrap = take_wrap_slot<PH>(h, M);
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  float s = 0.f;
  for (int p = 0; p < kSumParts; ++p) {
    float acc = 0.f;
    for (int b = part_block(p, nb); b < part_block(p + 1, nb); ++b) {
      const int m0 = b * kReduceBlock;
      uint64_t f[kReduceBlock];
      take_block<PH>(h, M, m0, f);
      if (m0 == 0) f[0] += wrap;
#pragma unroll
      for (int q = 0; q < kReduceBlock; ++q)
        if (m0 + q < M) acc = add_bin_term(acc, f[q], ia2q);
    }
    s += acc;
  }
  return s;
}

// Whole-wave neighbour exchange through DPP (no LDS traffic): the value of
// lane i-1 (lane 0 keeps its own) and of lane i+1 (lane 63 keeps its own).
__device__ __forceinline__ float from_lane_below(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_lane_above(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Copies a wave-uniform 64-bit value from SGPRs to a VGPR pair in one
// instruction (the data operand of an LDS atomic must be a VGPR).
__device__ __forceinline__ uint64_t uniform_to_vgpr(uint64_t s) {
  uint64_t v;
  asm("v_mov_b64 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

// ---------------------------------------------------------------- top-k lists
// Strict total order of peaks: larger S first, then lower frequency index.
__device__ __forceinline__ bool better(float av, int ai, float bv, int bi) {
  return av > bv || (av == bv && ai < bi);
}

template <int K>
struct TopList {
  float v[K];
  int i[K];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      v[q] = -INFINITY;
      i[q] = INT_MAX;
    }
  }
  // Inserts (s, k) when `pred`, keeping the K best in order.
  __device__ __forceinline__ void insert(float s, int k, bool pred) {
    if (pred && better(s, k, v[K - 1], i[K - 1])) {
      bool b[K];
#pragma unroll
      for (int q = 0; q < K; ++q) b[q] = better(s, k, v[q], i[q]);
#pragma unroll
      for (int q = K - 1; q >= 0; --q) {
        const bool prev = q > 0 ? b[q - 1] : false;
        if (prev) {
          v[q] = v[q - 1];
          i[q] = i[q - 1];
        } else if (b[q]) {
          v[q] = s;
          i[q] = k;
        }
      }
    }
  }
  __device__ __forceinline__ void pop_front() {
#pragma unroll
    for (int q = 0; q < K - 1; ++q) {
      v[q] = v[q + 1];
      i[q] = i[q + 1];
    }
    v[K - 1] = -INFINITY;
    i[K - 1] = INT_MAX;
  }
};

__device__ __forceinline__ int int_from_lane_below(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false);
}

// The k best peaks a wave has seen, spread over its lanes: lane r < k holds
// entry r (best first), the other lanes hold (-inf, INT_MAX).  Two VGPRs per
// list, however large k is; insertions run as a wave-uniform loop over the
// candidate lanes, which are few once the list has filled.
template <int CTRL>
__device__ __forceinline__ void best_from_dpp(float& v, int& i) {
  // the pair CTRL brings in, or (-inf, INT_MAX) where it brings none
  const float ov = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(-INFINITY), __float_as_int(v), CTRL, 0xf, 0xf, false));
  const int oi = __builtin_amdgcn_update_dpp(INT_MAX, i, CTRL, 0xf, 0xf, false);
  if (better(ov, oi, v, i)) {
    v = ov;
    i = oi;
  }
}

// The best (value, index) among the lanes where `pred` holds, in every lane
// ((-inf, INT_MAX) if none): row_shr by 1, 2, 4 and 8 leaves each row's best
// in its last lane, and the four row results are compared in order.
__device__ __forceinline__ void wave_best(float s, int idx, bool pred, float& bv, int& bi) {
  float v = pred ? s : -INFINITY;
  int i = pred ? idx : INT_MAX;
  best_from_dpp<0x111>(v, i);
  best_from_dpp<0x112>(v, i);
  best_from_dpp<0x114>(v, i);
  best_from_dpp<0x118>(v, i);
  bv = lane_value(v, 15);
  bi = __builtin_amdgcn_readlane(i, 15);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const float ov = lane_value(v, 16 * r + 15);
    const int oi = __builtin_amdgcn_readlane(i, 16 * r + 15);
    if (better(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
}

struct WaveTop {
  float v;
  int i;
  __device__ __forceinline__ void init() {
    v = -INFINITY;
    i = INT_MAX;
  }
  // Puts (cs, ci) into the list if it beats the k-th entry.
  __device__ __forceinline__ bool insert(float cs, int ci, int k, int lane) {
    if (!better(cs, ci, lane_value(v, k - 1), __builtin_amdgcn_readlane(i, k - 1))) return false;
    // entries better than the candidate form a prefix of length p
    const int p = __popcll(__ballot(lane < k && better(v, i, cs, ci)));
    const float vb = from_lane_below(v);
    const int ib = int_from_lane_below(i);
    if (lane == p) {
      v = cs;
      i = ci;
    } else if (lane > p && lane < k) {
      v = vb;
      i = ib;
    }
    return true;
  }
  // Offers (s, idx) of every lane where `pred` holds; k = list length.  The
  // indices of the lanes are distinct.  The list becomes the k best of the
  // list and the offers, whatever order they are taken in: lane by lane
  // when they are few, best first (at most k can enter) when there are
  // more than 2k of them.
  __device__ __forceinline__ void offer(float s, int idx, bool pred, int k, int lane) {
    const float tv = lane_value(v, k - 1);
    const int ti = __builtin_amdgcn_readlane(i, k - 1);
    bool cand = pred && better(s, idx, tv, ti);
    uint64_t m = __ballot(cand);
    if (__popcll(m) > 2 * k) {
      for (int r = 0; r < k; ++r) {
        float cs;
        int ci;
        wave_best(s, idx, cand, cs, ci);
        if (!insert(cs, ci, k, lane)) break;
        cand = cand && idx != ci;
      }
      return;
    }
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      insert(lane_value(s, l), __builtin_amdgcn_readlane(idx, l), k, lane);
    }
  }
  // Writes the list: (value, index) for r < k, index -1 where the value is -inf.
  __device__ __forceinline__ void store(int k, float* out_v, int32_t* out_i, int lane) const {
    if (lane < k) {
      out_v[lane] = v;
      out_i[lane] = v == -INFINITY ? -1 : i;
    }
  }
};

// Merges the 64 lanes' lists: writes the `k` best (value, index) of the wave,
// best first; missing entries are (-inf, -1).  Every lane must call it.
template <int K>
__device__ __forceinline__ void wave_select(TopList<K>& l, int k, float* out_v, int32_t* out_i, int lane) {
  for (int r = 0; r < k; ++r) {
    float bv;
    int bi;
    wave_best(l.v[0], l.i[0], true, bv, bi);  // the best head of the 64 lists
    const bool none = bv == -INFINITY;
    if (lane == 0) {
      out_v[r] = bv;
      out_i[r] = none ? -1 : bi;
    }
    if (!none && l.i[0] == bi) l.pop_front();
  }
}

// ---------------------------------------------------------------- chunk merge
// Offers chunk q's candidate list and the two peaks its first frequency and
// its predecessor's last one may form across the boundary (decided from the
// four edge values of each chunk); q0 = the curve's first chunk.
template <int K>
__device__ __forceinline__ void merge_slot(const MergeArgs& a, int q, int q0, int v, TopList<K>& l) {
  const int nv = a.n_var;
  const int64_t cq = ((int64_t)q * nv + v) * a.topk;
  for (int r = 0; r < a.topk; ++r) {
    const int ci = a.cand_idx[cq + r];
    l.insert(a.cand_val[cq + r], ci, ci >= 0);
  }
  if (q > q0) {
    // b = first frequency of this chunk, b-1 = last of the previous one
    const int b = a.slot_k0[q];
    const float* ep = a.edge + ((int64_t)(q - 1) * nv + v) * 4;
    const float* eq = a.edge + ((int64_t)q * nv + v) * 4;
    const float sa_left = ep[2], sa = ep[3], sb = eq[0], sb_right = eq[1];
    l.insert(sa, b - 1, sa > sa_left && sa >= sb);
    l.insert(sb, b, sb > sa && sb >= sb_right);
  }
}

// Peaks of curve c, variant v from its chunks' candidate lists: one wave,
// lanes take the chunks in turn, then the wave selects the curve's top k.
// Every lane of the wave must call it.
template <int K>
__device__ __forceinline__ void merge_curve(const MergeArgs& a, int c, int v, int lane) {
  TopList<K> l;
  l.init();
  const int q0 = a.curve_slot[c], q1 = a.curve_slot[c + 1];
  for (int q = q0 + lane; q < q1; q += kWave) merge_slot<K>(a, q, q0, v, l);
  const int64_t o = ((int64_t)v * a.n_curves + c) * a.topk;
  wave_select<K>(l, a.topk, a.out_val + o, a.out_idx + o, lane);
}

// The same with the W waves of a workgroup (every thread must call it): each
// wave selects the best k of its share of the chunks into LDS (lv, li: W * K
// entries), then wave 0 selects the curve's k from those.  The k best of a
// set under the strict order of `better` do not depend on how it is split,
// so the result equals merge_curve's.
template <int K, int W>
__device__ __forceinline__ void merge_curve_group(const MergeArgs& a, int c, int v, int wave, int lane, float* lv,
                                                  int32_t* li) {
  TopList<K> l;
  l.init();
  const int q0 = a.curve_slot[c], q1 = a.curve_slot[c + 1];
  for (int q = q0 + wave * kWave + lane; q < q1; q += W * kWave) merge_slot<K>(a, q, q0, v, l);
  wave_select<K>(l, a.topk, lv + wave * K, li + wave * K, lane);
  __syncthreads();
  if (wave == 0) {
    TopList<K> m;
    m.init();
    for (int q = lane; q < W * a.topk; q += kWave) {
      const int w = q / a.topk, r = q - w * a.topk;
      const int ci = li[w * K + r];
      m.insert(lv[w * K + r], ci, ci >= 0);
    }
    const int64_t o = ((int64_t)v * a.n_curves + c) * a.topk;
    wave_select<K>(m, a.topk, a.out_val + o, a.out_idx + o, lane);
  }
}

// ---------------------------------------------------------------- per-curve preparation
// Used by the prepare kernel and by the fused pass, so that both derive
// identical constants and records from the same inputs.  A workgroup of
// kPrepThreads threads handles one curve: thread t visits points t,
// t + kPrepThreads, ... in order; each wave reduces with an xor butterfly
// (both lanes of every exchange add the same two operands, so all lanes end
// with the same value) and the wave totals are combined in wave order.  The
// results are identical in every thread and reproducible.
constexpr int kPrepThreads = 256;
constexpr int kPrepWaves = kPrepThreads / kWave;
constexpr int kPrepRed = 5 * kPrepWaves;  // doubles of LDS the reduction needs

// Centring, reference time and fixed-point scales of one curve.
struct PrepConst {
  double mu, tref, s_w, s_y;
  double sw, ay;  // sum of w and of |w x|: the wide format's scales derive from them
};

__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
  for (int s = kWave / 2; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}
__device__ __forceinline__ double wave_min_all(double v) {
#pragma unroll
  for (int s = kWave / 2; s > 0; s >>= 1) v = fmin(v, __shfl_xor(v, s));
  return v;
}

// Every thread of the workgroup must call it (it holds barriers); `red` is
// kPrepRed doubles of LDS.  If `keep` is set, thread t also returns the
// (t, y, dy) of observation t there (0, 0, 1 where t >= n).  Weights w = 1/dy^2; the centre is the weighted
// mean, the plain mean or 0 (center 0, 1, 2); the reference time 0, min(t)
// or t_ref (tref_mode 0, 1, 2).  Fixed-point scales: the sum of the weights
// of any subset of points stays below 2^32 and the sum of |w x| below 2^31,
// so no bin sum can leave its 32-bit field.
__device__ __forceinline__ PrepConst curve_prep(const double* __restrict__ t, const double* __restrict__ y,
                                                const double* __restrict__ dy, int n, int center, int tref_mode,
                                                double t_ref, double* red, double* keep = nullptr) {
  const int th = threadIdx.x, lane = th & (kWave - 1), wave = th / kWave;
  double sw = 0.0, swy = 0.0, sy = 0.0, tmin = INFINITY;
  if (keep != nullptr) {
    keep[0] = 0.0;
    keep[1] = 0.0;
    keep[2] = 1.0;
  }
  for (int i = th; i < n; i += kPrepThreads) {
    const double d = dy[i];
    const double w = 1.0 / (d * d);
    const double yy = y[i];
    const double tt = t[i];
    if (keep != nullptr && i == th) {
      keep[0] = tt;
      keep[1] = yy;
      keep[2] = d;
    }
    sw += w;
    swy += w * yy;
    sy += yy;
    tmin = fmin(tmin, tt);
  }
  sw = wave_sum_all(sw);
  swy = wave_sum_all(swy);
  sy = wave_sum_all(sy);
  tmin = wave_min_all(tmin);
  __syncthreads();  // earlier readers of red are done
  if (lane == 0) {
    red[wave] = sw;
    red[kPrepWaves + wave] = swy;
    red[2 * kPrepWaves + wave] = sy;
    red[3 * kPrepWaves + wave] = tmin;
  }
  __syncthreads();
  sw = red[0];
  swy = red[kPrepWaves];
  sy = red[2 * kPrepWaves];
  tmin = red[3 * kPrepWaves];
#pragma unroll
  for (int w = 1; w < kPrepWaves; ++w) {
    sw += red[w];
    swy += red[kPrepWaves + w];
    sy += red[2 * kPrepWaves + w];
    tmin = fmin(tmin, red[3 * kPrepWaves + w]);
  }
  PrepConst k;
  k.mu = center == 0 ? swy / sw : (center == 1 ? sy / (double)n : 0.0);
  k.tref = tref_mode == 0 ? 0.0 : (tref_mode == 1 ? tmin : t_ref);
  double ay = 0.0;
  for (int i = th; i < n; i += kPrepThreads) {
    const double d = dy[i];
    const double w = 1.0 / (d * d);
    ay += fabs(w * (y[i] - k.mu));
  }
  ay = wave_sum_all(ay);
  if (lane == 0) red[4 * kPrepWaves + wave] = ay;
  __syncthreads();
  ay = red[4 * kPrepWaves];
#pragma unroll
  for (int w = 1; w < kPrepWaves; ++w) ay += red[4 * kPrepWaves + w];
  k.s_w = (4294967296.0 - 2.0 - 2.0 * (double)n) / sw;
  k.s_y = ay > 0.0 ? (2147483648.0 - 2.0 - (double)n) / ay : 1.0;
  k.sw = sw;
  k.ay = ay;
  return k;
}

// The record of one observation: time offset in the phase mode's encoding,
// fixed-point weight (at least 1, so that every occupied bin has W >= 1) and
// weighted residual.
__device__ __forceinline__ Rec make_rec(double t, double y, double dy, const PrepConst& k, int phase) {
  const double w = 1.0 / (dy * dy);
  const double wx = w * (y - k.mu);
  const uint64_t wq = (uint64_t)fmax(1.0, rint(w * k.s_w));
  const int64_t yq = (int64_t)rint(wx * k.s_y);
  Rec r;
  r.tau_bits = encode_tau(t - k.tref, phase);
  r.pk = (wq << 32) + (uint64_t)yq;
  return r;
}

// Wide format: 64-bit fields with the scales set a 2^-11 margin below the
// field limits, so a sum of rounded values (each at most half a unit above
// its exact product, and that product at most an ulp above) cannot reach
// 2^64 (weights) or 2^63 in magnitude (weighted residuals) for any binning.
// A unit is then Sum(w) / 2^64 of weight and Sum|w x| / 2^63 of residual,
// and a value that large is held to ~2^-53 relative by the FP64 product
// itself.
constexpr double kWideScaleW = 18446744073709551616.0 * (1.0 - 1.0 / 2048.0);
constexpr double kWideScaleY = 9223372036854775808.0 * (1.0 - 1.0 / 2048.0);

__device__ __forceinline__ double wide_scale_w(const PrepConst& k) { return kWideScaleW / k.sw; }
__device__ __forceinline__ double wide_scale_y(const PrepConst& k) { return k.ay > 0.0 ? kWideScaleY / k.ay : 1.0; }

__device__ __forceinline__ WRec make_wrec(double t, double y, double dy, const PrepConst& k, int phase) {
  const double w = 1.0 / (dy * dy);
  const double wx = w * (y - k.mu);
  WRec r;
  r.tau_bits = encode_tau(t - k.tref, phase);
  r.wq = (uint64_t)rint(w * wide_scale_w(k));
  r.yq = (uint64_t)(int64_t)rint(wx * wide_scale_y(k));
  r.pad = 0;
  return r;
}

__device__ __forceinline__ WideConst make_wide_const(const PrepConst& k, double inv_alpha2, double stat_scale) {
  WideConst c;
  c.inv_sw = 1.0 / wide_scale_w(k);
  c.inv_sy = 1.0 / wide_scale_y(k);
  c.ia2 = inv_alpha2;
  c.scale = stat_scale;
  return c;
}

// The Eq. 1 term of one bin from its two wide words, in data units and FP64:
// Y^2 / (W + 1/alpha^2), 0 for an empty bin with no prior.
__device__ __forceinline__ double add_wide_term(double acc, uint64_t wq, uint64_t yq, const WideConst& k) {
  const double W = (double)wq * k.inv_sw;
  const double Y = (double)(int64_t)yq * k.inv_sy;
  const double d = W + k.ia2;
  return d > 0.0 ? acc + Y * (Y / d) : acc;
}

// A lane's wide histogram: slot m holds the weight word at h + 2 m 64 and the
// residual word 64 words (512 bytes) further.
constexpr int kWideSlotWords = 2 * kWave;

// Reads and clears the wide slots of bins [m0, m0 + 8) (clamped to slot M,
// which is empty by then).
__device__ __forceinline__ void take_wide_block(uint64_t* h, int M, int m0, uint64_t (&fw)[kReduceBlock],
                                                uint64_t (&fy)[kReduceBlock]) {
#pragma unroll
  for (int q = 0; q < kReduceBlock; ++q) {
    uint64_t* sl = h + min(m0 + q, M) * kWideSlotWords;
    fw[q] = lds_take(sl);
    fy[q] = lds_take(sl + kWave);
  }
}

// The part sums of the bins [part_block(p0), part_block(p1)) blocks of one
// lane's wide histogram, in the fixed order of reduce_hist (each part from
// zero, in bin order), written to out[p - p0]; the range holding block 0
// also takes the wrap slot M of the fused FP64 fold.
template <int PH, int NP>
__device__ __forceinline__ void wide_parts(uint64_t* h, int M, int p0, const WideConst& k, double (&out)[NP]) {
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  uint64_t ww = 0, wy = 0;
  if (PH == PH_FP64 && part_block(p0, nb) == 0 && part_block(p0 + NP, nb) > 0) {
    ww = lds_take(h + M * kWideSlotWords);
    wy = lds_take(h + M * kWideSlotWords + kWave);
  }
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    const int p = p0 + pp;
    double acc = 0.0;
    for (int b = part_block(p, nb); b < part_block(p + 1, nb); ++b) {
      const int m0 = b * kReduceBlock;
      uint64_t fw[kReduceBlock], fy[kReduceBlock];
      take_wide_block(h, M, m0, fw, fy);
      if (m0 == 0) {
        fw[0] += ww;  // integer sums: adding the wrap slot is exact
        fy[0] += wy;
      }
#pragma unroll
      for (int q = 0; q < kReduceBlock; ++q)
        if (m0 + q < M) acc = add_wide_term(acc, fw[q], fy[q], k);
    }
    out[pp] = acc;
  }
}

__device__ __forceinline__ CurveConst make_curve_const(const PrepConst& k, double inv_alpha2, float stat_scale) {
  CurveConst c;
  c.kc = (float)(k.s_w / (k.s_y * k.s_y));
  c.ia2q = fmaxf((float)(inv_alpha2 * k.s_w), kMinPrior);  // see add_bin_term
  c.scale = stat_scale;
  c.pad = 0.f;
  return c;
}

}  // namespace dev
}  // namespace fpw
