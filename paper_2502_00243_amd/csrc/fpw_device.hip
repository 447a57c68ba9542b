// HIP kernels of the FPW periodogram for CDNA4 (gfx950).
//
// Statistic (Eq. 1 of Finkbeiner, Prince & Whitebook): for each light curve
// and trial frequency f, observations are folded into M phase bins
// (App. A phase-bin equation), the per-bin sums W_m = sum w and
// Y_m = sum w x are accumulated (App. A sparse form) and reduced to
// S = sum_m Y_m^2 / (W_m + 1/alpha^2).  Peaks of S over f are then selected
// (Sec. 3.5).
//
// Mapping to the chip:
//  * one lane = one trial frequency; a wave sweeps 64 (or 128) consecutive
//    frequencies of one curve, so every observation is wave-uniform and is
//    fetched once per wave through the scalar cache into SGPRs;
//  * each lane owns a private histogram of M+1 packed 64-bit fixed-point
//    words in LDS, laid out [bin][lane] so the 64 lanes of a wave always hit
//    distinct banks whatever their bins are;
//  * one `ds_add_u64` per (observation, frequency) accumulates both sums
//    exactly: the weight sits in the high word, the weighted residual in the
//    low word, and integer addition carries them without rounding;
//  * the phase is formed in FP64 (full rate on CDNA), and the bin index
//    comes out of the low word of one more FP64 fma, so a fold costs three
//    FP64 instructions plus the LDS address;
//  * work is a queue of (curve, frequency chunk) items, longest curves first,
//    popped by persistent waves with one atomic each; the peak selection is
//    fused so that large periodograms never reach HBM.
#include <float.h>
#include <math.h>

#include "fpw_internal.h"

namespace fpw {
namespace {

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

// FP64, fused: the fold is shifted by half a bin, phase' = frac(tau f - 1/(2M)),
// and round(M phase') (one fma into the magic constant) equals
// floor(M frac(tau f)) except within rounding of an edge; phase' just below 1
// rounds to M, which is bin 0.  tau f - 1/(2M) is formed with one rounding
// (fma), so the bin is exact up to ~M * ulp(tau f) bin widths.
template <>
struct Folder<PH_FP64> {
  double f, nh, md;
  __device__ __forceinline__ void init(double freq, int M) {
    f = freq;
    md = (double)M;
    nh = -0.5 / (double)M;
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
  __device__ __forceinline__ void init(double freq, int M) {
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
  __device__ __forceinline__ void init(double freq, int M) {
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
    const float fr = ph - floorf(ph);        // exact: ph < 2^23
    const float uh = mf * fr;
    const float ul = __builtin_fmaf(mf, fr, -uh);  // uh + ul = M*fr exactly
    const float c = __builtin_fmaf(mf, pl, ul);
    const float b0 = floorf(uh);
    const float r = (uh - b0) + c;           // uh - b0 exact
    int b = (int)b0 + (int)floorf(r);
    b = b % m;
    return b < 0 ? b + m : b;
  }
};

// Naive FP32 product, for the precision study only.
template <>
struct Folder<PH_FP32> {
  float f, mf;
  int m;
  __device__ __forceinline__ void init(double freq, int M) {
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

// ---------------------------------------------------------------- LDS histograms
__device__ __forceinline__ void lds_add(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t lds_take(uint64_t* p) {
  return __hip_atomic_exchange(p, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Eq. 1 term of one bin from its packed fixed-point word: Y_q^2 / (W_q + ia2q).
__device__ __forceinline__ float bin_term(uint64_t v, float ia2q) {
  const uint32_t l = lo32(v);
  const int32_t yq = (int32_t)l;
  const uint32_t wq = hi32(v) + (l >> 31);  // undo the borrow of a negative low word
  const float d = (float)wq + ia2q;
  const float yf = (float)yq;
  const float t = yf * (yf * __builtin_amdgcn_rcpf(d));
  return d > 0.f ? t : 0.f;
}

// Reads and clears one lane's histogram (slot m at h + 64 m) and returns
// sum_m Y_m^2 / (W_m + 1/alpha^2) in fixed-point units.
template <int PH>
__device__ __forceinline__ float reduce_hist(uint64_t* h, int M, float ia2q) {
  uint64_t v0 = lds_take(h);
  if (PH == PH_FP64) v0 += lds_take(h + M * kWave);
  float acc = bin_term(v0, ia2q);
  for (int m = 1; m < M; ++m) acc += bin_term(lds_take(h + m * kWave), ia2q);
  return acc;
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

// Merges the 64 lanes' lists: writes the `k` best (value, index) of the wave,
// best first; missing entries are (-inf, -1).  Every lane must call it.
template <int K>
__device__ __forceinline__ void wave_select(TopList<K>& l, int k, float* out_v, int32_t* out_i, int lane) {
  for (int r = 0; r < k; ++r) {
    float bv = l.v[0];
    int bi = l.i[0];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    const bool none = bv == -INFINITY;
    if (lane == 0) {
      out_v[r] = bv;
      out_i[r] = none ? -1 : bi;
    }
    if (!none && l.i[0] == bi) l.pop_front();
  }
}

// ---------------------------------------------------------------- batched kernel
// Read-only inputs of the batched kernel.  They are separate __restrict__
// kernel arguments so that the compiler may fetch them through the scalar
// cache (nothing the kernel writes can alias them).
struct RO {
  const Rec* __restrict__ rec;
  const int64_t* __restrict__ offsets;
  const CurveConst* __restrict__ cc;
  const double* __restrict__ freqs;
};

template <int PH, int FL, int KC>
__device__ __forceinline__ void process_item(const BatchArgs& a, const RO& ro, const Item& item, uint64_t* hist,
                                             int lane) {
  const int M = a.n_bins;
  const int slots = M + 1;
  const int c = item.curve, k0 = item.k0, k1 = item.k1;
  const int64_t p0 = ro.offsets[c];
  const int n = (int)(ro.offsets[c + 1] - p0);
  const Rec* __restrict__ rc = ro.rec + p0;
  const CurveConst cc = ro.cc[c];
  const float outscale = cc.kc * cc.scale;

  constexpr int KL = KC > 0 ? KC : 1;
  TopList<KL> list;
  if (KC > 0) list.init();
  float pend_s = -INFINITY, pend_left = -INFINITY;  // S at kb-1 and kb-2 (wave-uniform)
  bool pend = false;                                 // index kb-1 still waits for its right neighbour

  for (int kt = k0; kt < k1; kt += FL * kWave) {
    Folder<PH> fo[FL];
    uint64_t* h[FL];
#pragma unroll
    for (int j = 0; j < FL; ++j) {
      const int k = kt + j * kWave + lane;
      fo[j].init(ro.freqs[k < k1 ? k : k1 - 1], M);
      h[j] = hist + (j * slots) * kWave + lane;
    }
    // fold, bin and accumulate every observation of the curve
    int i = 0;
    for (; i + kBatch <= n; i += kBatch) {
      Rec r[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) r[q] = rc[i + q];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
#pragma unroll
        for (int j = 0; j < FL; ++j) lds_add(h[j] + fo[j].bin(r[q].tau_bits) * kWave, r[q].pk);
      }
    }
    for (; i < n; ++i) {
      const Rec r = rc[i];
#pragma unroll
      for (int j = 0; j < FL; ++j) lds_add(h[j] + fo[j].bin(r.tau_bits) * kWave, r.pk);
    }
    // reduce each sub-tile of 64 frequencies, store, and pick peaks
#pragma unroll
    for (int j = 0; j < FL; ++j) {
      const int kb = kt + j * kWave;
      if (kb >= k1) break;
      const float s = outscale * reduce_hist<PH>(h[j], M, cc.ia2q);
      const int k = kb + lane;
      const bool valid = k < k1;
      if (a.S != nullptr && valid) a.S[(int64_t)c * a.n_freq + k] = s;
      if (KC > 0) {
        const float sv = valid ? s : -INFINITY;
        const float up = __shfl_up(sv, 1);
        const float dn = __shfl_down(sv, 1);
        // index kb-1 (lane 63 of the previous sub-tile) now has its right neighbour
        const float s0 = __shfl(sv, 0);
        if (pend) list.insert(pend_s, kb - 1, lane == kWave - 1 && pend_s > pend_left && pend_s >= s0);
        // left neighbour, or "undecided" at a chunk start that is not frequency 0
        float left = up;
        bool decided = valid;
        if (lane == 0) {
          if (kb == k0) {
            left = -INFINITY;
            decided = decided && k0 == 0;
          } else {
            left = pend_s;
          }
        }
        // right neighbour: the chunk end, or the next sub-tile for lane 63
        float right = dn;
        const bool last_of_chunk = k == k1 - 1;
        if (last_of_chunk) {
          right = -INFINITY;
          decided = decided && k1 == a.n_freq;
        } else if (lane == kWave - 1) {
          decided = false;  // deferred to the next sub-tile
        }
        list.insert(s, k, decided && s > left && s >= right);
        // carry lane 63 (and 62) forward
        pend_s = __shfl(sv, kWave - 1);
        pend_left = __shfl(sv, kWave - 2);
        pend = kb + kWave - 1 < k1 - 1;
        // chunk-edge values for the merge
        if (valid) {
          float* e = a.edge + (int64_t)item.slot * 4;
          if (k == k0) {
            e[0] = s;
            if (k0 + 1 >= k1) e[1] = -INFINITY;
            if (k1 - 2 < k0) e[2] = -INFINITY;
          }
          if (k == k0 + 1) e[1] = s;
          if (k == k1 - 2) e[2] = s;
          if (k == k1 - 1) e[3] = s;
        }
      }
    }
  }
  if (KC > 0) {
    wave_select<KL>(list, a.topk, a.cand_val + (int64_t)item.slot * a.topk, a.cand_idx + (int64_t)item.slot * a.topk, lane);
  }
}

template <int PH, int FL, int KC>
__global__ __launch_bounds__(256) void batched_kernel(BatchArgs a, const Rec* __restrict__ rec,
                                                      const int64_t* __restrict__ offsets,
                                                      const CurveConst* __restrict__ ccs,
                                                      const double* __restrict__ freqs,
                                                      const Item* __restrict__ items) {
  const RO ro{rec, offsets, ccs, freqs};
  extern __shared__ __align__(16) uint64_t lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int slots = a.n_bins + 1;
  uint64_t* hist = lds + (size_t)wave * FL * slots * kWave;  // this wave's histograms: [j][bin][lane]
  for (int s = 0; s < FL * slots; ++s) hist[s * kWave + lane] = 0;
  for (;;) {
    int it = 0;
    if (lane == 0) it = (int)atomicAdd(a.queue, 1u);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= a.n_items) break;
    const Item item = items[it];
    process_item<PH, FL, KC>(a, ro, item, hist, lane);
  }
  // The last wave out resets the queue, so the next launch (or graph replay)
  // starts from zero without a memset.
  if (lane == 0) {
    __threadfence();
    const uint32_t total = gridDim.x * (blockDim.x / kWave);
    if (atomicAdd(a.queue + 1, 1u) == total - 1) {
      atomicExch(a.queue, 0u);
      atomicExch(a.queue + 1, 0u);
    }
  }
}

// ---------------------------------------------------------------- chunk merge
template <int K>
__global__ __launch_bounds__(256) void merge_kernel(MergeArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_curves) return;
  TopList<K> l;
  l.init();
  const int q0 = a.curve_slot[c], q1 = a.curve_slot[c + 1];
  for (int q = q0; q < q1; ++q) {
    for (int r = 0; r < a.topk; ++r) {
      const int ci = a.cand_idx[(int64_t)q * a.topk + r];
      l.insert(a.cand_val[(int64_t)q * a.topk + r], ci, ci >= 0);
    }
    if (q > q0) {
      // indices b = k0 of this chunk and b-1 = last of the previous one
      const int b = a.slot_k0[q];
      const float* ep = a.edge + (int64_t)(q - 1) * 4;
      const float* eq = a.edge + (int64_t)q * 4;
      const float sa_left = ep[2], sa = ep[3], sb = eq[0], sb_right = eq[1];
      l.insert(sa, b - 1, sa > sa_left && sa >= sb);
      l.insert(sb, b, sb > sa && sb >= sb_right);
    }
  }
  for (int r = 0; r < a.topk; ++r) {
    const bool none = l.v[r] == -INFINITY;
    a.out_val[(int64_t)c * a.topk + r] = l.v[r];
    a.out_idx[(int64_t)c * a.topk + r] = none ? -1 : l.i[r];
  }
}

// ---------------------------------------------------------------- top-k over a stored periodogram
template <int K>
__global__ __launch_bounds__(256) void topk_kernel(TopkArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (c >= a.n_curves) return;  // wave-uniform
  const float* S = a.S + (int64_t)c * a.n_freq;
  TopList<K> l;
  l.init();
  for (int k = lane; k < a.n_freq; k += kWave) {
    const float s = S[k];
    const float left = k > 0 ? S[k - 1] : -INFINITY;
    const float right = k + 1 < a.n_freq ? S[k + 1] : -INFINITY;
    l.insert(s, k, s > left && s >= right);
  }
  wave_select<K>(l, a.k, a.out_val + (int64_t)c * a.k, a.out_idx + (int64_t)c * a.k, lane);
}

// ---------------------------------------------------------------- prepare
// One workgroup per curve: inverse variances, centring, time offsets and the
// fixed-point scales, then the packed records.  Reductions use a fixed tree,
// so results are deterministic.
constexpr int kPrepThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  __syncthreads();
  red[t] = v;
  __syncthreads();
  for (int s = kPrepThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = red[t] + red[t + s];
    __syncthreads();
  }
  return red[0];
}
__device__ __forceinline__ double block_min(double v, double* red) {
  const int t = threadIdx.x;
  __syncthreads();
  red[t] = v;
  __syncthreads();
  for (int s = kPrepThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmin(red[t], red[t + s]);
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(PrepArgs a) {
  __shared__ double red[kPrepThreads];
  const int t = threadIdx.x;
  for (int64_t c = blockIdx.x; c < a.n_curves; c += gridDim.x) {
    const int64_t p0 = a.offsets[c];
    const int n = (int)(a.offsets[c + 1] - p0);
    double sw = 0.0, swy = 0.0, sy = 0.0, tmin = INFINITY;
    for (int i = t; i < n; i += kPrepThreads) {
      const double d = a.dy[p0 + i];
      const double w = 1.0 / (d * d);
      const double yy = a.y[p0 + i];
      sw += w;
      swy += w * yy;
      sy += yy;
      tmin = fmin(tmin, a.t[p0 + i]);
    }
    sw = block_sum(sw, red);
    swy = block_sum(swy, red);
    sy = block_sum(sy, red);
    tmin = block_min(tmin, red);
    const double mu = a.center == 0 ? swy / sw : (a.center == 1 ? sy / (double)n : 0.0);
    const double tref = a.tref_mode == 0 ? 0.0 : (a.tref_mode == 1 ? tmin : a.t_ref);
    double ay = 0.0;
    for (int i = t; i < n; i += kPrepThreads) {
      const double d = a.dy[p0 + i];
      const double w = 1.0 / (d * d);
      ay += fabs(w * (a.y[p0 + i] - mu));
    }
    ay = block_sum(ay, red);
    // Fixed-point scales: sum of |weights| < 2^32 and sum of |w x| < 2^31 for
    // any subset of points, so no bin sum can leave its 32-bit field.
    const double s_w = (4294967296.0 - 2.0 - 2.0 * (double)n) / sw;
    const double s_y = ay > 0.0 ? (2147483648.0 - 2.0 - (double)n) / ay : 1.0;
    for (int i = t; i < n; i += kPrepThreads) {
      const int64_t p = p0 + i;
      const double d = a.dy[p];
      const double w = 1.0 / (d * d);
      const double wx = w * (a.y[p] - mu);
      const double tau = a.t[p] - tref;
      const double wqd = fmax(1.0, rint(w * s_w));
      const uint64_t wq = (uint64_t)wqd;
      const int64_t yq = (int64_t)rint(wx * s_y);
      Rec r;
      r.tau_bits = encode_tau(tau, a.phase);
      r.pk = (wq << 32) + (uint64_t)yq;
      a.rec[p] = r;
      a.tau64[p] = tau;
      a.w64[p] = w;
      a.wx64[p] = wx;
    }
    if (t == 0) {
      CurveConst k;
      k.kc = (float)(s_w / (s_y * s_y));
      k.ia2q = (float)(a.inv_alpha2 * s_w);
      k.scale = a.stat_scale;
      k.pad = 0.f;
      a.cc[c] = k;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- plain FP64 comparator
// One launch per curve, one lane per frequency, FP64 histograms in LDS
// ([bin][lane], ds_add_f64), listing-order fold, IEEE division.
__global__ __launch_bounds__(64) void fp64_kernel(Fp64Args a) {
  extern __shared__ __align__(16) double hist64[];
  const int lane = threadIdx.x;
  const int M = a.n_bins;
  double* Wh = hist64 + lane;
  double* Yh = hist64 + M * kWave + lane;
  for (int m = 0; m < M; ++m) {
    Wh[m * kWave] = 0.0;
    Yh[m * kWave] = 0.0;
  }
  const int k = blockIdx.x * kWave + lane;
  Folder<PH_LISTING> fo;
  fo.init(a.freqs[k < a.n_freq ? k : a.n_freq - 1], M);
  const double* tau = a.tau + a.p0;
  const double* w = a.w + a.p0;
  const double* wx = a.wx + a.p0;
  for (int i = 0; i < a.n; ++i) {
    const int b = fo.bin((uint64_t)__double_as_longlong(tau[i]));
    __hip_atomic_fetch_add(Wh + b * kWave, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(Yh + b * kWave, wx[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  double s = 0.0;
  for (int m = 0; m < M; ++m) {
    const double d = Wh[m * kWave] + a.inv_alpha2;
    const double yv = Yh[m * kWave];
    if (d > 0.0) s += yv * yv / d;
  }
  if (k < a.n_freq) a.S[k] = a.scale * s;
}

// ---------------------------------------------------------------- bins (parity hook)
template <int PH>
__global__ __launch_bounds__(256) void bins_kernel(BinsArgs a) {
  const int64_t nf = a.f_end - a.f_begin;
  const int64_t total = nf * a.n;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t fi = g / a.n;
    const int i = (int)(g - fi * a.n);
    Folder<PH> fo;
    fo.init(a.freqs[a.f_begin + fi], a.n_bins);
    int b = fo.bin(encode_tau(a.tau64[a.p0 + i], PH));
    if (PH == PH_FP64 && b == a.n_bins) b = 0;
    a.out[g] = b;
  }
}

template <int PH, int FL, int KC>
void* batched_ptr() {
  return (void*)&batched_kernel<PH, FL, KC>;
}

template <int PH, int FL>
void* batched_ptr_k(int kc) {
  switch (kc) {
    case 0: return batched_ptr<PH, FL, 0>();
    case 8: return batched_ptr<PH, FL, 8>();
    default: return batched_ptr<PH, FL, 16>();
  }
}

void* batched_fn(int phase, int fl, int kc) {
  switch (phase) {
    case PH_FP64: return fl == 2 ? batched_ptr_k<PH_FP64, 2>(kc) : batched_ptr_k<PH_FP64, 1>(kc);
    case PH_LISTING: return fl == 2 ? batched_ptr_k<PH_LISTING, 2>(kc) : batched_ptr_k<PH_LISTING, 1>(kc);
    case PH_DF32: return batched_ptr_k<PH_DF32, 1>(kc);
    default: return batched_ptr_k<PH_FP32, 1>(kc);
  }
}

}  // namespace

int topk_capacity(int k) { return k <= 0 ? 0 : (k <= 8 ? 8 : 16); }

size_t batched_lds_bytes(const Shape& shape, int n_bins) {
  return (size_t)shape.waves_per_group * shape.freqs_per_lane * (size_t)(n_bins + 1) * kWave * sizeof(uint64_t);
}

hipError_t batched_groups_per_cu(const Shape& shape, int phase, int topk, size_t lds_bytes, int* out) {
  void* fn = batched_fn(phase, shape.freqs_per_lane, topk_capacity(topk));
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, shape.waves_per_group * kWave, lds_bytes);
}

hipError_t launch_batched(const BatchArgs& a, const Shape& shape, int phase, int grid_groups, size_t lds_bytes,
                          hipStream_t s) {
  void* fn = batched_fn(phase, shape.freqs_per_lane, topk_capacity(a.topk));
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  BatchArgs args = a;
  const Rec* rec = a.rec;
  const int64_t* offsets = a.offsets;
  const CurveConst* ccs = a.cc;
  const double* freqs = a.freqs;
  const Item* items = a.items;
  void* params[] = {&args, &rec, &offsets, &ccs, &freqs, &items};
  return hipLaunchKernel(fn, dim3(grid_groups), dim3(shape.waves_per_group * kWave), params, lds_bytes, s);
}

hipError_t launch_prepare(const PrepArgs& a, hipStream_t s) {
  const int64_t g = a.n_curves < 65536 ? a.n_curves : 65536;
  hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)g), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  const int blocks = (a.n_curves + 255) / 256;
  if (a.topk <= 8)
    hipLaunchKernelGGL(merge_kernel<8>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(merge_kernel<16>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_topk(const TopkArgs& a, hipStream_t s) {
  const int blocks = (a.n_curves + 3) / 4;
  if (a.k <= 8)
    hipLaunchKernelGGL(topk_kernel<8>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(topk_kernel<16>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fp64(const Fp64Args& a, hipStream_t s) {
  const int blocks = (a.n_freq + kWave - 1) / kWave;
  const size_t lds = (size_t)2 * a.n_bins * kWave * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)fp64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fp64_kernel, dim3(blocks), dim3(kWave), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_bins(const BinsArgs& a, hipStream_t s) {
  const int64_t total = (int64_t)(a.f_end - a.f_begin) * a.n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  switch (a.phase) {
    case PH_FP64: hipLaunchKernelGGL(bins_kernel<PH_FP64>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    case PH_LISTING: hipLaunchKernelGGL(bins_kernel<PH_LISTING>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    case PH_DF32: hipLaunchKernelGGL(bins_kernel<PH_DF32>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(bins_kernel<PH_FP32>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace fpw
