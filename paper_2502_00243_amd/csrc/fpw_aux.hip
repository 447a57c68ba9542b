// Auxiliary HIP kernels of libfpw: the per-curve prepare pass, the
// per-curve peak merge, peak selection over a stored periodogram, the plain
// FP64 comparator and the bin parity hook.
#include "fpw_common.h"

// histogram slots per wave of the entropy kernel: FPW_MAX_BINS + 1
#define FPW_ENTROPY_MAX_SLOTS 256

namespace fpw {
namespace {

using namespace dev;

// ---------------------------------------------------------------- chunk merge
// One wave per (curve, variant).
template <int K>
__global__ __launch_bounds__(256) void merge_kernel(MergeArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int gw = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (gw >= a.n_curves * a.n_var) return;  // wave-uniform
  const int v = gw / a.n_curves, c = gw - v * a.n_curves;
  merge_curve<K>(a, c, v, lane);
}

// One workgroup of four waves per (curve, variant), for curves cut into many
// chunks (the fused pass): the chunks' loads are spread over 256 lanes.
constexpr int kMergeGroupWaves = 4;

template <int K>
__global__ __launch_bounds__(kMergeGroupWaves * kWave) void merge_group_kernel(MergeArgs a) {
  __shared__ float lv[kMergeGroupWaves * K];
  __shared__ int32_t li[kMergeGroupWaves * K];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int v = blockIdx.x / a.n_curves, c = blockIdx.x - v * a.n_curves;
  merge_curve_group<K, kMergeGroupWaves>(a, c, v, wave, lane, lv, li);
}

// ---------------------------------------------------------------- top-k over a stored periodogram
// One workgroup of 8 waves per curve: the waves stride over the curve's
// periodogram (coalesced), each keeps per-lane lists and selects its best k,
// and the first wave selects the curve's k from the 8 x k candidates.
constexpr int kTopkWaves = 8;

template <int K>
__global__ __launch_bounds__(kTopkWaves * kWave) void topk_kernel(TopkArgs a) {
  __shared__ float cand_v[kTopkWaves * K];
  __shared__ int32_t cand_i[kTopkWaves * K];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int c = blockIdx.x;
  const float* S = a.S + (int64_t)c * a.n_freq;
  TopList<K> l;
  l.init();
  for (int k = threadIdx.x; k < a.n_freq; k += kTopkWaves * kWave) {
    const float s = S[k];
    const float left = k > 0 ? S[k - 1] : -INFINITY;
    const float right = k + 1 < a.n_freq ? S[k + 1] : -INFINITY;
    l.insert(s, k, s > left && s >= right);
  }
  wave_select<K>(l, a.k, cand_v + wave * K, cand_i + wave * K, lane);
  __syncthreads();
  if (wave == 0) {
    TopList<K> m;
    m.init();
    for (int q = lane; q < kTopkWaves * a.k; q += kWave) {
      const int w = q / a.k, r = q - w * a.k;
      const int ci = cand_i[w * K + r];
      m.insert(cand_v[w * K + r], ci, ci >= 0);
    }
    wave_select<K>(m, a.k, a.out_val + (int64_t)c * a.k, a.out_idx + (int64_t)c * a.k, lane);
  }
}

// ---------------------------------------------------------------- prepare
// One workgroup per curve: inverse variances, centring, time offsets and the
// fixed-point scales (curve_prep), then the packed records and the FP64
// arrays of the plain comparator.
// Curves in the wide format (fmt) also get their 32-byte records and FP64
// constants.
__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(PrepArgs a) {
  __shared__ double red[kPrepRed];
  const int t = threadIdx.x;
  // the queue counters of the pass's fold kernels
  if (a.queue != nullptr && blockIdx.x == 0 && t < a.n_queues) a.queue[t] = 0u;
  for (int64_t c = blockIdx.x; c < a.n_curves; c += gridDim.x) {
    const int64_t p0 = a.offsets[c];
    const int n = (int)(a.offsets[c + 1] - p0);
    const PrepConst k = curve_prep(a.t + p0, a.y + p0, a.dy + p0, n, a.center, a.tref_mode, a.t_ref, red);
    const bool wide = a.fmt != nullptr && a.fmt[c] == FMT_WIDE;  // workgroup-uniform
    const int64_t q0 = wide ? a.offw[c] : 0;
    for (int i = t; i < n; i += kPrepThreads) {
      const int64_t p = p0 + i;
      a.rec[p] = make_rec(a.t[p], a.y[p], a.dy[p], k, a.phase);
      if (wide) a.recw[q0 + i] = make_wrec(a.t[p], a.y[p], a.dy[p], k, a.phase);
      const double d = a.dy[p];
      const double w = 1.0 / (d * d);
      a.tau64[p] = a.t[p] - k.tref;
      a.w64[p] = w;
      a.wx64[p] = w * (a.y[p] - k.mu);
    }
    if (t == 0) {
      a.cc[c] = make_curve_const(k, a.inv_alpha2, a.stat_scale);
      if (wide) a.wc[c] = make_wide_const(k, a.inv_alpha2, a.stat_scale);
    }
  }
}

// Fixed-tree workgroup reductions of the shared-timestamp and baseline
// prepare kernels.
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

// ---------------------------------------------------------------- prepare, shared timestamps
// One workgroup per curve of a shared-timestamp batch: inverse variances and
// centring as above, fixed-point scales with 30-bit ranges (every bin sum of
// either quantity stays below 2^30 in magnitude), then the four signed
// base-256 digits of each quantity scattered into the curve's rows of the
// int8 tiles.
// Writes the digits of v to four consecutive tile rows (16 bytes apart).
__device__ __forceinline__ void put_digits(int8_t* tile_row, int32_t v, int) {
  // v = d0 + 256 d1 + 65536 d2 + 2^24 d3, each d in [-128, 127] for |v| <= 2^30
  int32_t r = v;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int32_t d = (int32_t)(int8_t)(r & 0xff);
    tile_row[i * 16] = (int8_t)d;
    r = (r - d) >> 8;
  }
  tile_row[3 * 16] = (int8_t)r;
}

__global__ __launch_bounds__(kPrepThreads) void prepare_shared_kernel(SharedPrepArgs a) {
  __shared__ double red[kPrepThreads];
  const int t = threadIdx.x;
  const int n = a.n_points;
  for (int c = blockIdx.x; c < a.n_curves; c += gridDim.x) {
    const double* y = a.y + (int64_t)c * n;
    const double* dy = a.dy + (int64_t)c * n;
    double sw = 0.0, swy = 0.0, sy = 0.0;
    for (int i = t; i < n; i += kPrepThreads) {
      const double w = 1.0 / (dy[i] * dy[i]);
      sw += w;
      swy += w * y[i];
      sy += y[i];
    }
    sw = block_sum(sw, red);
    swy = block_sum(swy, red);
    sy = block_sum(sy, red);
    const double mu = a.center == 0 ? swy / sw : (a.center == 1 ? sy / (double)n : 0.0);
    double ay = 0.0;
    for (int i = t; i < n; i += kPrepThreads) {
      const double w = 1.0 / (dy[i] * dy[i]);
      ay += fabs(w * (y[i] - mu));
    }
    ay = block_sum(ay, red);
    const double s_w = (1073741824.0 - 2.0 - 2.0 * (double)n) / sw;
    const double s_y = ay > 0.0 ? (1073741824.0 - 2.0 - (double)n) / ay : 1.0;
    // rows of curve `sub` of its group: 8 (2 (sub / 2) + q) + 4 (sub % 2) + digit
    const int g = c / kSharedGroupCurves, sub = c % kSharedGroupCurves;
    const int row0 = 16 * (sub >> 1) + 4 * (sub & 1);
    for (int i = t; i < n; i += kPrepThreads) {
      const double w = 1.0 / (dy[i] * dy[i]);
      const double wx = w * (y[i] - mu);
      const int32_t wq = (int32_t)fmax(1.0, rint(w * s_w));
      const int32_t yq = (int32_t)rint(wx * s_y);
      const int kb = i >> 5, h = (i >> 4) & 1, j = i & 15;
      int8_t* base = a.vals + ((int64_t)g * a.n_kblocks + kb) * kSharedTileBytes + (32 * h + row0) * 16 + j;
      put_digits(base, wq, 0);
      put_digits(base + 8 * 16, yq, 0);
    }
    if (t == 0) {
      CurveConst k;
      k.kc = (float)(s_w / (s_y * s_y));
      k.ia2q = fmaxf((float)(a.inv_alpha2 * s_w), kMinPrior);  // see add_bin_term
      k.scale = a.stat_scale;
      k.pad = 0.f;
      a.cc[c] = k;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- prepare, marginalised baseline
// One workgroup per curve: weights, centring and time offsets as above;
// Chebyshev terms T_1 = s, T_2 = 2 s^2 - 1 of s = 2 (t - t_min)/(t_max - t_min) - 1;
// fixed-point weight, residual and w T_k; then the per-curve constants from
// the rounded values: H = I + beta^2 [sum a_k a_l / w~] (a_0 = w~) and
// g = H^-1 beta [sum a_k y~ / w~], solved in FP64.

// x = Q^-1 b for a symmetric positive definite 3x3 Q (upper triangle q00 q01 q02 q11 q12 q22),
// by elimination without pivoting.
__device__ __forceinline__ void spd3_solve(const double* q, const double* b, double* x) {
  const double a00 = q[0], a01 = q[1], a02 = q[2];
  const double l1 = a01 / a00, l2 = a02 / a00;
  const double a11 = q[3] - l1 * a01, a12 = q[4] - l1 * a02, a22 = q[5] - l2 * a02;
  const double m2 = a12 / a11;
  const double c22 = a22 - m2 * a12;
  const double y0 = b[0], y1 = b[1] - l1 * y0, y2 = b[2] - l2 * y0 - m2 * (b[1] - l1 * y0);
  x[2] = y2 / c22;
  x[1] = (y1 - a12 * x[2]) / a11;
  x[0] = (y0 - a01 * x[1] - a02 * x[2]) / a00;
}

__device__ __forceinline__ double block_max(double v, double* red) { return -block_min(-v, red); }

__global__ __launch_bounds__(kPrepThreads) void bm_prepare_kernel(BmPrepArgs a) {
  __shared__ double red[kPrepThreads];
  const int t = threadIdx.x;
  if (a.queue != nullptr && blockIdx.x == 0 && t == 0) *a.queue = 0u;  // the next fold kernel's queue counter
  for (int64_t c = blockIdx.x; c < a.n_curves; c += gridDim.x) {
    const int64_t p0 = a.offsets[c];
    const int n = (int)(a.offsets[c + 1] - p0);
    double sw = 0.0, swy = 0.0, sy = 0.0, tmin = INFINITY, tmax = -INFINITY;
    for (int i = t; i < n; i += kPrepThreads) {
      const double d = a.dy[p0 + i];
      const double w = 1.0 / (d * d);
      const double yy = a.y[p0 + i];
      sw += w;
      swy += w * yy;
      sy += yy;
      tmin = fmin(tmin, a.t[p0 + i]);
      tmax = fmax(tmax, a.t[p0 + i]);
    }
    sw = block_sum(sw, red);
    swy = block_sum(swy, red);
    sy = block_sum(sy, red);
    tmin = block_min(tmin, red);
    tmax = block_max(tmax, red);
    const double mu = a.center == 0 ? swy / sw : (a.center == 1 ? sy / (double)n : 0.0);
    const double tref = a.tref_mode == 0 ? 0.0 : (a.tref_mode == 1 ? tmin : a.t_ref);
    const double span = tmax - tmin;
    double ay = 0.0;
    for (int i = t; i < n; i += kPrepThreads) {
      const double d = a.dy[p0 + i];
      const double w = 1.0 / (d * d);
      ay += fabs(w * (a.y[p0 + i] - mu));
    }
    ay = block_sum(ay, red);
    const double s_w = (4294967296.0 - 2.0 - 2.0 * (double)n) / sw;
    const double s_y = ay > 0.0 ? (2147483648.0 - 2.0 - (double)n) / ay : 1.0;
    const double s_z = (2147483648.0 - 2.0 - (double)n) / sw;  // |w T_k| <= w
    // sums of the rounded values: h[0..5] (upper triangle of sum a_k a_l / w~), z[0..2]
    double h[6] = {0, 0, 0, 0, 0, 0}, z[3] = {0, 0, 0};
    for (int i = t; i < n; i += kPrepThreads) {
      const int64_t p = p0 + i;
      const double d = a.dy[p];
      const double w = 1.0 / (d * d);
      const double wx = w * (a.y[p] - mu);
      const double sc = span > 0.0 ? 2.0 * (a.t[p] - tmin) / span - 1.0 : 0.0;
      const double T1 = a.n_terms >= 2 ? sc : 0.0;
      const double T2 = a.n_terms >= 3 ? 2.0 * sc * sc - 1.0 : 0.0;
      const double wqd = fmax(1.0, rint(w * s_w));
      const int64_t yq = (int64_t)rint(wx * s_y);
      const int64_t z1 = (int64_t)rint(w * T1 * s_z);
      const int64_t z2 = (int64_t)rint(w * T2 * s_z);
      Rec r;
      r.tau_bits = (uint64_t)__double_as_longlong(a.t[p] - tref);
      r.pk = ((uint64_t)wqd << 32) + (uint64_t)yq;
      a.rec[p] = r;
      if (a.n_terms >= 3) a.z64[p] = (uint64_t)(z2 * 4294967296LL + z1);
      if (a.n_terms == 2) a.z32[p] = (uint32_t)z1;
      const double wt = wqd / s_w, yt = (double)yq / s_y, a1 = (double)z1 / s_z, a2 = (double)z2 / s_z;
      h[0] += wt;
      h[1] += a1;
      h[2] += a2;
      h[3] += a1 * a1 / wt;
      h[4] += a1 * a2 / wt;
      h[5] += a2 * a2 / wt;
      z[0] += yt;
      z[1] += a1 * yt / wt;
      z[2] += a2 * yt / wt;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) h[q] = block_sum(h[q], red);
#pragma unroll
    for (int q = 0; q < 3; ++q) z[q] = block_sum(z[q], red);
    if (t == 0) {
      BaseConst b;
      const double b2 = a.beta * a.beta;
      // rows of absent terms are the identity, so they leave g and S unchanged
      b.H[0] = 1.0 + b2 * h[0];
      b.H[1] = b2 * h[1];
      b.H[2] = b2 * h[2];
      b.H[3] = 1.0 + b2 * h[3];
      b.H[4] = b2 * h[4];
      b.H[5] = 1.0 + b2 * h[5];
      const double zb[3] = {a.beta * z[0], a.beta * z[1], a.beta * z[2]};
      spd3_solve(b.H, zb, b.g);
      b.inv_sw = 1.0 / s_w;
      b.inv_sy = 1.0 / s_y;
      b.inv_sz = 1.0 / s_z;
      b.beta = a.beta;
      b.ia2 = a.inv_alpha2;
      b.scale = a.stat_scale;
      a.bc[c] = b;
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
  fo.init(a.freqs[k < a.n_freq ? k : a.n_freq - 1], M, 0.0);
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
    fo.init(a.freqs[a.f_begin + fi], a.n_bins, a.fold_nh);
    int b = fo.bin(encode_tau(a.tau64[a.p0 + i], PH));
    if (PH == PH_FP64 && b == a.n_bins) b = 0;
    a.out[g] = b;
  }
}

// ---------------------------------------------------------------- phase entropy (App. C)
// One wave per (curve, slot): the curve's observations are binned at the
// slot's frequency with the plan's fold, counted with LDS atomics in a
// per-wave histogram, and H = -sum p log p is reduced across the wave in FP64.
constexpr int kEntropyWaves = 4;

template <int PH>
__global__ __launch_bounds__(kEntropyWaves * 64) void entropy_kernel(EntropyArgs a) {
  __shared__ uint32_t cnt[kEntropyWaves][FPW_ENTROPY_MAX_SLOTS];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int gw = blockIdx.x * kEntropyWaves + wv;
  if (gw >= a.n_curves * a.k) return;  // wave-uniform
  const int c = gw / a.k;
  const int idx = a.freq_idx[gw];
  if (idx < 0 || idx >= a.n_freq) {
    if (lane == 0) {
      a.H[gw] = NAN;
      a.E[gw] = NAN;
      a.V[gw] = NAN;
    }
    return;
  }
  const int M = a.n_bins;
  for (int m = lane; m <= M; m += kWave) cnt[wv][m] = 0;
  const int64_t p0 = a.offsets[c];
  const int n = (int)(a.offsets[c + 1] - p0);
  Folder<PH> fo;
  fo.init(a.freqs[idx], M, a.fold_nh);
  for (int i = lane; i < n; i += kWave) {
    int b = fo.bin(encode_tau(a.tau64[p0 + i], PH));
    if (b >= M) b = 0;  // the fused fold files phases just below 1 as M
    atomicAdd(&cnt[wv][b], 1u);
  }
  double h = 0.0;
  const double inv_n = 1.0 / (double)n;
  for (int m = lane; m < M; m += kWave) {
    const uint32_t nm = cnt[wv][m];
    if (nm > 0) {
      const double p = (double)nm * inv_n;
      h -= p * log(p);
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) h += __shfl_xor(h, off);
  if (lane == 0) {
    const double Md = M, Nd = n;
    a.H[gw] = (float)h;
    a.E[gw] = (float)(log(Md) - (Md - 1.0) / (2.0 * Nd) - (Md - 1.0) * (Md + 1.0) / (12.0 * Nd * Nd));
    a.V[gw] = (float)((Md - 1.0) / (2.0 * Nd * Nd) + (Md * Md - 1.0) / (6.0 * Nd * Nd * Nd));
  }
}

}  // namespace

hipError_t launch_prepare(const PrepArgs& a, hipStream_t s) {
  const int64_t g = a.n_curves < 65536 ? a.n_curves : 65536;
  hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)g), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prepare_shared(const SharedPrepArgs& a, hipStream_t s) {
  const int g = a.n_curves < 65536 ? a.n_curves : 65536;
  hipLaunchKernelGGL(prepare_shared_kernel, dim3((unsigned)g), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bm_prepare(const BmPrepArgs& a, hipStream_t s) {
  const int64_t g = a.n_curves < 65536 ? a.n_curves : 65536;
  hipLaunchKernelGGL(bm_prepare_kernel, dim3((unsigned)g), dim3(kPrepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s, bool group) {
  if (group) {
    const dim3 grid((unsigned)(a.n_curves * a.n_var)), block(kMergeGroupWaves * kWave);
    if (a.topk <= 8)
      hipLaunchKernelGGL(merge_group_kernel<8>, grid, block, 0, s, a);
    else
      hipLaunchKernelGGL(merge_group_kernel<16>, grid, block, 0, s, a);
    return hipGetLastError();
  }
  const int blocks = (a.n_curves * a.n_var + 3) / 4;
  if (a.topk <= 8)
    hipLaunchKernelGGL(merge_kernel<8>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(merge_kernel<16>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_topk(const TopkArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)a.n_curves), block(kTopkWaves * kWave);
  if (a.k <= 8)
    hipLaunchKernelGGL(topk_kernel<8>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(topk_kernel<16>, grid, block, 0, s, a);
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

namespace fpw {

hipError_t launch_entropy(const EntropyArgs& a, hipStream_t s) {
  const int waves = a.n_curves * a.k;
  const int blocks = (waves + kEntropyWaves - 1) / kEntropyWaves;
  switch (a.phase) {
    case PH_FP64: hipLaunchKernelGGL(entropy_kernel<PH_FP64>, dim3(blocks), dim3(kEntropyWaves * 64), 0, s, a); break;
    case PH_LISTING: hipLaunchKernelGGL(entropy_kernel<PH_LISTING>, dim3(blocks), dim3(kEntropyWaves * 64), 0, s, a); break;
    case PH_DF32: hipLaunchKernelGGL(entropy_kernel<PH_DF32>, dim3(blocks), dim3(kEntropyWaves * 64), 0, s, a); break;
    default: hipLaunchKernelGGL(entropy_kernel<PH_FP32>, dim3(blocks), dim3(kEntropyWaves * 64), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace fpw
