// Baseline-marginalised FPW (App. A, general case) on the general batch.
//
// The model adds a baseline drift B c (K Chebyshev terms, prior C_B = B B^T)
// to the periodic bins P and the noise.  With G = (C_B + C_sigma)^-1 (Woodbury
// on the low-rank C_B), the statistic
//     S = X^T G P (I + P^T G P)^-1 P^T G X
// reduces, with the per-bin sums W_m, Y_m and Z_mk = sum over bin m of
// w_i B_ik, to
//     v = Y - Z g,  L = diag(W + 1/alpha^2),  r = Z^T L^-1 v,  Q = H - Z^T L^-1 Z,
//     S = v^T L^-1 v + r^T Q^-1 r,
// where H = I + B^T C_sigma^-1 B and g = H^-1 B^T C_sigma^-1 X are per-curve
// constants (both terms are non-negative; Q >= I).  Z_m0 = beta W_m, so with
// K <= 3 the kernel needs one more packed 64-bit sum per bin, (Z_1, Z_2),
// accumulated with a second ds_add_u64 per (point, frequency).  The epilogue
// runs in FP64: the bin sums are exact integers and the constants were formed
// from the same rounded values (the constant direction of Q is then exactly
// the prior's 1, not a difference of two large sums).
#include "fpw_common.h"

namespace fpw {
namespace {

using namespace dev;

constexpr int kBmBatch = 4;

// slots per lane: M (weight, residual) words, then M (Z_1, Z_2) words
template <int PH>
__global__ __launch_bounds__(kWave) void bm_kernel(BmArgs a, const RecB* __restrict__ rec,
                                                   const int64_t* __restrict__ offsets,
                                                   const BaseConst* __restrict__ bcs,
                                                   const double* __restrict__ freqs,
                                                   const Item* __restrict__ items) {
  extern __shared__ __align__(16) uint64_t lds[];
  const int lane = threadIdx.x;
  const int M = a.n_bins;
  uint64_t* hw = lds + lane;                  // [m][lane]: weight and residual
  uint64_t* hz = lds + (size_t)M * kWave + lane;  // [m][lane]: w T_1 and w T_2
  for (int m = 0; m < M; ++m) {
    hw[m * kWave] = 0;
    hz[m * kWave] = 0;
  }
  for (;;) {
    int it = 0;
    if (lane == 0) it = (int)atomicAdd(a.queue, 1u);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= a.n_items) break;
    const Item item = items[it];
    const int c = item.curve, k0 = item.k0, k1 = item.k1;
    const int64_t p0 = offsets[c];
    const int n = (int)(offsets[c + 1] - p0);
    const RecB* __restrict__ rc = rec + p0;
    const BaseConst bc = bcs[c];
    for (int kt = k0; kt < k1; kt += kWave) {
      const int k = kt + lane;
      Folder<PH> fo;
      fo.init(freqs[k < k1 ? k : k1 - 1], M);
      // records are read four at a time through the scalar cache before any
      // is used, so one wait covers the batch
      int p = 0;
      for (; p + kBmBatch <= n; p += kBmBatch) {
        RecB r[kBmBatch];
#pragma unroll
        for (int q = 0; q < kBmBatch; ++q) r[q] = rc[p + q];
#pragma unroll
        for (int q = 0; q < kBmBatch; ++q) {
          const uint32_t b0 = (uint32_t)fo.bin(r[q].tau_bits);
          const uint32_t b = min(b0, b0 - (uint32_t)M);  // the fused fold reports bin 0 as M
          lds_add(hw + b * kWave, uniform_to_vgpr(r[q].pk));
          lds_add(hz + b * kWave, uniform_to_vgpr(r[q].pz));
        }
      }
      for (; p < n; ++p) {
        const RecB r = rc[p];
        const uint32_t b0 = (uint32_t)fo.bin(r.tau_bits);
        const uint32_t b = min(b0, b0 - (uint32_t)M);
        lds_add(hw + b * kWave, uniform_to_vgpr(r.pk));
        lds_add(hz + b * kWave, uniform_to_vgpr(r.pz));
      }
      // FP64 epilogue: v^T L^-1 v and the 3x3 correction
      double s1 = 0.0, r0 = 0.0, r1 = 0.0, r2 = 0.0;
      double p00 = 0.0, p01 = 0.0, p02 = 0.0, p11 = 0.0, p12 = 0.0, p22 = 0.0;
      for (int m = 0; m < M; ++m) {
        const uint64_t vw = lds_take(hw + m * kWave);
        const uint64_t vz = lds_take(hz + m * kWave);
        const uint32_t lw = lo32(vw), lz = lo32(vz);
        const uint32_t wq = hi32(vw) + (lw >> 31);
        const int32_t yq = (int32_t)lw;
        const int32_t z1q = (int32_t)lz;
        const int32_t z2q = (int32_t)(hi32(vz) + (lz >> 31));
        const double W = (double)wq * bc.inv_sw;
        const double Y = (double)yq * bc.inv_sy;
        const double Z0 = bc.beta * W;
        const double Z1 = bc.beta * ((double)z1q * bc.inv_sz);
        const double Z2 = bc.beta * ((double)z2q * bc.inv_sz);
        const double d = W + bc.ia2;
        const double inv = d > 0.0 ? 1.0 / d : 0.0;  // an empty bin adds nothing
        const double v = Y - (Z0 * bc.g[0] + Z1 * bc.g[1] + Z2 * bc.g[2]);
        const double vi = v * inv;
        s1 += v * vi;
        r0 += Z0 * vi;
        r1 += Z1 * vi;
        r2 += Z2 * vi;
        const double z0i = Z0 * inv, z1i = Z1 * inv, z2i = Z2 * inv;
        p00 += Z0 * z0i;
        p01 += Z0 * z1i;
        p02 += Z0 * z2i;
        p11 += Z1 * z1i;
        p12 += Z1 * z2i;
        p22 += Z2 * z2i;
      }
      // r^T Q^-1 r with Q = H - P (symmetric positive definite, Q >= I)
      const double q00 = bc.H[0] - p00, q01 = bc.H[1] - p01, q02 = bc.H[2] - p02;
      const double q11 = bc.H[3] - p11, q12 = bc.H[4] - p12, q22 = bc.H[5] - p22;
      const double l1 = q01 / q00, l2 = q02 / q00;
      const double a11 = q11 - l1 * q01, a12 = q12 - l1 * q02, a22 = q22 - l2 * q02;
      const double m2 = a12 / a11;
      const double c22 = a22 - m2 * a12;
      const double y1 = r1 - l1 * r0;
      const double y2 = r2 - l2 * r0 - m2 * y1;
      const double s2 = r0 * r0 / q00 + y1 * y1 / a11 + y2 * y2 / c22;
      if (k < k1) a.S[(int64_t)c * a.n_freq + k] = (float)((s1 + s2) * bc.scale);
    }
  }
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(a.queue + 1, 1u) == gridDim.x - 1) {
      atomicExch(a.queue, 0u);
      atomicExch(a.queue + 1, 0u);
    }
  }
}

}  // namespace

size_t bm_lds_bytes(int n_bins) { return (size_t)2 * n_bins * kWave * sizeof(uint64_t); }

hipError_t bm_groups_per_cu(int phase, int n_bins, int* out) {
  const void* fn = phase == PH_LISTING ? (const void*)bm_kernel<PH_LISTING> : (const void*)bm_kernel<PH_FP64>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bm_lds_bytes(n_bins));
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, kWave, bm_lds_bytes(n_bins));
}

hipError_t launch_bm(const BmArgs& a, int phase, int grid, hipStream_t s) {
  const void* fn = phase == PH_LISTING ? (const void*)bm_kernel<PH_LISTING> : (const void*)bm_kernel<PH_FP64>;
  const size_t lds = bm_lds_bytes(a.n_bins);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  BmArgs args = a;
  const RecB* rec = a.rec;
  const int64_t* offsets = a.offsets;
  const BaseConst* bcs = a.bc;
  const double* freqs = a.freqs;
  const Item* items = a.items;
  void* params[] = {&args, &rec, &offsets, &bcs, &freqs, &items};
  return hipLaunchKernel(fn, dim3(grid), dim3(kWave), params, lds, s);
}

}  // namespace fpw
