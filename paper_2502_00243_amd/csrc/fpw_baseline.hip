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

// Observations reach the lanes as in the general kernel's vector source: the
// lanes of each row of 16 load 16 consecutive records (one coalesced load),
// and each record is then broadcast to its row with 64-bit DPP row_newbcast
// moves.  Only vector-memory counters are waited on, so the LDS atomics of
// earlier points stay in flight.
constexpr int kGroup = 16;

// Extra sums per bin: none with one baseline term (Z_0 = beta W needs no sum
// of its own), one 32-bit word (w T_1) with two, one 64-bit word (w T_1,
// w T_2) with three.
enum { NZ_NONE = 0, NZ_PAIR = 1, NZ_ONE = 2 };

template <int Q>
__device__ __forceinline__ uint32_t row_bcast32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x150 + Q, 0xf, 0xf, true);
}
__device__ __forceinline__ void lds_add32(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t lds_take32(uint32_t* p) {
  return __hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One point q of the current group: fold, bin, and the sums.
template <int PH, int NZ, int Q>
__device__ __forceinline__ void bm_point(const RecB& cur, const Folder<PH>& fo, uint32_t M, uint64_t* hw, uint64_t* hz,
                                         uint32_t* hz32) {
  const uint32_t b0 = (uint32_t)fo.bin(row_bcast<Q>(cur.tau_bits));
  const uint32_t b = min(b0, b0 - M);  // the fused fold reports bin 0 as M
  lds_add(hw + b * kWave, row_bcast<Q>(cur.pk));
  if (NZ == NZ_PAIR) lds_add(hz + b * kWave, row_bcast<Q>(cur.pz));
  if (NZ == NZ_ONE) lds_add32(hz32 + b * kWave, row_bcast32<Q>(lo32(cur.pz)));
}

// Slots per lane: M (weight, residual) words, then M extra words ([m][lane]).
template <int PH, int NZ>
__global__ __launch_bounds__(kWave) void bm_kernel(BmArgs a, const RecB* __restrict__ rec,
                                                   const int64_t* __restrict__ offsets,
                                                   const BaseConst* __restrict__ bcs,
                                                   const double* __restrict__ freqs,
                                                   const Item* __restrict__ items) {
  extern __shared__ __align__(16) uint64_t lds[];
  const int lane = threadIdx.x;
  const int M = a.n_bins;
  uint64_t* hw = lds + lane;                      // [m][lane]: weight and residual
  uint64_t* hz = lds + (size_t)M * kWave + lane;  // [m][lane]: w T_1 and w T_2 (64-bit pair)
  uint32_t* hz32 = reinterpret_cast<uint32_t*>(lds + (size_t)M * kWave) + lane;  // [m][lane]: w T_1 alone
  for (int m = 0; m < M; ++m) {
    hw[m * kWave] = 0;
    if (NZ == NZ_PAIR) hz[m * kWave] = 0;
    if (NZ == NZ_ONE) hz32[m * kWave] = 0;
  }
  const int sub = lane & (kGroup - 1);
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
      RecB cur = rc[sub < n ? sub : n - 1];
      for (int g = 0; g < n; g += kGroup) {
        const int nxt = g + kGroup + sub;
        const RecB next = rc[nxt < n ? nxt : n - 1];  // prefetch (clamped, in bounds)
        const int cnt = n - g;                         // wave-uniform
        if (cnt >= kGroup) {
          static_for<0, kGroup>([&](auto qc) { bm_point<PH, NZ, decltype(qc)::value>(cur, fo, (uint32_t)M, hw, hz, hz32); });
        } else {
          static_for<0, kGroup>([&](auto qc) {
            if (decltype(qc)::value < cnt) bm_point<PH, NZ, decltype(qc)::value>(cur, fo, (uint32_t)M, hw, hz, hz32);
          });
        }
        cur = next;
      }
      // FP64 epilogue: v^T L^-1 v and the 3x3 correction
      double s1 = 0.0, r0 = 0.0, r1 = 0.0, r2 = 0.0;
      double p00 = 0.0, p01 = 0.0, p02 = 0.0, p11 = 0.0, p12 = 0.0, p22 = 0.0;
      for (int m = 0; m < M; ++m) {
        const uint64_t vw = lds_take(hw + m * kWave);
        const uint64_t vz = NZ == NZ_PAIR ? lds_take(hz + m * kWave)
                            : (NZ == NZ_ONE ? (uint64_t)(int64_t)(int32_t)lds_take32(hz32 + m * kWave) : (uint64_t)0);
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

size_t bm_lds_bytes(int n_bins, int n_terms) {
  const size_t per_slot = n_terms >= 3 ? 16 : (n_terms == 2 ? 12 : 8);
  return per_slot * n_bins * kWave;
}

namespace {
const void* bm_fn(int phase, int n_terms) {
  const bool lst = phase == PH_LISTING;
  if (n_terms >= 3) return lst ? (const void*)bm_kernel<PH_LISTING, NZ_PAIR> : (const void*)bm_kernel<PH_FP64, NZ_PAIR>;
  if (n_terms == 2) return lst ? (const void*)bm_kernel<PH_LISTING, NZ_ONE> : (const void*)bm_kernel<PH_FP64, NZ_ONE>;
  return lst ? (const void*)bm_kernel<PH_LISTING, NZ_NONE> : (const void*)bm_kernel<PH_FP64, NZ_NONE>;
}
}  // namespace

hipError_t bm_groups_per_cu(int phase, int n_bins, int n_terms, int* out) {
  const void* fn = bm_fn(phase, n_terms);
  const size_t lds = bm_lds_bytes(n_bins, n_terms);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, kWave, lds);
}

hipError_t launch_bm(const BmArgs& a, int phase, int grid, hipStream_t s) {
  const void* fn = bm_fn(phase, a.n_terms);
  const size_t lds = bm_lds_bytes(a.n_bins, a.n_terms);
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
