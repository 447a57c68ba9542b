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
// K <= 3 the kernel needs at most one more sum per bin: none for K = 1, the
// 32-bit word Z_1 for K = 2 (a ds_add_u32), the packed pair (Z_1, Z_2) for
// K = 3 (a second ds_add_u64).  The epilogue runs in FP64: the bin sums are
// exact integers and the constants were formed from the same rounded values
// (the constant direction of Q is then exactly the prior's 1, not a
// difference of two large sums).  Observations come through the general
// kernel's point sources, and for large histograms several waves share one,
// as in the general kernel.
#include "fpw_common.h"

namespace fpw {
namespace {

using namespace dev;

// Where a wave's observations come from, as in the general kernel.
//  BSRC_SCALAR: wave-uniform scalar loads of 8 records at a time into SGPRs;
//    tau is a scalar operand of the fold, the packed words take one move each.
//  BSRC_DPP: the lanes of each row of 16 load 16 consecutive records (one
//    coalesced load) and each record is broadcast to its row with 64-bit DPP
//    row_newbcast moves; only vector-memory counters are waited on.
enum BmSource { BSRC_SCALAR = 0, BSRC_DPP = 1 };
constexpr int kGroup = 16;

// Extra sums per bin: none with one baseline term (Z_0 = beta W needs no sum
// of its own), one 32-bit word (w T_1) with two, one 64-bit word (w T_1,
// w T_2) with three.
enum BmExtra { NZ_NONE = 0, NZ_PAIR = 1, NZ_ONE = 2 };

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

// Histogram slot stride in 64-bit words: with the 64-bit pair the two sums
// of a bin are interleaved, [m][2][lane], so the second atomic reuses the
// first one's address with a constant offset; otherwise [m][lane].
template <int NZ>
constexpr int kSlotWords = (NZ == NZ_PAIR ? 2 : 1) * kWave;

// The sums of one observation at the lane's bin b (0 <= b <= M; slot M is
// the fused fold's name for bin 0 and is added to bin 0 when read).
template <int NZ>
__device__ __forceinline__ void bm_add(int b, uint64_t pk, uint64_t pz, uint64_t* hw, uint64_t* hz, uint32_t* hz32) {
  lds_add(hw + b * kSlotWords<NZ>, pk);
  if (NZ == NZ_PAIR) lds_add(hz + b * kSlotWords<NZ>, pz);
  if (NZ == NZ_ONE) lds_add32(hz32 + b * kWave, lo32(pz));
}

// Baseline sums per observation as stored for NZ: 64-bit pair, 32-bit word, or none.
template <int NZ>
using ZWord = typename std::conditional<NZ == NZ_PAIR, uint64_t, uint32_t>::type;

// Folds and adds observations [0, n) of rc / zc (n >= 1).
template <int PH, int NZ, int SRC>
__device__ __forceinline__ void bm_accumulate(const Rec* __restrict__ rc, const ZWord<NZ>* __restrict__ zc, int n,
                                              const Folder<PH>& fo, uint64_t* hw, uint64_t* hz, uint32_t* hz32,
                                              int lane) {
  if (SRC == BSRC_SCALAR) {
    int i = 0;
    for (; i + kBatch <= n; i += kBatch) {
      Rec r[kBatch];
      ZWord<NZ> z[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) r[q] = rc[i + q];
      if (NZ != NZ_NONE) {
#pragma unroll
        for (int q = 0; q < kBatch; ++q) z[q] = zc[i + q];
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q)
        bm_add<NZ>(fo.bin(r[q].tau_bits), uniform_to_vgpr(r[q].pk),
                   NZ == NZ_PAIR ? uniform_to_vgpr((uint64_t)z[q]) : (NZ == NZ_ONE ? (uint64_t)z[q] : 0), hw, hz, hz32);
    }
    for (; i < n; ++i) {
      const Rec r = rc[i];
      const uint64_t z = NZ == NZ_NONE ? 0 : (uint64_t)zc[i];
      bm_add<NZ>(fo.bin(r.tau_bits), uniform_to_vgpr(r.pk), NZ == NZ_PAIR ? uniform_to_vgpr(z) : z, hw, hz, hz32);
    }
  } else {
    const int sub = lane & (kGroup - 1);
    Rec cur = rc[sub < n ? sub : n - 1];
    ZWord<NZ> curz = NZ == NZ_NONE ? 0 : zc[sub < n ? sub : n - 1];
    for (int g = 0; g < n; g += kGroup) {
      const int nxt = g + kGroup + sub;
      const int ld = nxt < n ? nxt : n - 1;  // prefetch (clamped, in bounds)
      const Rec next = rc[ld];
      const ZWord<NZ> nextz = NZ == NZ_NONE ? 0 : zc[ld];
      const int cnt = n - g;  // wave-uniform
      auto point = [&](auto qc) {
        constexpr int q = decltype(qc)::value;
        bm_add<NZ>(fo.bin(row_bcast<q>(cur.tau_bits)), row_bcast<q>(cur.pk),
                   NZ == NZ_PAIR ? row_bcast<q>((uint64_t)curz) : (uint64_t)row_bcast32<q>((uint32_t)curz), hw, hz, hz32);
      };
      if (cnt >= kGroup) {
        static_for<0, kGroup>(point);  // a full group, straight-line
      } else {
        static_for<0, kGroup>([&](auto qc) {
          if (decltype(qc)::value < cnt) point(qc);
        });
      }
      cur = next;
      curz = nextz;
    }
  }
}

// 1/d for d > 0 to within an ulp or so: the hardware estimate refined by two
// Newton steps (each roughly doubles the correct bits), half the instructions
// of a correctly rounded division.  The epilogue needs full FP64 accuracy
// here: Q = H - Z^T L^-1 Z subtracts sums of size beta^2 sum W.
__device__ __forceinline__ double recip64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Per-lane sums of the FP64 epilogue over a range of bins: v^T L^-1 v, r = Z^T L^-1 v
// and P = Z^T L^-1 Z (upper triangle), indexed as below.
enum { SV = 0, SR0, SR1, SR2, SP00, SP01, SP02, SP11, SP12, SP22, kBmSums };
struct BmSums {
  double v[kBmSums];
};

// The sums that K terms can make non-zero (Z_1 = 0 for K = 1, Z_2 = 0 for
// K <= 2): only these pass between the waves of a shared histogram.
template <int NZ>
constexpr int kLiveSums = NZ == NZ_NONE ? 3 : (NZ == NZ_ONE ? 6 : kBmSums);
template <int NZ>
constexpr int live_sum(int j) {
  constexpr int none[3] = {SV, SR0, SP00};
  constexpr int one[6] = {SV, SR0, SR1, SP00, SP01, SP11};
  return NZ == NZ_NONE ? none[j] : (NZ == NZ_ONE ? one[j] : j);
}

// Reads and clears bins [mb, me) of one lane's histograms and returns their
// sums; the range that starts at bin 0 also takes the wrap slot M.
template <int PH, int NZ>
__device__ __forceinline__ BmSums bm_bins(uint64_t* hw, uint64_t* hz, uint32_t* hz32, int M, int mb, int me,
                                          const BaseConst& bc) {
  BmSums a{};
  uint64_t wrap_w = 0, wrap_z = 0;
  constexpr int SW = kSlotWords<NZ>;
  if (PH == PH_FP64 && mb == 0 && me > 0) {
    wrap_w = lds_take(hw + M * SW);
    if (NZ == NZ_PAIR) wrap_z = lds_take(hz + M * SW);
    if (NZ == NZ_ONE) wrap_z = lds_take32(hz32 + M * kWave);
  }
  for (int m = mb; m < me; ++m) {
    uint64_t vw = lds_take(hw + m * SW);
    uint64_t vz = NZ == NZ_PAIR ? lds_take(hz + m * SW) : (NZ == NZ_ONE ? (uint64_t)lds_take32(hz32 + m * kWave) : 0);
    if (m == 0) {  // integer sums: adding the wrap slot is exact (modulo the word, like every addition)
      vw += wrap_w;
      vz += wrap_z;
    }
    if (NZ == NZ_ONE) vz = (uint64_t)(int64_t)(int32_t)lo32(vz);
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
    const double inv = d > 0.0 ? recip64(d) : 0.0;  // an empty bin adds nothing
    const double v = Y - (Z0 * bc.g[0] + Z1 * bc.g[1] + Z2 * bc.g[2]);
    const double vi = v * inv;
    a.v[SV] += v * vi;
    a.v[SR0] += Z0 * vi;
    a.v[SR1] += Z1 * vi;
    a.v[SR2] += Z2 * vi;
    const double z0i = Z0 * inv, z1i = Z1 * inv, z2i = Z2 * inv;
    a.v[SP00] += Z0 * z0i;
    a.v[SP01] += Z0 * z1i;
    a.v[SP02] += Z0 * z2i;
    a.v[SP11] += Z1 * z1i;
    a.v[SP12] += Z1 * z2i;
    a.v[SP22] += Z2 * z2i;
  }
  return a;
}

// S = v^T L^-1 v + r^T Q^-1 r with Q = H - P (symmetric positive definite,
// Q >= I), by an LDL^T factorisation of the 3x3 Q.
__device__ __forceinline__ double bm_statistic(const BmSums& a, const BaseConst& bc) {
  const double q00 = bc.H[0] - a.v[SP00], q01 = bc.H[1] - a.v[SP01], q02 = bc.H[2] - a.v[SP02];
  const double q11 = bc.H[3] - a.v[SP11], q12 = bc.H[4] - a.v[SP12], q22 = bc.H[5] - a.v[SP22];
  const double r0 = a.v[SR0], r1 = a.v[SR1], r2 = a.v[SR2];
  const double l1 = q01 / q00, l2 = q02 / q00;
  const double a11 = q11 - l1 * q01, a12 = q12 - l1 * q02, a22 = q22 - l2 * q02;
  const double m2 = a12 / a11;
  const double c22 = a22 - m2 * a12;
  const double y1 = r1 - l1 * r0;
  const double y2 = r2 - l2 * r0 - m2 * y1;
  const double s2 = r0 * r0 / q00 + y1 * y1 / a11 + y2 * y2 / c22;
  return a.v[SV] + s2;
}

// Slots per histogram lane: M+1 (weight, residual) words and M+1 extra
// words (slot M is bin 0 seen through the fused fold): interleaved per bin
// for the 64-bit pair, else the extra words after the (weight, residual)
// words.  SH == 1:
// one wave per workgroup with its own histograms.  SH > 1: the SH waves of a
// workgroup share them; each folds a contiguous slice of the curve's
// observations, then each takes the epilogue sums of a contiguous range of
// bins, and wave 0 adds them (in wave order) and forms S.  After the
// histograms: the partial sums [SH-1][live sums][lane] (FP64) and the group's item
// index.
template <int PH, int NZ, int SH, int SRC>
// (The sums' pointer is untyped in the signature: a type that depends on an
// unnamed enum would mangle differently in the host and device compilations.)
__global__ __launch_bounds__(kWave * SH) void bm_kernel(BmArgs a, const Rec* __restrict__ rec,
                                                        const void* __restrict__ zs,
                                                        const int64_t* __restrict__ offsets,
                                                        const BaseConst* __restrict__ bcs,
                                                        const double* __restrict__ freqs,
                                                        const Item* __restrict__ items) {
  extern __shared__ __align__(16) uint64_t lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform: keeps slice loads scalar
  const int M = a.n_bins;
  const int slots = M + 1;
  constexpr int SW = kSlotWords<NZ>;
  uint64_t* hw = lds + lane;          // slot m at hw + m SW: weight and residual
  uint64_t* hz = lds + kWave + lane;  // NZ_PAIR, slot m at hz + m SW: w T_1 and w T_2
  uint32_t* hz32 = reinterpret_cast<uint32_t*>(lds + (size_t)slots * kWave) + lane;  // NZ_ONE, [m][lane]: w T_1
  // histogram size in 64-bit words: 8, 12 or 16 bytes per (slot, lane)
  const int hist_words = (NZ == NZ_NONE ? 2 : (NZ == NZ_ONE ? 3 : 4)) * slots * kWave / 2;
  double* part = reinterpret_cast<double*>(lds + hist_words);
  int* group_item = reinterpret_cast<int*>(part + (SH - 1) * kLiveSums<NZ> * kWave);
  for (int m = wave; m < slots; m += SH) {
    hw[m * SW] = 0;
    if (NZ == NZ_PAIR) hz[m * SW] = 0;
    if (NZ == NZ_ONE) hz32[m * kWave] = 0;
  }
  // the waves of a shared histogram clear their own slots but fold into
  // all of them: clearing completes before any wave's first atomic
  if (SH > 1) __syncthreads();
  // With at most one item per consumer (a wave, or a workgroup sharing a
  // histogram), consumer c takes item c and no atomics are needed.
  // Otherwise every item is popped from the queue, whose counter the pass's
  // prepare kernel has zeroed, the first one too: that staggers the
  // consumers' starts, which keeps their later pops apart (taking the first
  // item by index measured 4.8 % slower on 1000 curves x 1e5 frequencies).
  const int per_group = SH > 1 ? 1 : (int)(blockDim.x / kWave);
  const bool by_index = a.n_items <= (int)gridDim.x * per_group;
  for (int round = 0;; ++round) {
    int it = 0;
    if (by_index) {
      if (round > 0) break;
      it = (int)blockIdx.x * per_group + (SH > 1 ? 0 : wave);
    } else if (SH > 1) {
      // one pop per workgroup; the previous item's barriers order this write
      // after every wave's read of the previous index
      if (threadIdx.x == 0) *group_item = (int)atomicAdd(a.queue, 1u);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(*group_item);
    } else {
      if (lane == 0) it = (int)atomicAdd(a.queue, 1u);
      it = __builtin_amdgcn_readfirstlane(it);
    }
    if (it >= a.n_items) break;
    const Item item = items[it];
    const int c = item.curve, k0 = item.k0, k1 = item.k1;
    const int64_t p0 = offsets[c];
    const int n_all = (int)(offsets[c + 1] - p0);
    const int lo = SH > 1 ? (int)((int64_t)wave * n_all / SH) : 0;
    const int n = SH > 1 ? (int)((int64_t)(wave + 1) * n_all / SH) - lo : n_all;
    const Rec* __restrict__ rc = rec + p0 + lo;
    const ZWord<NZ>* __restrict__ zc = static_cast<const ZWord<NZ>*>(zs) + p0 + lo;
    const BaseConst bc = bcs[c];
    for (int kt = k0; kt < k1; kt += kWave) {
      const int k = kt + lane;
      if (n > 0) {
        Folder<PH> fo;
        fo.init(freqs[k < k1 ? k : k1 - 1], M, a.fold_nh);
        bm_accumulate<PH, NZ, SRC>(rc, zc, n, fo, hw, hz, hz32, lane);
      }
      if constexpr (SH == 1) {
        const BmSums sums = bm_bins<PH, NZ>(hw, hz, hz32, M, 0, M, bc);
        if (k < k1) a.S[(int64_t)c * a.n_freq + k] = (float)(bm_statistic(sums, bc) * bc.scale);
      } else {
        __syncthreads();  // every slice is in the histograms
        BmSums sums = bm_bins<PH, NZ>(hw, hz, hz32, M, wave * M / SH, (wave + 1) * M / SH, bc);
        constexpr int NL = kLiveSums<NZ>;
        if (wave > 0) {
          double* pp = part + (size_t)(wave - 1) * NL * kWave + lane;
#pragma unroll
          for (int j = 0; j < NL; ++j) pp[j * kWave] = sums.v[live_sum<NZ>(j)];
        }
        __syncthreads();  // partial sums visible, histograms clear for the next sub-tile
        if (wave == 0) {
#pragma unroll
          for (int w = 1; w < SH; ++w) {
            const double* pp = part + (size_t)(w - 1) * NL * kWave + lane;
#pragma unroll
            for (int j = 0; j < NL; ++j) sums.v[live_sum<NZ>(j)] += pp[j * kWave];
          }
          if (k < k1) a.S[(int64_t)c * a.n_freq + k] = (float)(bm_statistic(sums, bc) * bc.scale);
        }
      }
    }
  }
}

}  // namespace

size_t bm_lds_bytes(int n_bins, int n_terms, int share) {
  const size_t per_slot = n_terms >= 3 ? 16 : (n_terms == 2 ? 12 : 8);
  const size_t hist = per_slot * (n_bins + 1) * kWave;
  if (share <= 1) return hist;
  const int live = n_terms >= 3 ? kLiveSums<NZ_PAIR> : (n_terms == 2 ? kLiveSums<NZ_ONE> : kLiveSums<NZ_NONE>);
  return hist + (size_t)(share - 1) * live * kWave * sizeof(double) + 16;
}

namespace {
template <int PH, int SH, int SRC>
const void* bm_fn_sh(int n_terms) {
  if (n_terms >= 3) return (const void*)bm_kernel<PH, NZ_PAIR, SH, SRC>;
  if (n_terms == 2) return (const void*)bm_kernel<PH, NZ_ONE, SH, SRC>;
  return (const void*)bm_kernel<PH, NZ_NONE, SH, SRC>;
}
template <int PH, int SRC>
const void* bm_fn_ph(int n_terms, int share) {
  return share == 4 ? bm_fn_sh<PH, 4, SRC>(n_terms) : (share == 2 ? bm_fn_sh<PH, 2, SRC>(n_terms) : bm_fn_sh<PH, 1, SRC>(n_terms));
}
// source: 0 scalar loads, 1 vector loads + DPP broadcast
const void* bm_fn(int phase, int n_terms, int share, int source) {
  if (source == BSRC_DPP)
    return phase == PH_LISTING ? bm_fn_ph<PH_LISTING, BSRC_DPP>(n_terms, share) : bm_fn_ph<PH_FP64, BSRC_DPP>(n_terms, share);
  return phase == PH_LISTING ? bm_fn_ph<PH_LISTING, BSRC_SCALAR>(n_terms, share)
                             : bm_fn_ph<PH_FP64, BSRC_SCALAR>(n_terms, share);
}
}  // namespace

hipError_t bm_groups_per_cu(int phase, int n_bins, int n_terms, int share, int source, int* out) {
  const void* fn = bm_fn(phase, n_terms, share, source);
  const size_t lds = bm_lds_bytes(n_bins, n_terms, share);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, kWave * share, lds);
}

hipError_t launch_bm(const BmArgs& a, int phase, int grid, hipStream_t s) {
  const int share = a.share > 1 ? a.share : 1;
  const void* fn = bm_fn(phase, a.n_terms, share, a.source);
  const size_t lds = bm_lds_bytes(a.n_bins, a.n_terms, share);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  BmArgs args = a;
  const Rec* rec = a.rec;
  const void* zs = a.z;
  const int64_t* offsets = a.offsets;
  const BaseConst* bcs = a.bc;
  const double* freqs = a.freqs;
  const Item* items = a.items;
  void* params[] = {&args, &rec, &zs, &offsets, &bcs, &freqs, &items};
  return hipLaunchKernel(fn, dim3(grid), dim3(kWave * share), params, lds, s);
}

}  // namespace fpw
