// Shared-timestamp batches on the matrix cores.
//
// When many curves are observed at the same times (Sec. 4: the batch function
// for light curves that share timestamps; App. C: all sources of one image
// field), the bin of an observation depends only on (frequency, time), so one
// fold serves every curve.  For a fixed frequency f the per-bin sums of all
// curves are then one matrix product,
//
//     [W | Y]_{(curve), m} = sum over points p of V[(curve, quantity), p] * [bin(f, p) == m],
//
// a dense contraction over the points.  Here it runs exactly on the int8
// matrix cores: V holds the four signed base-256 digits of each point's
// fixed-point weight and weighted residual (rows of the A operand), the
// one-hot indicator of the bins is the B operand (columns = (frequency, bin)
// pairs), and v_mfma_i32_32x32x32_i8 accumulates in int32 without rounding.
// The digit sums are recombined (two's-complement wrap is exact because
// every bin sum lies within 30 bits), and the statistic of Eq. 1 is formed
// as in the general kernel.
//
// Workgroup: 8 waves sharing one block of curves (CG tiles of 4 curves).  The
// curves' digit tiles are staged in LDS (in chunks of up to 512 points); each
// wave owns fw frequencies per round (fw * M <= 32 NB columns, NB = 2 or 3
// B tiles), folds the chunk's points at those frequencies into bytes in its
// private LDS, builds the one-hot operand from them and issues CG * NB
// products per 32 points (with two B tiles the K loop is software-pipelined
// so the one-hot work overlaps the products' issue).
#include <algorithm>

#include "fpw_common.h"

namespace fpw {
namespace {

using namespace dev;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));


// Bytes of `bins` equal to m become 64, the others 0.  Every bin and every
// column's m is below 64 (padding columns use m = 63 > any bin, or there is
// no padding when M = 64), so x = bins ^ m has bytes in [0, 63] and
// (x ^ 0x3f) + 1 = 0x40 - x per byte with no borrow between bytes; its bit 6
// is set exactly where x == 0.  mmx = (m * 0x01010101) ^ 0x3f3f3f3f.  Two
// instructions per four bytes; the products then carry a factor 64, which
// the epilogue removes exactly.
__device__ __forceinline__ int one_hot4(uint32_t bins, uint32_t mmx) {
  return (int)(((bins ^ mmx) + 0x01010101u) & 0x40404040u);
}

// Digit sums of one quantity (registers e .. e+3 of a product, each 64 times
// the true sum) recombined to the exact 32-bit value: digit 0 is divided by
// 64, digit i > 0 is scaled by 2^(8 i - 6); the wrap-around of the sum is
// exact because the true value fits in 30 bits.
__device__ __forceinline__ uint32_t recombine64(const v16i& c, int e) {
  return ((uint32_t)(c[e] >> 6)) + ((uint32_t)c[e + 1] << 2) + ((uint32_t)c[e + 2] << 10) + ((uint32_t)c[e + 3] << 18);
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NB: B tiles (32 columns each) per wave.
template <int PH, int CG, int NB>
__global__ __launch_bounds__(kSharedWaves * kWave) __attribute__((amdgpu_waves_per_eu(1, 2))) void shared_kernel(SharedArgs a) {
  constexpr int kNB = NB;
  constexpr int kTermStride = 32 * NB + 1;  // floats per curve row of the term table (odd: no bank conflicts)
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int n = lane & 31, h = lane >> 5;
  const int M = a.n_bins;
  const int KCB = a.chunk_kblocks, KC = KCB * 32;
  unsigned char* vals = lds;
  unsigned char* priv = lds + (size_t)CG * KCB * kSharedTileBytes + (size_t)wave * a.priv_bytes;
  uint32_t* binw = reinterpret_cast<uint32_t*>(priv);  // [fw][KC] bytes, 4 per word
  float* terms = reinterpret_cast<float*>(priv);       // [4 CG][kTermStride], after the products
  const int g0 = blockIdx.y * CG;                      // first curve group of the block
  const int n_chunks = (a.n_kblocks + KCB - 1) / KCB;

  // column (frequency slot, bin) of each B tile; padding columns match nothing
  int colf[kNB];
  uint32_t colm[kNB];
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const int col = 32 * b + n;
    int m = 63;
    colf[b] = 0;
    if (col < a.fw * M) {
      colf[b] = col / M;
      m = col - colf[b] * M;
    }
    colm[b] = ((uint32_t)m * 0x01010101u) ^ 0x3f3f3f3fu;
  }
  // prior term of the two curves per A tile this lane finishes: 4 ai + 2 u + h
  float ia2q[CG][2];
#pragma unroll
  for (int ai = 0; ai < CG; ++ai)
#pragma unroll
    for (int u = 0; u < 2; ++u) ia2q[ai][u] = a.cc[(int64_t)(g0 + ai) * kSharedGroupCurves + 2 * u + h].ia2q;

  for (int r = 0; r < a.rounds; ++r) {
    const int f0 = ((blockIdx.x * a.rounds + r) * kSharedWaves + wave) * a.fw;
    // accumulators: the pipelined two-tile loop starts each round with
    // products whose addend is zero (an inline constant); the three-tile
    // path clears them here (peeling its first K-block measured slower)
    v16i acc[CG][kNB];
    if constexpr (kNB != 2) {
#pragma unroll
      for (int ai = 0; ai < CG; ++ai)
#pragma unroll
        for (int b = 0; b < kNB; ++b) acc[ai][b] = (v16i){};
    }

    for (int ch = 0; ch < n_chunks; ++ch) {
      const int kb0 = ch * KCB;
      const int kbn = min(KCB, a.n_kblocks - kb0);
      if (n_chunks > 1 || r == 0) {
        __syncthreads();  // every wave is done with the previous chunk
        const int pieces = CG * kbn * (kSharedTileBytes / 16);
        for (int i = tid; i < pieces; i += kSharedWaves * kWave) {
          const int t = i >> 6, piece = i & 63;
          const int ai = t / kbn, kbl = t - ai * kbn;
          const v4i v = *reinterpret_cast<const v4i*>(
              a.vals + ((int64_t)(g0 + ai) * a.n_kblocks + kb0 + kbl) * kSharedTileBytes + piece * 16);
          *reinterpret_cast<v4i*>(vals + (size_t)(kbl * CG + ai) * kSharedTileBytes + piece * 16) = v;
        }
        __syncthreads();
      }
      // This wave's bins of the chunk's points, one byte each.  A lane owns
      // the words d = lane and lane + 64 (four points each; KC <= 512) and
      // folds their times at every frequency of the wave.
      const int nd = kbn * 8;
      double tv[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int d = min(lane + kWave * j, nd - 1);
        const double* tp = a.tau + (int64_t)kb0 * 32 + d * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) tv[j][q] = tp[q];
      }
      for (int fl = 0; fl < a.fw; ++fl) {
        Folder<PH> fo;
        fo.init(a.freqs[min(f0 + fl, a.n_freq - 1)], M, a.fold_nh);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int d = lane + kWave * j;
          uint32_t word = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t bin = (uint32_t)fo.bin((uint64_t)__double_as_longlong(tv[j][q]));
            // the fused FP64 fold reports bin 0 as M: min(bin, bin - M) folds it back
            word |= min(bin, bin - (uint32_t)M) << (8 * q);
          }
          if (d < nd) binw[fl * (KC / 4) + d] = word;
        }
      }
      wave_lds_fence();
      // Products.  The chunk's tiles sit in LDS as [K-block][curve group], so
      // every A read is an immediate offset from one base pointer.
      const unsigned char* bbase[kNB];
#pragma unroll
      for (int b = 0; b < kNB; ++b) bbase[b] = priv + colf[b] * KC + h * 16;
      const unsigned char* abase = vals + lane * 16;
      auto read_a = [&](int kb, v4i (&av)[CG]) {
#pragma unroll
        for (int ai = 0; ai < CG; ++ai) av[ai] = *reinterpret_cast<const v4i*>(abase + (kb * CG + ai) * kSharedTileBytes);
      };
      auto read_bins = [&](int kb, v4i (&nb)[kNB]) {
#pragma unroll
        for (int b = 0; b < kNB; ++b) nb[b] = *reinterpret_cast<const v4i*>(bbase[b] + kb * 32);
      };
      if constexpr (kNB == 2) {
        // Software-pipelined: the products of K-block kb run while the bins
        // of kb + 1 (read one step earlier) become one-hot operands and the
        // reads for kb + 1 (A tiles) and kb + 2 (bins) are in flight; the
        // issue order alternates one product and two VALU instructions, so
        // the VALU work sits in the matrix cores' shadow.  Reads past the
        // last K-block are clamped to it (harmless rereads).
        v4i bv[kNB], nb0[kNB], nb1[kNB], av0[CG], av1[CG];
        read_bins(0, nb0);
#pragma unroll
        for (int b = 0; b < kNB; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) bv[b][i] = one_hot4((uint32_t)nb0[b][i], colm[b]);
        read_bins(min(1, kbn - 1), nb0);
        read_a(0, av0);
        // one K-block: products with (av, bv); bv <- one-hot of nb (the next
        // K-block's bins); reads of the next A tiles into an and of the bins
        // two K-blocks ahead into nn
        auto step = [&](int kb, v4i (&av)[CG], v4i (&an)[CG], v4i (&nb)[kNB], v4i (&nn)[kNB], auto first) {
          read_a(min(kb + 1, kbn - 1), an);
          read_bins(min(kb + 2, kbn - 1), nn);
#pragma unroll
          for (int b = 0; b < kNB; ++b) {
#pragma unroll
            for (int ai = 0; ai < CG; ++ai)
              acc[ai][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av[ai], bv[b], decltype(first)::value ? (v16i){} : acc[ai][b],
                                                               0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[b][i] = one_hot4((uint32_t)nb[b][i], colm[b]);
          }
#pragma unroll
          for (int q = 0; q < CG * kNB; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix product
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // two VALU instructions
          }
        };
        // two K-blocks per iteration, so the operand sets swap roles without
        // copies; the round's first two are peeled (the very first product
        // of each accumulator adds to zero)
        const std::false_type later{};
        int kb = 0;
        if (ch == 0) {
          step(0, av0, av1, nb0, nb1, std::true_type{});
          if (kbn > 1) step(1, av1, av0, nb1, nb0, later);
          kb = 2;
        }
        for (; kb + 1 < kbn; kb += 2) {
          step(kb, av0, av1, nb0, nb1, later);
          step(kb + 1, av1, av0, nb1, nb0, later);
        }
        if (kb < kbn) step(kb, av0, av1, nb0, nb1, later);
      } else {
        // one K-block: its bins become one-hot operands, then its products
        auto block = [&](int kb) {
          v4i av[CG], bv[kNB];
          read_a(kb, av);
          read_bins(kb, bv);
#pragma unroll
          for (int b = 0; b < kNB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[b][i] = one_hot4((uint32_t)bv[b][i], colm[b]);
#pragma unroll
          for (int ai = 0; ai < CG; ++ai)
#pragma unroll
            for (int b = 0; b < kNB; ++b)
              acc[ai][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av[ai], bv[b], acc[ai][b], 0, 0, 0);
        };
        // four K-blocks per step
        for (int kb4 = 0; kb4 < kbn; kb4 += 4) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (kb4 + j < kbn) block(kb4 + j);
        }
      }
    }

    // Epilogue.  Lane (n, h) of product (ai, b) holds column 32 b + n and, in
    // registers 8 u + 4 q + i, digit i of quantity q of curve 4 ai + 2 u + h.
    wave_lds_fence();
#pragma unroll
    for (int ai = 0; ai < CG; ++ai) {
#pragma unroll
      for (int b = 0; b < kNB; ++b) {
        const v16i& c = acc[ai][b];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t wq = recombine64(c, 8 * u);
          const int yq = (int)recombine64(c, 8 * u + 4);
          const float d = (float)wq + ia2q[ai][u];  // ia2q >= kMinPrior: an empty bin adds 0
          const float yf = (float)yq;
          terms[(4 * ai + 2 * u + h) * kTermStride + 32 * b + n] = yf * (yf * __builtin_amdgcn_rcpf(d));
        }
      }
    }
    wave_lds_fence();
    for (int pi = lane; pi < a.fw * 4 * CG; pi += kWave) {
      const int fl = pi / (4 * CG), cl = pi - fl * (4 * CG);
      const float* tr = terms + cl * kTermStride + fl * M;
      float s = 0.f;
      for (int m = 0; m < M; ++m) s += tr[m];
      const int c = g0 * kSharedGroupCurves + cl, k = f0 + fl;
      if (c < a.n_curves && k < a.n_freq) {
        const CurveConst cc = a.cc[c];
        a.S[(int64_t)c * a.n_freq + k] = s * cc.kc * cc.scale;
      }
    }
    wave_lds_fence();
  }
}

}  // namespace

void shared_shape(int n_bins, int* nb, int* fw) {
  // column use of nb tiles: fw M / (32 nb); three tiles read each A operand
  // once for three products instead of two, so they win ties
  const int f2 = std::min(kSharedMaxFw, 64 / n_bins), f3 = std::min(kSharedMaxFw, 96 / n_bins);
  const double u2 = f2 * n_bins / 64.0, u3 = f3 * n_bins / 96.0;
  // (with M = 64 two tiles hold exactly one frequency: no padding column,
  // which the one-hot form relies on)
  if (u3 >= u2 - 0.01 && n_bins < 64) {
    *nb = 3;
    *fw = f3;
  } else {
    *nb = 2;
    *fw = f2;
  }
}

hipError_t launch_shared(const SharedArgs& a, int phase, int curve_groups, int nb, int grid_x, int grid_y,
                         size_t lds_bytes, hipStream_t s) {
  if (curve_groups != 4 || (nb != 2 && nb != 3)) return hipErrorInvalidValue;
  const bool lst = phase == PH_LISTING;
  const void* fn = nb == 3 ? (lst ? (const void*)shared_kernel<PH_LISTING, 4, 3> : (const void*)shared_kernel<PH_FP64, 4, 3>)
                           : (lst ? (const void*)shared_kernel<PH_LISTING, 4, 2> : (const void*)shared_kernel<PH_FP64, 4, 2>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  SharedArgs args = a;
  void* params[] = {&args};
  return hipLaunchKernel(fn, dim3((unsigned)grid_x, (unsigned)grid_y), dim3(kSharedWaves * kWave), params, lds_bytes, s);
}

}  // namespace fpw
