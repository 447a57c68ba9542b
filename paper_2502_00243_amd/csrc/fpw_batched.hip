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
//  * each lane owns a histogram of M+1 packed 64-bit fixed-point words in
//    LDS, laid out [bin][lane] so the 64 lanes of a wave always hit distinct
//    banks whatever their bins are;
//  * one `ds_add_u64` per (observation, frequency) accumulates both sums
//    exactly: the weight sits in the high word, the weighted residual in the
//    low word, and integer addition carries them without rounding;
//  * the phase is formed in FP64 (full rate on CDNA), and the bin index
//    comes out of the low word of one more FP64 fma, so a fold costs three
//    FP64 instructions plus the LDS address;
//  * work is a queue of (curve, frequency chunk) items, longest curves first,
//    popped by persistent waves (or groups of waves) with one atomic each
//    (small plans: one item per wave or group, taken by index);
//    the peak selection is fused so that large periodograms never reach HBM;
//  * for large M a histogram per wave leaves room for few waves per CU, so
//    SH > 1 waves of a workgroup share one: each folds a contiguous slice of
//    the curve's observations into it (LDS atomics from different waves add
//    up exactly), then each reduces whole parts of the bin sum and wave 0
//    adds the part sums in order;
//  * S is summed in one fixed order for every launch shape (see kSumParts),
//    so the result does not depend on the shape.
#include "fpw_common.h"

namespace fpw {
namespace {

using namespace dev;

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

// Where a wave's observations come from.
//  SRC_SCALAR: wave-uniform scalar loads (8 records per batch) into SGPRs; tau
//    is an SGPR operand of the fold and the packed word takes one v_mov_b64.
//    Waiting for a scalar load also waits for the wave's outstanding LDS
//    atomics, which high occupancy (small M) hides.
//  SRC_DPP: one coalesced vector load brings 16 records into every row of 16
//    lanes; each record is broadcast with two 64-bit DPP row_newbcast moves.
//    Only vector-memory counters are waited on, so LDS atomics stay in
//    flight; this suits large M, where the histograms leave room for few
//    waves per CU.
//  SRC_LANES (fused pass of small plans): each lane forms the record of one
//    observation of a block of 64 and the wave broadcasts them one by one
//    with readlane, so the fold waits on no memory at all.
enum { SRC_SCALAR = 0, SRC_DPP = 1, SRC_LANES = 2 };

// The observations of a wave: the prepared records (scalar and DPP
// sources), or, in the fused pass, records formed on the fly from the raw
// inputs and the curve's constants (SRC_LANES).
struct RecSource {
  const Rec* __restrict__ rc;
  __device__ __forceinline__ Rec operator()(int i) const { return rc[i]; }
};
// SRC_LANES: the wave takes the blocks of 64 observations that start at
// first, first + stride, ... (below n_all) of a curve; `r0` is the lane's
// record of the first block, formed beforehand.
template <int PH>
struct LaneSource {
  const double* __restrict__ t;
  const double* __restrict__ y;
  const double* __restrict__ dy;
  PrepConst k;
  int first, stride, n_all;
  Rec r0;
  __device__ __forceinline__ Rec operator()(int i) const { return make_rec(t[i], y[i], dy[i], k, PH); }
};

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int q) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, q);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), q);
  return ((uint64_t)hi << 32) | lo;
}

template <int PH, int FL, int SRC, class Src>
__device__ __forceinline__ void accumulate(const Src& src, int n, const Folder<PH> (&fo)[FL],
                                           uint64_t* const (&h)[FL], int lane) {
  if constexpr (SRC == SRC_LANES) {
    for (int base = src.first; base < src.n_all; base += src.stride) {
      const int cnt = min(kWave, src.n_all - base);  // wave-uniform
      const Rec r = base == src.first ? src.r0 : src(base + (lane < cnt ? lane : cnt - 1));
      int q = 0;
      for (; q + 4 <= cnt; q += 4) {
        // four bins formed side by side before their atomics, so the FP64 chains overlap
        const uint64_t t0 = lane_u64(r.tau_bits, q), t1 = lane_u64(r.tau_bits, q + 1);
        const uint64_t t2 = lane_u64(r.tau_bits, q + 2), t3 = lane_u64(r.tau_bits, q + 3);
#pragma unroll
        for (int j = 0; j < FL; ++j) {
          const int b0 = fo[j].bin(t0), b1 = fo[j].bin(t1), b2 = fo[j].bin(t2), b3 = fo[j].bin(t3);
          lds_add(h[j] + b0 * kWave, uniform_to_vgpr(lane_u64(r.pk, q)));
          lds_add(h[j] + b1 * kWave, uniform_to_vgpr(lane_u64(r.pk, q + 1)));
          lds_add(h[j] + b2 * kWave, uniform_to_vgpr(lane_u64(r.pk, q + 2)));
          lds_add(h[j] + b3 * kWave, uniform_to_vgpr(lane_u64(r.pk, q + 3)));
        }
      }
      for (; q < cnt; ++q) {
        const uint64_t tb = lane_u64(r.tau_bits, q);
        const uint64_t pk = uniform_to_vgpr(lane_u64(r.pk, q));
#pragma unroll
        for (int j = 0; j < FL; ++j) lds_add(h[j] + fo[j].bin(tb) * kWave, pk);
      }
    }
  } else if constexpr (SRC == SRC_SCALAR) {
    const Rec* __restrict__ rc = src.rc;
    int i = 0;
    for (; i + kBatch <= n; i += kBatch) {
      Rec r[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) r[q] = rc[i + q];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const uint64_t pk = uniform_to_vgpr(r[q].pk);
#pragma unroll
        for (int j = 0; j < FL; ++j) lds_add(h[j] + fo[j].bin(r[q].tau_bits) * kWave, pk);
      }
    }
    for (; i < n; ++i) {
      const Rec r = rc[i];
      const uint64_t pk = uniform_to_vgpr(r.pk);
#pragma unroll
      for (int j = 0; j < FL; ++j) lds_add(h[j] + fo[j].bin(r.tau_bits) * kWave, pk);
    }
  } else {
    constexpr int kGroup = 16;
    const int sub = lane & (kGroup - 1);
    Rec cur = src(sub < n ? sub : n - 1);
    for (int g = 0; g < n; g += kGroup) {
      const int nxt = g + kGroup + sub;
      const Rec next = src(nxt < n ? nxt : n - 1);  // prefetch (clamped, always in bounds)
      const int cnt = n - g;  // wave-uniform
      if (cnt >= kGroup) {
        // a full group, straight-line: bins of four points are formed side by
        // side before their four atomics, so the FP64 chains overlap
        static_for<0, kGroup / 4>([&](auto rc4) {
          constexpr int q0 = 4 * decltype(rc4)::value;
          const uint64_t t0 = row_bcast<q0>(cur.tau_bits), t1 = row_bcast<q0 + 1>(cur.tau_bits);
          const uint64_t t2 = row_bcast<q0 + 2>(cur.tau_bits), t3 = row_bcast<q0 + 3>(cur.tau_bits);
#pragma unroll
          for (int j = 0; j < FL; ++j) {
            const int b0 = fo[j].bin(t0), b1 = fo[j].bin(t1), b2 = fo[j].bin(t2), b3 = fo[j].bin(t3);
            lds_add(h[j] + b0 * kWave, row_bcast<q0>(cur.pk));
            lds_add(h[j] + b1 * kWave, row_bcast<q0 + 1>(cur.pk));
            lds_add(h[j] + b2 * kWave, row_bcast<q0 + 2>(cur.pk));
            lds_add(h[j] + b3 * kWave, row_bcast<q0 + 3>(cur.pk));
          }
        });
      } else {
        static_for<0, kGroup>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if (q < cnt) {
            const uint64_t tb = row_bcast<q>(cur.tau_bits);
            const uint64_t pk = row_bcast<q>(cur.pk);
#pragma unroll
            for (int j = 0; j < FL; ++j) lds_add(h[j] + fo[j].bin(tb) * kWave, pk);
          }
        });
      }
      cur = next;
    }
  }
}

// One derived variant (k fine bins per coarse bin, the first coarse bin
// starting at fine bin o; Sec. 3.4) from prefix slots.  The slots are split
// into R consecutive ranges, range r = slots lo[r] .. lo[r+1]-1 (lo[R] = M);
// a slot x that a window reads holds L(x) = F(lo[r]) + ... + F(x) for its
// range r, base[r] = F(0) + ... + F(lo[r] - 1), and base[R] is the total.
// The windows are taken in order, the one that wraps around the end last;
// each window's packed sum is the difference of two prefixes (exact in
// 64-bit wrap-around arithmetic), and a range's base enters once per range,
// not once per window.  Slots past a range's last window are read in the
// batches of four but not used.
template <int R>
__device__ __forceinline__ float derived_sum(const uint64_t* h, int M, int k, int o, const int (&lo)[R + 1],
                                             const uint64_t (&base)[R + 1], float ia2q) {
  // F(0) + ... + F(o - 1), the prefix before the first window (0 when o == 0)
  uint64_t start = 0;
  if (o > 0) {
    uint64_t b = base[0];
#pragma unroll
    for (int r = 1; r < R; ++r)
      if (o - 1 >= lo[r]) b = base[r];  // the last range starting at or before o - 1 holds it
    start = b + h[(o - 1) * kWave];
  }
  uint64_t prev_p = start;  // prefix through the last slot of the previous window
  int e = o + k - 1;        // last slot of the next window
  float out = 0.f;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int hi = lo[r + 1];
    if (e >= hi) continue;
    uint64_t prev = prev_p - base[r];
    while (e < hi) {
      uint64_t pe[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) pe[q] = h[min(e + q * k, M) * kWave];
      int next = e;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (e + q * k < hi) {
          out = add_bin_term(out, pe[q] - prev, ia2q);
          prev = pe[q];
          next = e + (q + 1) * k;
        }
      }
      e = next;
    }
    prev_p = prev + base[r];
  }
  if (o > 0) out = add_bin_term(out, base[R] - prev_p + start, ia2q);  // the window that wraps around
  return out;
}

// Clears the prefix slots (need bits) in [lo, hi).
__device__ __forceinline__ void clear_need_range(uint64_t* h, int lo, int hi, const Variants& vs) {
  for (int w = lo >> 5; w * 32 < hi; ++w) {
    uint32_t bits = vs.need[w];
    while (bits) {
      const int m = w * 32 + __builtin_ctz(bits);
      bits &= bits - 1;
      if (m >= lo && m < hi) h[m * kWave] = 0;
    }
  }
}

// Reduces one lane's fine histogram for every variant: variant v sums k[v]
// consecutive fine bins (from fine bin o[v], cyclically) into each coarse
// bin, exactly, then adds the Eq. 1 terms.
//  1. One pass over the fine bins in order, read and cleared eight at a time:
//     variant 0 (the fine bins themselves) takes its terms directly, and the
//     running prefix F(0) + ... + F(m) is written back only to the slots
//     some derived variant reads.
//  2. Each derived variant walks its windows (derived_sum, one range); then
//     the prefix slots are cleared.
template <int PH, int NV>
__device__ __forceinline__ void reduce_variants(uint64_t* h, int M, float ia2q, const Variants& vs, float (&out)[NV]) {
  const uint64_t wrap = take_wrap_slot<PH>(h, M);
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  uint64_t run = 0;
  float fine = 0.f, fine_parts = 0.f;  // variant 0 in the order of reduce_hist
  int part = 0;
  for (int m0 = 0, b = 0; m0 < M; m0 += kReduceBlock, ++b) {
    while (part < kSumParts && b == part_block(part + 1, nb)) {  // the parts ending here (empty ones add 0)
      fine_parts += fine;
      fine = 0.f;
      ++part;
    }
    uint64_t f[kReduceBlock];
    take_block<PH>(h, M, m0, f);
    if (m0 == 0) f[0] += wrap;
#pragma unroll
    for (int q = 0; q < kReduceBlock; ++q) {
      const int m = m0 + q;
      if (m < M) {
        run += f[q];
        fine = add_bin_term(fine, f[q], ia2q);
        if ((vs.need[m >> 5] >> (m & 31)) & 1u) h[m * kWave] = run;
      }
    }
  }
  out[0] = fine_parts + fine;
  const int lo[2] = {0, M};
  const uint64_t base[2] = {0, run};
#pragma unroll
  for (int v = 1; v < NV; ++v) out[v] = v < vs.n ? derived_sum<1>(h, M, vs.k[v], vs.o[v], lo, base, ia2q) : 0.f;
  clear_need_range(h, 0, M, vs);
}

// The part sums of reduce_hist that one wave of a histogram shared by SH
// waves owns (parts [w K/SH, (w+1) K/SH), K = kSumParts), read and cleared,
// each written to part_sums[p][lane].  The wave whose first block is block 0
// also takes the wrap slot.  Slots of other waves' parts are neither read
// nor cleared.
template <int PH, int SH>
__device__ __forceinline__ void reduce_parts(uint64_t* h, int M, int wave, float ia2q, float* part_sums, int lane) {
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  const int p0 = wave * kSumParts / SH, p1 = (wave + 1) * kSumParts / SH;
  const bool first = part_block(p0, nb) == 0 && part_block(p1, nb) > 0;
  const uint64_t wrap = first ? take_wrap_slot<PH>(h, M) : (uint64_t)0;
  for (int p = p0; p < p1; ++p) {
    float acc = 0.f;
    for (int b = part_block(p, nb); b < part_block(p + 1, nb); ++b) {
      const int m0 = b * kReduceBlock;
      uint64_t f[kReduceBlock];
#pragma unroll
      for (int q = 0; q < kReduceBlock; ++q) f[q] = m0 + q < M ? lds_take(h + (m0 + q) * kWave) : (uint64_t)0;
      if (m0 == 0) f[0] += wrap;
#pragma unroll
      for (int q = 0; q < kReduceBlock; ++q)
        if (m0 + q < M) acc = add_bin_term(acc, f[q], ia2q);
    }
    part_sums[p * kWave + lane] = acc;
  }
}

// Several variants from a histogram shared by SH waves (the reduction of
// reduce_variants split over the waves).
//  Phase 1 (every wave, its own parts as in reduce_parts): takes the fine
//    slots, writes the part sums of variant 0 to part_sums, writes the prefix
//    of its own range (from the range start) back to the slots a derived
//    variant reads, and its range total to totals[wave].
//  Phase 2 (after a barrier): the wave computes the derived variants it owns
//    (Variants::own, balanced on the host) with derived_sum over the SH
//    ranges, the bases being sums of the range totals.  Reads are plain: a
//    slot may serve variants of several waves.  The sums stay in the owner's
//    registers: the owner also stores those variants' S and keeps their
//    peaks.
//  Then (after a barrier) each wave clears the prefix slots of its range.
template <int PH, int SH>
__device__ __forceinline__ void variants_phase1(uint64_t* h, int M, int wave, float ia2q, const Variants& vs,
                                                float* part_sums, uint64_t* totals, int lane) {
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  const int p0 = wave * kSumParts / SH, p1 = (wave + 1) * kSumParts / SH;
  const bool first = part_block(p0, nb) == 0 && part_block(p1, nb) > 0;
  const uint64_t wrap = first ? take_wrap_slot<PH>(h, M) : (uint64_t)0;
  uint64_t run = 0;
  for (int p = p0; p < p1; ++p) {
    float acc = 0.f;
    for (int b = part_block(p, nb); b < part_block(p + 1, nb); ++b) {
      const int m0 = b * kReduceBlock;
      uint64_t f[kReduceBlock];
#pragma unroll
      for (int q = 0; q < kReduceBlock; ++q) f[q] = m0 + q < M ? lds_take(h + (m0 + q) * kWave) : (uint64_t)0;
      if (m0 == 0) f[0] += wrap;
#pragma unroll
      for (int q = 0; q < kReduceBlock; ++q) {
        const int m = m0 + q;
        if (m < M) {
          run += f[q];
          acc = add_bin_term(acc, f[q], ia2q);
          if ((vs.need[m >> 5] >> (m & 31)) & 1u) h[m * kWave] = run;
        }
      }
    }
    part_sums[p * kWave + lane] = acc;
  }
  totals[wave * kWave + lane] = run;
}

// Derived variants per wave (at most): the kernel's register slots for them.
template <int NV, int SH>
constexpr int kOwned = (NV - 1 + SH - 1) / SH;

template <int NV, int SH>
__device__ __forceinline__ void variants_phase2(const uint64_t* h, int M, int wave, float ia2q, const Variants& vs,
                                                const uint64_t* totals, float (&own)[kOwned<NV, SH>], int lane) {
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  int lo[SH + 1];
  uint64_t base[SH + 1];
  lo[0] = 0;
  base[0] = 0;
#pragma unroll
  for (int r = 1; r <= SH; ++r) {
    lo[r] = r < SH ? min(M, part_block(r * kSumParts / SH, nb) * kReduceBlock) : M;
    base[r] = base[r - 1] + totals[(r - 1) * kWave + lane];
  }
#pragma unroll
  for (int j = 0; j < kOwned<NV, SH>; ++j) {
    const int v = vs.own[SH == 4][wave][j];
    own[j] = v == 0 ? 0.f : derived_sum<SH>(h, M, vs.k[v], vs.o[v], lo, base, ia2q);
  }
}

// Clears the prefix slots (need bits) of this wave's range.
template <int SH>
__device__ __forceinline__ void clear_need_slots(uint64_t* h, int M, int wave, const Variants& vs) {
  const int nb = (M + kReduceBlock - 1) / kReduceBlock;
  clear_need_range(h, part_block(wave * kSumParts / SH, nb) * kReduceBlock,
                   min(M, part_block((wave + 1) * kSumParts / SH, nb) * kReduceBlock), vs);
}

// Peak bookkeeping of one periodogram variant along a work item.
struct PeakState {
  WaveTop top;
  float pend_s, pend_left;  // S at kb-1 and kb-2 (wave-uniform)
  __device__ __forceinline__ void init() {
    top.init();
    pend_s = -INFINITY;
    pend_left = -INFINITY;
  }
  // One sub-tile of 64 frequencies kb .. kb+63 (lane = kb + lane), S value s.
  // `pend`: index kb-1 still waits for its right neighbour.  Writes the four
  // chunk-edge values to e.
  __device__ __forceinline__ void step(float s, int kb, int k0, int k1, int n_freq, bool pend, int topk, float* e,
                                       int lane) {
    const int k = kb + lane;
    const bool valid = k < k1;
    const float sv = valid ? s : -INFINITY;
    const float up = from_lane_below(sv);
    const float dn = from_lane_above(sv);
    const float s0 = lane_value(sv, 0);
    // index kb-1 (lane 63 of the previous sub-tile) now has its right neighbour
    if (pend && pend_s > pend_left && pend_s >= s0) top.offer(pend_s, kb - 1, lane == 0, topk, lane);
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
    if (k == k1 - 1) {
      right = -INFINITY;
      decided = decided && k1 == n_freq;
    } else if (lane == kWave - 1) {
      decided = false;  // deferred to the next sub-tile
    }
    top.offer(s, k, decided && s > left && s >= right, topk, lane);
    pend_s = lane_value(sv, kWave - 1);
    pend_left = lane_value(sv, kWave - 2);
    // chunk-edge values for the merge
    if (valid) {
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
};

// SH > 1: the SH waves of the workgroup work on the same item with one shared
// histogram; `part` holds the kSumParts part sums of S, and with several
// variants `totals` the range totals.  With one variant only wave 0 (the
// lead) stores S and keeps the peaks; with several, each wave stores and
// keeps the peaks of the derived variants it computed (Variants::own) and
// the lead those of variant 0, so the work after the last barrier of a
// sub-tile is spread over the group and each wave holds few peak states.
// The observations [lo, lo + n) of a curve of n_all that wave `wave` of SH
// folds (all of them when SH == 1).
template <int SH>
__device__ __forceinline__ int slice_begin(int wave, int n_all) {
  return SH > 1 ? (int)((int64_t)wave * n_all / SH) : 0;
}
template <int SH>
__device__ __forceinline__ int slice_size(int wave, int n_all) {
  return SH > 1 ? (int)((int64_t)(wave + 1) * n_all / SH) - slice_begin<SH>(wave, n_all) : n_all;
}

// With one periodogram and fused peaks, the lead wave also sums the part
// sums, stores S and steps the peak list after a sub-tile's last barrier,
// while the other waves already fold the next sub-tile; it folds
// kLeadLighter observations fewer than an even share (the others split the
// rest evenly), so the waves reach the next barrier closer together
// (measured 0.1-2 % per pass across plan sizes; the sums, being integer, do
// not depend on the split).
constexpr int kLeadLighter = 16;
template <int SH, bool LIGHT>
__device__ __forceinline__ void lead_slices(int wave, int n_all, int& lo, int& n) {
  if constexpr (SH == 1 || !LIGHT) {
    lo = slice_begin<SH>(wave, n_all);
    n = slice_size<SH>(wave, n_all);
  } else {
    const int b1 = max(0, n_all / SH - kLeadLighter);
    if (wave == 0) {
      lo = 0;
      n = b1;
    } else {
      lo = b1 + (int)((int64_t)(wave - 1) * (n_all - b1) / (SH - 1));
      n = b1 + (int)((int64_t)wave * (n_all - b1) / (SH - 1)) - lo;
    }
  }
}

// One work item: `src` yields this wave's n observations of the item's
// curve, `cc` holds the curve's constants.
// `f_first`, if set, holds the lane's frequency of the item's first
// sub-tile (loaded early by the caller).
template <int PH, int FL, int PK, int SRC, int NV, int SH, class Src>
__device__ __forceinline__ void process_item(const BatchArgs& a, const RO& ro, const Item& item, const CurveConst cc,
                                             const Src& src, int n, uint64_t* hist, int lane, int wave, float* part,
                                             uint64_t* totals, const double* f_first = nullptr) {
  static_assert(SH == 1 || FL == 1, "a shared histogram serves one frequency per lane");
  static_assert(kSumParts % SH == 0, "each wave owns whole parts of the sum");
  const int M = a.n_bins;
  const int slots = M + 1;
  const int c = item.curve, k0 = item.k0, k1 = item.k1;
  const bool lead = SH == 1 || wave == 0;
  const float outscale = cc.kc * cc.scale;
  const int nvar = NV == 1 ? 1 : a.var.n;
  const int64_t var_stride = (int64_t)a.n_curves * a.n_freq;
  // periodograms this wave stores and keeps peaks for: slot p is variant
  // slot_var(p) (NV stands for none)
  constexpr bool kSplit = SH > 1 && NV > 1;
  constexpr int NP = kSplit ? kOwned<NV, SH> + 1 : NV;
  auto slot_var = [&](int p) -> int {
    if constexpr (!kSplit) return p;
    if (p == 0) return lead ? 0 : NV;
    const int v = a.var.own[SH == 4][wave][p - 1];
    return v == 0 ? NV : v;
  };

  PeakState peaks[NP];
  if (PK) {
#pragma unroll
    for (int p = 0; p < NP; ++p) peaks[p].init();
  }
  bool pend = false;  // the last index of the previous sub-tile waits for its right neighbour

  for (int kt = k0; kt < k1; kt += FL * kWave) {
    Folder<PH> fo[FL];
    uint64_t* h[FL];
#pragma unroll
    for (int j = 0; j < FL; ++j) {
      const int k = kt + j * kWave + lane;
      fo[j].init(f_first != nullptr && FL == 1 && kt == k0 ? *f_first : ro.freqs[k < k1 ? k : k1 - 1], M, a.fold_nh);
      h[j] = hist + (j * slots) * kWave + lane;
    }
    // fold, bin and accumulate every observation of the curve (of this wave's slice)
    if (SH == 1 || n > 0) accumulate<PH, FL, SRC>(src, n, fo, h, lane);
    // reduce each sub-tile of 64 frequencies, store, and pick peaks
#pragma unroll
    for (int j = 0; j < FL; ++j) {
      const int kb = kt + j * kWave;
      if (kb >= k1) break;
      float sv[NP];
      if constexpr (SH > 1 && NV == 1) {
        __syncthreads();  // every slice is in the histogram
        reduce_parts<PH, SH>(h[j], M, wave, cc.ia2q, part, lane);
        __syncthreads();  // part sums visible, histogram clear for the next sub-tile
        if (!lead) continue;
        float s = 0.f;
#pragma unroll
        for (int p = 0; p < kSumParts; ++p) s += part[p * kWave + lane];
        sv[0] = s;
      } else if constexpr (SH > 1) {
        __syncthreads();  // every slice is in the histogram
        variants_phase1<PH, SH>(h[j], M, wave, cc.ia2q, a.var, part, totals, lane);
        __syncthreads();  // prefixes, range totals and part sums visible
        float own[kOwned<NV, SH>];
        variants_phase2<NV, SH>(h[j], M, wave, cc.ia2q, a.var, totals, own, lane);
        float s0 = 0.f;
        if (lead) {
#pragma unroll
          for (int p = 0; p < kSumParts; ++p) s0 += part[p * kWave + lane];
        }
        __syncthreads();  // every derived variant has read its prefixes, the lead the part sums
        clear_need_slots<SH>(h[j], M, wave, a.var);
        __syncthreads();  // histogram clear for the next sub-tile
        sv[0] = s0;
#pragma unroll
        for (int q = 0; q < kOwned<NV, SH>; ++q) sv[1 + q] = own[q];
      } else if constexpr (NV == 1) {
        sv[0] = reduce_hist<PH>(h[j], M, cc.ia2q);
      } else {
        reduce_variants<PH, NV>(h[j], M, cc.ia2q, a.var, sv);
      }
      const int k = kb + lane;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int v = slot_var(p);
        if (v < nvar) {
          const float s = outscale * sv[p];
          if (a.S != nullptr && k < k1) a.S[v * var_stride + (int64_t)c * a.n_freq + k] = s;
          if (PK) peaks[p].step(s, kb, k0, k1, a.n_freq, pend, a.topk, a.edge + ((int64_t)item.slot * nvar + v) * 4, lane);
        }
      }
      pend = kb + kWave - 1 < k1 - 1;
    }
  }
  if (PK && (kSplit || lead)) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int v = slot_var(p);
      if (v < nvar) {
        const int64_t o = ((int64_t)item.slot * nvar + v) * a.topk;
        peaks[p].top.store(a.topk, a.cand_val + o, a.cand_idx + o, lane);
      }
    }
  }
}

// The DPP-source shapes with private histograms serve large M, where LDS
// admits at most ~2 waves per SIMD; telling the compiler so lets it spend
// registers on overlapping the FP64 fold chains instead of minimising them.
//
// LDS: SH == 1: one histogram set per wave, [wave][j][bin][lane].  SH > 1
// (the workgroup is the SH waves of one histogram): [bin][lane], then the
// part sums [kSumParts][lane] (float), with several variants the range
// totals [SH][lane] (64-bit), and the item index of the group.
template <int PH, int FL, int PK, int SRC, int NV, int SH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, SRC == SRC_DPP && SH == 1 ? 2 : 10))) void batched_kernel(BatchArgs a, const Rec* __restrict__ rec,
                                                      const int64_t* __restrict__ offsets,
                                                      const CurveConst* __restrict__ ccs,
                                                      const double* __restrict__ freqs,
                                                      const Item* __restrict__ items) {
  const RO ro{rec, offsets, ccs, freqs};
  extern __shared__ __align__(16) uint64_t lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform: keeps slice loads scalar
  const int slots = a.n_bins + 1;
  uint64_t* hist = lds + (SH > 1 ? (size_t)0 : (size_t)wave * FL * slots * kWave);
  float* part = reinterpret_cast<float*>(lds + (size_t)slots * kWave);
  uint64_t* totals = reinterpret_cast<uint64_t*>(part + kSumParts * kWave);  // used when NV > 1
  int* group_item = reinterpret_cast<int*>(totals + (NV > 1 ? SH * kWave : 0));
  if (SH > 1) {
    for (int s = wave; s < slots; s += SH) hist[s * kWave + lane] = 0;
    // every wave clears its own slots but folds into all of them: the
    // clearing must be complete before any wave's first atomic (the queue
    // path has a barrier after its pop; taking items by index has none)
    __syncthreads();
  } else {
    for (int s = 0; s < FL * slots; ++s) hist[s * kWave + lane] = 0;
  }
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
    const int64_t p0 = ro.offsets[item.curve];
    const int n_all = (int)(ro.offsets[item.curve + 1] - p0);
    int lo = 0, ns = 0;
    lead_slices<SH, NV == 1 && PK == 1>(wave, n_all, lo, ns);
    const RecSource src{ro.rec + p0 + lo};
    process_item<PH, FL, PK, SRC, NV, SH>(a, ro, item, ro.cc[item.curve], src, ns, hist, lane, wave, part, totals);
  }
}

// ---------------------------------------------------------------- wide-format kernel
// Curves whose weights span too wide a range for the packed 32-bit fields
// (fpw_plan decides per curve) keep their per-bin sums in two 64-bit words:
// the weight and the weighted residual each take their own ds_add_u64 (the
// second at a 512-byte offset from the first), and the epilogue decodes them
// to FP64.  Otherwise the kernel works as the batched one: one lane per
// frequency, wave-uniform scalar loads of the records (four 32-byte records
// per batch), items taken from the second queue counter, SH waves sharing a
// histogram, the bin terms summed in the same fixed part order, fused peaks.

template <int PH>
__device__ __forceinline__ void accumulate_wide(const WRec* __restrict__ rc, int n, const Folder<PH>& fo, uint64_t* h) {
  constexpr int kWideBatch = 4;
  int i = 0;
  for (; i + kWideBatch <= n; i += kWideBatch) {
    WRec r[kWideBatch];
#pragma unroll
    for (int q = 0; q < kWideBatch; ++q) r[q] = rc[i + q];
#pragma unroll
    for (int q = 0; q < kWideBatch; ++q) {
      uint64_t* sl = h + fo.bin(r[q].tau_bits) * kWideSlotWords;
      lds_add(sl, uniform_to_vgpr(r[q].wq));
      lds_add(sl + kWave, uniform_to_vgpr(r[q].yq));
    }
  }
  for (; i < n; ++i) {
    const WRec r = rc[i];
    uint64_t* sl = h + fo.bin(r.tau_bits) * kWideSlotWords;
    lds_add(sl, uniform_to_vgpr(r.wq));
    lds_add(sl + kWave, uniform_to_vgpr(r.yq));
  }
}

// One work item of a wide-format curve; `rc` holds this wave's n records.
template <int PH, int PK, int SH>
__device__ __forceinline__ void process_item_wide(const BatchArgs& a, const double* __restrict__ freqs, const Item& item,
                                                  const WideConst wc, const WRec* __restrict__ rc, int n,
                                                  uint64_t* hist, int lane, int wave, double* part) {
  static_assert(kSumParts % SH == 0, "each wave owns whole parts of the sum");
  const int M = a.n_bins;
  const int c = item.curve, k0 = item.k0, k1 = item.k1;
  const bool lead = SH == 1 || wave == 0;
  uint64_t* h = hist + lane;
  PeakState peaks;
  if (PK) peaks.init();
  bool pend = false;
  for (int kb = k0; kb < k1; kb += kWave) {
    const int k = kb + lane;
    Folder<PH> fo;
    fo.init(freqs[k < k1 ? k : k1 - 1], M, a.fold_nh);
    if (SH == 1 || n > 0) accumulate_wide<PH>(rc, n, fo, h);
    double sum = 0.0;
    if constexpr (SH > 1) {
      constexpr int NP = kSumParts / SH;
      __syncthreads();  // every slice is in the histogram
      double ps[NP];
      wide_parts<PH, NP>(h, M, wave * NP, wc, ps);
#pragma unroll
      for (int q = 0; q < NP; ++q) part[(wave * NP + q) * kWave + lane] = ps[q];
      __syncthreads();  // part sums visible, histogram clear for the next sub-tile
      if (!lead) continue;
#pragma unroll
      for (int p = 0; p < kSumParts; ++p) sum += part[p * kWave + lane];
    } else {
      double ps[kSumParts];
      wide_parts<PH, kSumParts>(h, M, 0, wc, ps);
#pragma unroll
      for (int p = 0; p < kSumParts; ++p) sum += ps[p];
    }
    const float sv = (float)(sum * wc.scale);
    if (a.S != nullptr && k < k1) a.S[(int64_t)c * a.n_freq + k] = sv;
    if (PK) peaks.step(sv, kb, k0, k1, a.n_freq, pend, a.topk, a.edge + (int64_t)item.slot * 4, lane);
    pend = kb + kWave - 1 < k1 - 1;
  }
  if (PK && lead) {
    const int64_t o = (int64_t)item.slot * a.topk;
    peaks.top.store(a.topk, a.cand_val + o, a.cand_idx + o, lane);
  }
}

// LDS: SH == 1: one wave per workgroup, its histogram [slot][2][lane];
// SH > 1: the group's histogram, then the part sums [kSumParts][lane]
// (FP64) and the group's item index.
template <int PH, int PK, int SH>
__global__ __launch_bounds__(64 * SH) void wide_kernel(BatchArgs a, const WRec* __restrict__ recw,
                                                       const int64_t* __restrict__ offw,
                                                       const WideConst* __restrict__ wcs,
                                                       const double* __restrict__ freqs,
                                                       const Item* __restrict__ items) {
  extern __shared__ __align__(16) uint64_t lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform: keeps slice loads scalar
  const int slots = a.n_bins + 1;
  uint64_t* hist = lds;
  double* part = reinterpret_cast<double*>(lds + (size_t)slots * kWideSlotWords);
  int* group_item = reinterpret_cast<int*>(part + kSumParts * kWave);
  for (int sl = wave; sl < slots; sl += SH) {
    hist[sl * kWideSlotWords + lane] = 0;
    hist[sl * kWideSlotWords + kWave + lane] = 0;
  }
  if (SH > 1) __syncthreads();  // every slot is clear before any wave folds into it
  // as in the batched kernel: by index with at most one item per consumer,
  // else every item (the first too) popped from this launch's counter
  const bool by_index = a.n_items <= (int)gridDim.x;
  for (int round = 0;; ++round) {
    int it = 0;
    if (by_index) {
      if (round > 0) break;
      it = (int)blockIdx.x;
    } else if (SH > 1) {
      if (threadIdx.x == 0) *group_item = (int)atomicAdd(a.queue, 1u);
      __syncthreads();
      it = __builtin_amdgcn_readfirstlane(*group_item);
    } else {
      if (lane == 0) it = (int)atomicAdd(a.queue, 1u);
      it = __builtin_amdgcn_readfirstlane(it);
    }
    if (it >= a.n_items) break;
    const Item item = items[it];
    const int64_t p0 = offw[item.curve];
    const int n_all = (int)(offw[item.curve + 1] - p0);
    const int lo = slice_begin<SH>(wave, n_all);
    process_item_wide<PH, PK, SH>(a, freqs, item, wcs[item.curve], recw + p0 + lo, slice_size<SH>(wave, n_all), hist,
                                  lane, wave, part);
  }
}

template <int PH, int PK>
void* wide_ptr_sh(int share) {
  return share == 4 ? (void*)&wide_kernel<PH, PK, 4>
                    : (share == 2 ? (void*)&wide_kernel<PH, PK, 2> : (void*)&wide_kernel<PH, PK, 1>);
}

// Built for the FP64 folds (fused and listing order).
void* wide_fn(int phase, int pk, int share) {
  if (phase == PH_FP64) return pk ? wide_ptr_sh<PH_FP64, 1>(share) : wide_ptr_sh<PH_FP64, 0>(share);
  if (phase == PH_LISTING) return pk ? wide_ptr_sh<PH_LISTING, 1>(share) : wide_ptr_sh<PH_LISTING, 0>(share);
  return nullptr;
}

// ---------------------------------------------------------------- fused pass
// For small plans the dependent launches of a pass cost more than their
// work.  Here the prepare step is fused into the fold: one workgroup of four
// waves per work item reduces the curve's constants (the prepare kernel's
// function, so the same values); wave w folds the blocks of 64 observations
// starting at 64 w, 64 w + 256, ... into the shared histogram from records
// its lanes form (the prepare kernel's records, bit for bit) and broadcast
// with readlane; the item's S and candidate peaks are stored as by the
// batched kernel.  Items map to workgroups one to one; there is no queue.
// The per-curve merge follows as its own kernel: merging here would need a
// device-wide release of every item's candidates, which costs more on this
// chip (its L2 is per XCD) than the launch boundary.
constexpr int kFusedShare = 4;

template <int PH, int PK>
__global__ __launch_bounds__(kFusedShare * kWave) void fused_kernel(BatchArgs a, FusedArgs o) {
  extern __shared__ __align__(16) uint64_t lds[];
  __shared__ double red[kPrepRed];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform: keeps slice loads scalar
  const Item item = a.items[blockIdx.x];
  const int c = item.curve;
  const int64_t p0 = a.offsets[c];
  const int n_all = (int)(a.offsets[c + 1] - p0);
  const int slots = a.n_bins + 1;
  uint64_t* hist = lds;
  float* part = reinterpret_cast<float*>(lds + (size_t)slots * kWave);
  for (int s = wave; s < slots; s += kFusedShare) hist[s * kWave + lane] = 0;
  // (the barriers of curve_prep order the clearing before any accumulation)
  // the first sub-tile's frequency, loaded while the curve is reduced
  const double f0 = a.freqs[min(item.k0 + lane, item.k1 - 1)];
  // thread t = 64 w + lane reads observation t in curve_prep, which is this
  // lane's observation of wave w's first block: its record needs no reload
  double keep[3];
  const PrepConst k = curve_prep(o.t + p0, o.y + p0, o.dy + p0, n_all, o.center, o.tref_mode, o.t_ref, red, keep);
  const LaneSource<PH> src{o.t + p0, o.y + p0, o.dy + p0, k, wave * kWave, kFusedShare * kWave, n_all,
                           make_rec(keep[0], keep[1], keep[2], k, PH)};
  const RO ro{nullptr, a.offsets, nullptr, a.freqs};
  // (the count passed only tells whether this wave has observations)
  process_item<PH, 1, PK, SRC_LANES, 1, kFusedShare>(a, ro, item, make_curve_const(k, o.inv_alpha2, o.stat_scale), src,
                                                     n_all - wave * kWave, hist, lane, wave, part, nullptr, &f0);
}

void* fused_fn(int phase, int pk) {
  switch (phase) {
    case PH_FP64: return pk ? (void*)&fused_kernel<PH_FP64, 1> : (void*)&fused_kernel<PH_FP64, 0>;
    case PH_LISTING: return pk ? (void*)&fused_kernel<PH_LISTING, 1> : (void*)&fused_kernel<PH_LISTING, 0>;
    case PH_DF32: return pk ? (void*)&fused_kernel<PH_DF32, 1> : (void*)&fused_kernel<PH_DF32, 0>;
    default: return pk ? (void*)&fused_kernel<PH_FP32, 1> : (void*)&fused_kernel<PH_FP32, 0>;
  }
}

template <int PH, int FL, int PK, int SRC, int NV, int SH>
void* batched_ptr() {
  return (void*)&batched_kernel<PH, FL, PK, SRC, NV, SH>;
}

template <int PH, int FL, int SRC, int NV, int SH = 1>
void* batched_ptr_k(int pk) {
  return pk ? batched_ptr<PH, FL, 1, SRC, NV, SH>() : batched_ptr<PH, FL, 0, SRC, NV, SH>();
}

template <int PH, int SRC, int NV>
void* batched_ptr_sh(int pk, int share) {
  return share == 4 ? batched_ptr_k<PH, 1, SRC, NV, 4>(pk) : batched_ptr_k<PH, 1, SRC, NV, 2>(pk);
}

template <int PH>
void* batched_ptr_src(int fl, int pk, int src, int nv, int share) {
  if (share > 1) {
    if constexpr (PH == PH_DF32 || PH == PH_FP32) {  // study modes: one variant only
      if (fl != 1 || nv > 1) return nullptr;
      return src == SRC_DPP ? batched_ptr_sh<PH, SRC_DPP, 1>(pk, share) : batched_ptr_sh<PH, SRC_SCALAR, 1>(pk, share);
    } else {
      if (fl != 1) return nullptr;
      if (nv > 4) return src == SRC_DPP ? batched_ptr_sh<PH, SRC_DPP, kMaxVariants>(pk, share)
                                        : batched_ptr_sh<PH, SRC_SCALAR, kMaxVariants>(pk, share);
      if (nv > 1) return src == SRC_DPP ? batched_ptr_sh<PH, SRC_DPP, 4>(pk, share)
                                        : batched_ptr_sh<PH, SRC_SCALAR, 4>(pk, share);
      return src == SRC_DPP ? batched_ptr_sh<PH, SRC_DPP, 1>(pk, share) : batched_ptr_sh<PH, SRC_SCALAR, 1>(pk, share);
    }
  }
  if (nv > 4) return src == SRC_DPP ? batched_ptr_k<PH, 1, SRC_DPP, kMaxVariants>(pk)
                                    : batched_ptr_k<PH, 1, SRC_SCALAR, kMaxVariants>(pk);
  if (nv > 1) return src == SRC_DPP ? batched_ptr_k<PH, 1, SRC_DPP, 4>(pk) : batched_ptr_k<PH, 1, SRC_SCALAR, 4>(pk);
  if (src == SRC_DPP) return batched_ptr_k<PH, 1, SRC_DPP, 1>(pk);
  if (PH == PH_DF32 || PH == PH_FP32) return batched_ptr_k<PH, 1, SRC_SCALAR, 1>(pk);
  return fl == 2 ? batched_ptr_k<PH, 2, SRC_SCALAR, 1>(pk) : batched_ptr_k<PH, 1, SRC_SCALAR, 1>(pk);
}

// Instantiated shapes: two frequencies per lane exist for the FP64 folds with
// scalar point loads and one variant only; several variants take one
// frequency per lane, with room for 4 variants (for 2-4 of them) or 8 (the
// smaller instance holds fewer registers: measured 20 % faster with 2 or 3
// variants); shared histograms (2 or 4 waves) take one frequency per lane,
// and with the FP32-based folds one variant.  Null for a shape that is not
// built.
void* batched_fn(int phase, int fl, int pk, int src, int nv, int share) {
  switch (phase) {
    case PH_FP64: return batched_ptr_src<PH_FP64>(fl, pk, src, nv, share);
    case PH_LISTING: return batched_ptr_src<PH_LISTING>(fl, pk, src, nv, share);
    case PH_DF32: return batched_ptr_src<PH_DF32>(1, pk, src, nv, share);
    default: return batched_ptr_src<PH_FP32>(1, pk, src, nv, share);
  }
}

}  // namespace

int topk_capacity(int k) { return k <= 0 ? 0 : (k <= 8 ? 8 : 16); }

bool batched_shape_built(const Shape& shape, int phase, int n_var) {
  return batched_fn(phase, shape.freqs_per_lane, 0, shape.point_source, n_var, shape.share) != nullptr;
}

size_t batched_lds_bytes(const Shape& shape, int n_bins, int n_var) {
  const size_t hist = (size_t)(n_bins + 1) * kWave * sizeof(uint64_t);
  if (shape.share > 1) {
    size_t extra = (size_t)kSumParts * kWave * sizeof(float) + 16;
    if (n_var > 1) extra += (size_t)shape.share * kWave * sizeof(uint64_t);
    return hist + extra;
  }
  return (size_t)shape.waves_per_group * shape.freqs_per_lane * hist;
}

hipError_t batched_groups_per_cu(const Shape& shape, int phase, int topk, int n_var, size_t lds_bytes, int* out) {
  void* fn = batched_fn(phase, shape.freqs_per_lane, topk > 0, shape.point_source, n_var, shape.share);
  if (fn == nullptr) return hipErrorInvalidDeviceFunction;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, shape.waves_per_group * kWave, lds_bytes);
}

size_t fused_lds_bytes(int n_bins) {
  return (size_t)(n_bins + 1) * kWave * sizeof(uint64_t) + (size_t)kSumParts * kWave * sizeof(float);
}

int fused_waves() { return kFusedShare; }

hipError_t launch_fused(const BatchArgs& a, const FusedArgs& o, int phase, hipStream_t s) {
  void* fn = fused_fn(phase, a.topk > 0);
  const size_t lds_bytes = fused_lds_bytes(a.n_bins);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  BatchArgs args = a;
  FusedArgs fused = o;
  void* params[] = {&args, &fused};
  return hipLaunchKernel(fn, dim3((unsigned)a.n_items), dim3(kFusedShare * kWave), params, lds_bytes, s);
}

hipError_t launch_batched(const BatchArgs& a, const Shape& shape, int phase, int grid_groups, size_t lds_bytes,
                          hipStream_t s) {
  void* fn = batched_fn(phase, shape.freqs_per_lane, a.topk > 0, shape.point_source, a.var.n, shape.share);
  if (fn == nullptr) return hipErrorInvalidDeviceFunction;
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

size_t wide_lds_bytes(int n_bins, int share) {
  const size_t hist = (size_t)(n_bins + 1) * kWideSlotWords * sizeof(uint64_t);
  return share > 1 ? hist + (size_t)kSumParts * kWave * sizeof(double) + 16 : hist;
}

hipError_t wide_groups_per_cu(int phase, int topk, int n_bins, int share, int* out) {
  void* fn = wide_fn(phase, topk > 0, share);
  if (fn == nullptr) return hipErrorInvalidDeviceFunction;
  const size_t lds = wide_lds_bytes(n_bins, share);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, kWave * share, lds);
}

hipError_t launch_wide(const BatchArgs& a, int phase, int share, int grid_groups, hipStream_t s) {
  void* fn = wide_fn(phase, a.topk > 0, share);
  if (fn == nullptr) return hipErrorInvalidDeviceFunction;
  const size_t lds = wide_lds_bytes(a.n_bins, share);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  BatchArgs args = a;
  const WRec* recw = a.recw;
  const int64_t* offw = a.offw;
  const WideConst* wc = a.wc;
  const double* freqs = a.freqs;
  const Item* items = a.items;
  void* params[] = {&args, &recw, &offw, &wc, &freqs, &items};
  return hipLaunchKernel(fn, dim3(grid_groups), dim3(kWave * share), params, lds, s);
}

}  // namespace fpw
