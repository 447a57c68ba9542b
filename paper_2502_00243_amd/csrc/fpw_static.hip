// The evaluation pass that allocates nothing (fpw_eval_static): for callers
// that cannot call hipMalloc (code under HIP graph capture, serving loops,
// harnesses that forbid it).  Inputs and outputs are the caller's device
// buffers; everything else the pass needs — sanitised curve offsets, the
// prepared records, per-curve constants, work items, peak candidates and the
// queue counter — lives in one file-scope device array, `scratch`, of
// kStaticScratchBytes per GPU, held until the process ends.
//
// The pass is three launches of existing designs: a prepare kernel (one
// workgroup per curve: weights, centring, reference time, the wide-format
// records and constants, and the work items in natural order), the
// wide-format fold kernel (two 64-bit sums per bin: every curve within its
// bound of 1e-6, whatever the spread of its weights, so no host-side
// analysis of the data is needed), and the per-curve peak merge.  The fold
// takes the listing order (exact floor bins), which needs no plan-wide range
// of tau f.  Every access stays in bounds whatever the input values: curve
// ranges are clamped to [0, n_points].
#include "fpw_common.h"

#include <mutex>

namespace fpw {
namespace {

using namespace dev;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Device address of `scratch` per device (hipGetSymbolAddress once per
// device, with that device current; the array's name is only a host-side
// stand-in and must never be passed to a kernel).
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

hipError_t scratch_of_current_device(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return hipSuccess;
}

struct StaticPrepArgs {
  const int64_t* offsets;  // caller's [n_curves + 1], device
  const double* t;
  const double* y;
  const double* dy;
  int64_t n_curves, n_points;
  int center, tref_mode;
  double t_ref, inv_alpha2, stat_scale;
  int32_t n_freq, chunk, per_curve;  // items: per_curve chunks of `chunk` frequencies per curve
  int64_t* offs;           // [n_curves + 1] clamped curve starts (scratch)
  WRec* recw;              // [n_points] (scratch)
  WideConst* wc;           // [n_curves] (scratch)
  Item* items;             // [n_curves * per_curve] (scratch)
  int32_t* slot_k0;        // [n_items]
  int32_t* curve_slot;     // [n_curves + 1]
  uint32_t* queue;         // [1]
};

// One workgroup per curve (grid-strided): the curve's constants (the prepare
// kernel's own function), its wide records and constants, its items.  A
// curve whose weights exceed the wide format's bound (1e-6 on every bin; see
// fpw.h) gets a NaN scale, so its S is NaN and it has no peaks.
__global__ __launch_bounds__(kPrepThreads) void static_prepare_kernel(StaticPrepArgs a) {
  __shared__ double red[kPrepRed];
  const int th = threadIdx.x, lane = th & (kWave - 1), wave = th / kWave;
  if (blockIdx.x == 0 && th == 0) *a.queue = 0u;
  for (int64_t c = blockIdx.x; c < a.n_curves; c += gridDim.x) {
    const int64_t p0 = min(max(a.offsets[c], (int64_t)0), a.n_points);
    const int64_t p1 = min(max(a.offsets[c + 1], p0), a.n_points);
    const int n = (int)min(p1 - p0, (int64_t)(1 << 30));
    if (th == 0) {
      a.offs[c] = p0;
      if (c == a.n_curves - 1) a.offs[c + 1] = p1;
    }
    PrepConst k{};
    if (n > 0) k = curve_prep(a.t + p0, a.y + p0, a.dy + p0, n, a.center, a.tref_mode, a.t_ref, red);
    // the wide format's bound needs min w and sum(1/w) = sum(dy^2) beside sum(w)
    double wmin = INFINITY, h = 0.0;
    for (int i = th; i < n; i += kPrepThreads) {
      const double d = a.dy[p0 + i];
      wmin = fmin(wmin, 1.0 / (d * d));
      h += d * d;
    }
    wmin = wave_min_all(wmin);
    h = wave_sum_all(h);
    __syncthreads();  // curve_prep's readers of red are done
    if (lane == 0) {
      red[wave] = wmin;
      red[kPrepWaves + wave] = h;
    }
    __syncthreads();
    wmin = red[0];
    h = red[kPrepWaves];
#pragma unroll
    for (int w = 1; w < kPrepWaves; ++w) {
      wmin = fmin(wmin, red[w]);
      h += red[kPrepWaves + w];
    }
    __syncthreads();  // red is free for the next curve
    for (int i = th; i < n; i += kPrepThreads) {
      const int64_t p = p0 + i;
      a.recw[p] = make_wrec(a.t[p], a.y[p], a.dy[p], k, PH_LISTING);
    }
    if (th == 0) {
      WideConst wc = make_wide_const(k, a.inv_alpha2, a.stat_scale);
      const double e_w = k.sw / (2.0 * kWideScaleW * wmin);
      const double e_y = sqrt(h * k.sw) / (2.0 * kWideScaleY);
      if (n > 0 && !(fmax(e_w, 0x1p-53) <= 1e-6 && e_y <= 1e-6)) wc.scale = NAN;
      a.wc[c] = wc;
    }
    // items of this curve, natural order; a trailing chunk of one frequency
    // joins its predecessor (every chunk of a multi-frequency grid keeps two
    // frequencies for the cross-chunk peak test)
    for (int j = th; j < a.per_curve; j += kPrepThreads) {
      const int32_t k0 = j * a.chunk;
      int32_t k1 = min(k0 + a.chunk, a.n_freq);
      if (j == a.per_curve - 1) k1 = a.n_freq;
      const int64_t i = c * a.per_curve + j;
      Item it;
      it.curve = (int32_t)c;
      it.k0 = k0;
      it.k1 = k1;
      it.slot = (int32_t)i;
      a.items[i] = it;
      a.slot_k0[i] = k0;
    }
    if (th == 0) {
      a.curve_slot[c] = (int32_t)(c * a.per_curve);
      if (c == a.n_curves - 1) a.curve_slot[c + 1] = (int32_t)((c + 1) * a.per_curve);
    }
  }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// Scratch layout of one call, in bytes from the array's start; false when it
// does not fit.
bool static_layout(int64_t n_curves, int64_t n_points, int64_t n_items, int topk, StaticLayout* l) {
  size_t o = 0;
  l->offs = o;
  o = align256(o + (size_t)(n_curves + 1) * sizeof(int64_t));
  l->recw = o;
  o = align256(o + (size_t)n_points * sizeof(WRec));
  l->wc = o;
  o = align256(o + (size_t)n_curves * sizeof(WideConst));
  l->items = o;
  o = align256(o + (size_t)n_items * sizeof(Item));
  l->slot_k0 = o;
  o = align256(o + (size_t)n_items * sizeof(int32_t));
  l->curve_slot = o;
  o = align256(o + (size_t)(n_curves + 1) * sizeof(int32_t));
  l->cand_val = o;
  o = align256(o + (size_t)n_items * (size_t)topk * sizeof(float));
  l->cand_idx = o;
  o = align256(o + (size_t)n_items * (size_t)topk * sizeof(int32_t));
  l->edge = o;
  o = align256(o + (size_t)n_items * 4 * sizeof(float));
  l->queue = o;
  o = align256(o + sizeof(uint32_t));
  l->total = o;
  return o <= kStaticScratchBytes;
}

hipError_t launch_static_pass(const StaticPass& s, hipStream_t st) {
  unsigned char* base = nullptr;
  hipError_t e = scratch_of_current_device(&base);
  if (e != hipSuccess) return e;
  StaticLayout l;
  if (!static_layout(s.n_curves, s.n_points, s.n_items, s.topk, &l)) return hipErrorInvalidValue;
  StaticPrepArgs p{};
  p.offsets = s.offsets;
  p.t = s.t;
  p.y = s.y;
  p.dy = s.dy;
  p.n_curves = s.n_curves;
  p.n_points = s.n_points;
  p.center = s.center;
  p.tref_mode = s.tref_mode;
  p.t_ref = s.t_ref;
  p.inv_alpha2 = s.inv_alpha2;
  p.stat_scale = s.stat_scale;
  p.n_freq = s.n_freq;
  p.chunk = s.chunk;
  p.per_curve = s.per_curve;
  p.offs = reinterpret_cast<int64_t*>(base + l.offs);
  p.recw = reinterpret_cast<WRec*>(base + l.recw);
  p.wc = reinterpret_cast<WideConst*>(base + l.wc);
  p.items = reinterpret_cast<Item*>(base + l.items);
  p.slot_k0 = reinterpret_cast<int32_t*>(base + l.slot_k0);
  p.curve_slot = reinterpret_cast<int32_t*>(base + l.curve_slot);
  p.queue = reinterpret_cast<uint32_t*>(base + l.queue);
  const int64_t g = s.n_curves < 65536 ? s.n_curves : 65536;
  hipLaunchKernelGGL(static_prepare_kernel, dim3((unsigned)g), dim3(kPrepThreads), 0, st, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchArgs a{};
  a.freqs = s.freqs;
  a.items = p.items;
  a.n_items = (int32_t)s.n_items;
  a.n_freq = s.n_freq;
  a.n_bins = s.n_bins;
  a.topk = s.topk;
  a.n_curves = (int32_t)s.n_curves;
  a.var.n = 1;
  a.var.k[0] = 1;
  a.fold_nh = 0.0;
  a.S = s.S;
  a.cand_val = reinterpret_cast<float*>(base + l.cand_val);
  a.cand_idx = reinterpret_cast<int32_t*>(base + l.cand_idx);
  a.edge = reinterpret_cast<float*>(base + l.edge);
  a.queue = p.queue;
  a.recw = p.recw;
  a.offw = p.offs;
  a.wc = p.wc;
  e = launch_wide(a, PH_LISTING, s.share, s.grid, st);
  if (e != hipSuccess || s.topk <= 0) return e;
  MergeArgs m{};
  m.cand_val = a.cand_val;
  m.cand_idx = a.cand_idx;
  m.edge = a.edge;
  m.slot_k0 = p.slot_k0;
  m.curve_slot = p.curve_slot;
  m.n_curves = (int32_t)s.n_curves;
  m.n_freq = s.n_freq;
  m.topk = s.topk;
  m.n_var = 1;
  m.out_idx = s.idx;
  m.out_val = s.val;
  return launch_merge(m, st);
}

}  // namespace fpw
