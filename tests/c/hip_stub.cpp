// CPU stand-ins for the HIP runtime calls and the device launchers that the
// host runtime (fpw_host.cpp) uses: device memory is host memory, copies are
// memcpy, kernel launches and graph replays do nothing.  Linked with the host
// runtime and host_driver.cpp, it lets the plan / pass / shape logic run on
// the CPU under AddressSanitizer and UndefinedBehaviorSanitizer.  The sizes
// returned by the LDS and occupancy stand-ins only need to be plausible.
#include <hip/hip_runtime_api.h>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include "fpw_internal.h"

// Failure injection: after stub_fail(kind, n) the n-th call of that kind
// (counted from then on) fails, so that the host runtime's error paths run:
// kind 1 hipMalloc (out of memory), 2 hipMemcpy / hipMemcpyAsync /
// hipMemsetAsync, 3 any kernel launcher, 4 hipStreamBeginCapture; kind 0
// turns it off.  stub_failed() tells whether it has fired.
namespace {
int g_kind = 0;
long g_at = 0, g_seen = 0;
bool g_fired = false;
bool fail_now(int kind) {
  if (g_kind != kind || g_fired) return false;
  if (++g_seen != g_at) return false;
  g_fired = true;
  return true;
}
}  // namespace

extern "C" {
void stub_fail(int kind, long nth) {
  g_kind = kind;
  g_at = nth;
  g_seen = 0;
  g_fired = false;
}
int stub_failed(void) { return g_fired ? 1 : 0; }

hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) {
  if (fail_now(1)) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  *p = std::malloc(n ? n : 1);
  return hipSuccess;
}
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (fail_now(2)) return hipErrorInvalidValue;
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  if (fail_now(2)) return hipErrorInvalidValue;
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) {
  if (fail_now(2)) return hipErrorInvalidValue;
  std::memset(p, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)std::malloc(8); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { std::free(e); return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.f; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_t* p, int) { std::memset(p, 0, sizeof(*p)); std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-"); return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { std::free(g); return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t g) { std::free(g); return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) { *e = (hipGraphExec_t)std::malloc(8); return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return fail_now(4) ? hipErrorInvalidValue : hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)std::malloc(8); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)std::malloc(8); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { std::free(s); return hipSuccess; }
}

namespace fpw {
hipError_t launch_prepare(const PrepArgs&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_batched(const BatchArgs&, const Shape&, int, int, size_t, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_merge(const MergeArgs&, hipStream_t, bool) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_fused(const BatchArgs& a, const FusedArgs& o, int, hipStream_t) {
  // one workgroup per item
  if (a.n_items < 1 || a.items == nullptr || o.t == nullptr) return hipErrorInvalidValue;
  return fail_now(3) ? hipErrorLaunchFailure : hipSuccess;
}
hipError_t launch_wide(const BatchArgs& a, int phase, int share, int grid, hipStream_t) {
  // only wide items, built for the FP64 folds, shares 1/2/4, a grid the items fill
  if (a.n_items < 1 || a.items == nullptr || a.recw == nullptr || a.offw == nullptr || a.wc == nullptr ||
      a.queue == nullptr || phase > 1 || !(share == 1 || share == 2 || share == 4) || grid < 1 || grid > a.n_items)
    return hipErrorInvalidValue;
  return fail_now(3) ? hipErrorLaunchFailure : hipSuccess;
}
size_t wide_lds_bytes(int n_bins, int share) { return (size_t)(n_bins + 1) * 1024 + (share > 1 ? 2064 : 0); }
hipError_t wide_groups_per_cu(int, int, int, int, int* out) { *out = 2; return hipSuccess; }
bool static_layout(int64_t n_curves, int64_t n_points, int64_t n_items, int topk, StaticLayout* l) {
  *l = StaticLayout{};
  l->total = (size_t)(32 * n_points + 44 * n_curves + (36 + 8 * topk) * n_items + 2560);
  return l->total <= kStaticScratchBytes;
}
hipError_t launch_static_pass(const StaticPass& s, hipStream_t) {
  // sizes and outputs as the entry point promises; the layout fits
  StaticLayout l;
  if (s.n_items < 1 || s.n_curves < 1 || s.n_points < s.n_curves || s.chunk < 64 || s.chunk % 64 != 0 ||
      s.per_curve < 1 || s.n_items != s.per_curve * s.n_curves || (int64_t)(s.per_curve - 1) * s.chunk >= s.n_freq ||
      s.grid < 1 || s.grid > s.n_items || (s.topk > 0) != (s.idx != nullptr) || (s.S == nullptr && s.idx == nullptr) ||
      !static_layout(s.n_curves, s.n_points, s.n_items, s.topk, &l))
    return hipErrorInvalidValue;
  return fail_now(3) ? hipErrorLaunchFailure : hipSuccess;
}
size_t fused_lds_bytes(int n_bins) { return (size_t)(n_bins + 1) * 512 + 1024; }
int fused_waves() { return 4; }
hipError_t launch_topk(const TopkArgs&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_fp64(const Fp64Args&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_bins(const BinsArgs&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_entropy(const EntropyArgs&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_prepare_shared(const SharedPrepArgs&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_shared(const SharedArgs&, int, int, int, int, int, size_t, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
void shared_shape(int, int* nb, int* fw) { *nb = 2; *fw = 8; }
hipError_t launch_bm_prepare(const BmPrepArgs&, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t launch_bm(const BmArgs&, int, int, hipStream_t) { return fail_now(3) ? hipErrorLaunchFailure : hipSuccess; }
hipError_t bm_groups_per_cu(int, int, int, int, int, int* out) { *out = 4; return hipSuccess; }
size_t bm_lds_bytes(int n_bins, int n_terms, int share) {
  const size_t per_slot = n_terms >= 3 ? 16 : (n_terms == 2 ? 12 : 8);
  const size_t hist = per_slot * (n_bins + 1) * 64;
  return share <= 1 ? hist : hist + (size_t)(share - 1) * 10 * 64 * 8 + 16;
}
int topk_capacity(int k) { return k <= 0 ? 0 : (k <= 8 ? 8 : 16); }
bool batched_shape_built(const Shape&, int, int) { return true; }
size_t batched_lds_bytes(const Shape& s, int n_bins, int) { return (size_t)s.waves_per_group * (n_bins + 1) * 512; }
hipError_t batched_groups_per_cu(const Shape&, int, int, int, size_t, int* out) { *out = 4; return hipSuccess; }
}  // namespace fpw
