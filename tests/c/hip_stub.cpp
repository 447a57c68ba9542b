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

extern "C" {
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) { *p = std::malloc(n ? n : 1); return hipSuccess; }
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { std::memset(p, v, n); return hipSuccess; }
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
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)std::malloc(8); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)std::malloc(8); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { std::free(s); return hipSuccess; }
}

namespace fpw {
hipError_t launch_prepare(const PrepArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_batched(const BatchArgs&, const Shape&, int, int, size_t, hipStream_t) { return hipSuccess; }
hipError_t launch_merge(const MergeArgs&, hipStream_t, bool) { return hipSuccess; }
hipError_t launch_fused(const BatchArgs& a, const FusedArgs& o, int, hipStream_t) {
  // one workgroup per item
  if (a.n_items < 1 || a.items == nullptr || o.t == nullptr) return hipErrorInvalidValue;
  return hipSuccess;
}
size_t fused_lds_bytes(int n_bins) { return (size_t)(n_bins + 1) * 512 + 1024; }
int fused_waves() { return 4; }
hipError_t launch_topk(const TopkArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_fp64(const Fp64Args&, hipStream_t) { return hipSuccess; }
hipError_t launch_bins(const BinsArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_entropy(const EntropyArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_prepare_shared(const SharedPrepArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_shared(const SharedArgs&, int, int, int, int, int, size_t, hipStream_t) { return hipSuccess; }
void shared_shape(int, int* nb, int* fw) { *nb = 2; *fw = 8; }
hipError_t launch_bm_prepare(const BmPrepArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_bm(const BmArgs&, int, int, hipStream_t) { return hipSuccess; }
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
