// Counting stand-ins for the HIP runtime and for the library's kernel
// launchers, so that the library's host code runs on a machine without a GPU
// (under the host sanitizers).  Each launcher only counts the launch; the
// runtime keeps "device" memory in host memory.  fake_fail_after(n) makes the
// n-th following runtime call or launch fail, to drive the entry points'
// LNM_ERR_DEVICE paths.  Test infrastructure only.
#include <cstdio>
#include <cstring>

#include "internal.h"

static long g_launches = 0;
static long g_fail_after = -1;  // < 0: never

static hipError_t tick() {
  if (g_fail_after < 0) return hipSuccess;
  return g_fail_after-- == 0 ? hipErrorLaunchFailure : hipSuccess;
}

extern "C" long fake_launch_count() { return g_launches; }
extern "C" void fake_fail_after(long n) { g_fail_after = n; }

hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorNoDevice; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  p->multiProcessorCount = 256;
  std::snprintf(p->gcnArchName, sizeof p->gcnArchName, "gfx950:host-check");
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  const hipError_t e = tick();
  if (e == hipSuccess && n) std::memcpy(dst, src, n);
  return e;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  const hipError_t e = tick();
  if (e == hipSuccess && n) std::memset(dst, v, n);
  return e;
}
hipError_t hipStreamSynchronize(hipStream_t) { return tick(); }
static char g_event_tokens[65536 * 2 + 16];
static size_t g_next_event = 0;
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(&g_event_tokens[g_next_event++ % sizeof g_event_tokens]);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "fake device error"; }

namespace lnm {
#define LAUNCH(...)    \
  {                    \
    ++g_launches;      \
    return tick();     \
  }
hipError_t launch_relayout(const MarchDev&, float*, hipStream_t) LAUNCH()
hipError_t launch_march(const MarchDev&, const CamDev&, const MarchBuf&, float*, hipStream_t) LAUNCH()
hipError_t launch_reference(const MarchDev&, const CamDev&, int, float*, hipStream_t) LAUNCH()
hipError_t launch_splitk_reduce(const ConvArgs&, int, hipStream_t) LAUNCH()
hipError_t launch_conv3x3_f32(int, int, const ConvArgs&, hipStream_t, const HeadFuse*) LAUNCH()
hipError_t launch_conv3x3_bf16(int, const ConvArgs&, hipStream_t, const HeadFuse*) LAUNCH()
hipError_t launch_conv3x3_fp8(int, const ConvArgs&, hipStream_t, const HeadFuse*) LAUNCH()
hipError_t launch_amax(const float*, long, float*, float*, hipStream_t) LAUNCH()
hipError_t launch_head(const HeadArgs&, hipStream_t, const CompositeArgs*) LAUNCH()
hipError_t launch_composite(const CompositeArgs&, hipStream_t) LAUNCH()
hipError_t launch_composite_batch(const CompositeBatchArgs&, hipStream_t) LAUNCH()
hipError_t launch_adapters(int, const AdapterArgs&, int, hipStream_t) LAUNCH()
hipError_t launch_adapters_front(int, const AdapterArgs&, int, hipStream_t) LAUNCH()
hipError_t launch_adapters_train(int, const AdapterTrainArgs&, const float*, float*, float*, hipStream_t) LAUNCH()
hipError_t launch_fill_zero(float*, long, hipStream_t) LAUNCH()
hipError_t launch_shadow_map_sphere(int, float, float, float, float, float, float*, hipStream_t) LAUNCH()
hipError_t launch_composite_shadowed(const ShadowArgs&, hipStream_t) LAUNCH()
hipError_t launch_wgrad3x3(int, const WgradArgs&, int* n_partials, hipStream_t) {
  *n_partials = 4;
  ++g_launches;
  return tick();
}
hipError_t launch_wgrad_reduce(const float*, int, int, int, int, int, float*, hipStream_t) LAUNCH()
hipError_t launch_loss(const float*, const float*, float*, float*, long, float*, hipStream_t) LAUNCH()
hipError_t launch_colsum(const float*, long, int, float*, float*, hipStream_t) LAUNCH()
hipError_t launch_relu_mask(float*, const float*, long, hipStream_t) LAUNCH()
hipError_t launch_head_bwd(const float*, const float*, const float*, long, int, float*, float*, float*, float*,
                           hipStream_t) LAUNCH()
hipError_t launch_route_concat(const float*, int, int, int, int, int, float*, float*, hipStream_t) LAUNCH()
hipError_t launch_route_pool(const float*, const float*, int, int, int, int, float*, hipStream_t) LAUNCH()
hipError_t launch_adam(float*, const float*, float*, float*, long, float, float, float, float, int, hipStream_t) LAUNCH()
hipError_t launch_pack_f32(const float*, const float*, const LayerDesc&, int, char*, size_t, size_t, hipStream_t)
    LAUNCH()
}  // namespace lnm
