// lnm_frame_static: the whole frame (lnm_frame) on a workspace the library
// owns, for callers that cannot allocate device memory.
//
// The workspace is one file-scope device array, so every device the library
// runs on holds its own copy of it (LNM_STATIC_SCRATCH_BYTES) from the moment
// the code object is loaded there until the process ends.  Host code never
// passes the array's name to a kernel: in host code that name stands for a
// host-side symbol, not a device address.  lnm_ctx_create looks up the
// device address once per context, with the context's device current, and
// every launch uses that address.
#include "internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[LNM_STATIC_SCRATCH_BYTES];

}  // namespace

namespace lnm {

hipError_t static_scratch_address(void** out) {
  *out = nullptr;
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

}  // namespace lnm

using namespace lnm;

extern "C" lnm_status lnm_frame_static(lnm_ctx ctx, lnm_net net, const lnm_volume* vol, const lnm_camera* cam,
                                       const lnm_march_params* prm, const lnm_light* lights, int32_t n_lights,
                                       float* guide, float* lightmaps, float* rgba, void* stream) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (!ctx->static_scratch) return fail(LNM_ERR_DEVICE, "the context has no static workspace");
  const size_t need = frame_workspace_bytes(net, vol, cam, prm);
  if (need > (size_t)LNM_STATIC_SCRATCH_BYTES)
    return fail(LNM_ERR_SHAPE, "frame needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                   std::to_string((size_t)LNM_STATIC_SCRATCH_BYTES) +
                                   " of the static workspace; use lnm_frame with a workspace of that size");
  // need == 0 means invalid arguments: frame_impl reports which
  return frame_impl(ctx, net, vol, cam, prm, lights, n_lights, guide, lightmaps, rgba, ctx->static_scratch,
                    (size_t)LNM_STATIC_SCRATCH_BYTES, stream);
}
