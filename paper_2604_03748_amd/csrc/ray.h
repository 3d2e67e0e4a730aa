// Small fp32 vector helpers and the camera ray of a pixel, shared by the
// march and the shading kernels (device code only).
#pragma once
#include "internal.h"

namespace lnm {

struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 scale3(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ V3 normalize3(V3 a) { return scale3(a, 1.0f / sqrtf(dot3(a, a))); }

// Ray through the centre of pixel (i, j): pinhole (origin at the eye) or
// orthographic (parallel rays along f from the image plane through the eye).
__device__ __forceinline__ void camera_ray(const CamDev& c, int i, int j, V3* o, V3* d) {
  const float sx = 2.0f * ((float)i + 0.5f) / (float)c.W - 1.0f;
  const float sy = 1.0f - 2.0f * ((float)j + 0.5f) / (float)c.H;
  const V3 f = v3(c.f[0], c.f[1], c.f[2]), r = v3(c.r[0], c.r[1], c.r[2]), u = v3(c.u[0], c.u[1], c.u[2]);
  const float a = sx * c.aspect;
  if (c.proj == LNM_PERSPECTIVE) {
    *o = v3(c.eye[0], c.eye[1], c.eye[2]);
    *d = normalize3(v3(f.x + c.tan_half * (a * r.x + sy * u.x), f.y + c.tan_half * (a * r.y + sy * u.y),
                       f.z + c.tan_half * (a * r.z + sy * u.z)));
  } else {
    const float e = c.half_extent;
    *o = v3(c.eye[0] + e * (a * r.x + sy * u.x), c.eye[1] + e * (a * r.y + sy * u.y),
            c.eye[2] + e * (a * r.z + sy * u.z));
    *d = f;
  }
}

}  // namespace lnm
