// Depth-based screen-space obstacle shadowing (Section 4.5).
//
// A directional light gets an orthographic light space (e1, e2, l) around a
// shared origin; its shadow map holds, per texel, the light-space depth of
// the obstacle surface nearest the light.  The shading pass projects each
// pixel's smoke surface point P = o + D d (D from the guiding map) into that
// space and multiplies the light's six-way term by 0 when the texel's
// occluder is closer to the light than P (beyond a bias), else by 1.
//
// Both kernels are one lane per output element and HBM/launch bound: the
// shading pass reads 36 bytes and writes 16 per pixel (plus one 4-byte
// shadow-map texel per shadowed light, which stays in L2 for maps up to a
// few MB).
#include <cmath>

#include "head.h"
#include "internal.h"
#include "ray.h"

namespace lnm {
namespace {

__global__ __launch_bounds__(256) void shadow_map_sphere_kernel(int S, float E, float cu, float cv, float cz, float r2,
                                                                float* __restrict__ depth) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= S * S) return;
  const int i = t % S, j = t / S;
  const float u = -E + 2.0f * E * ((float)i + 0.5f) / (float)S;
  const float v = -E + 2.0f * E * ((float)j + 0.5f) / (float)S;
  const float du = u - cu, dv = v - cv;
  const float q = r2 - du * du - dv * dv;
  depth[t] = q >= 0.0f ? cz + sqrtf(q) : -INFINITY;
}

__global__ __launch_bounds__(256) void composite_shadowed_kernel(ShadowArgs a) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= a.c.P) return;
  const int q = p % (a.cam.W * a.cam.H);
  const int i = q % a.cam.W, j = q / a.cam.W;
  const float* L = a.c.lm + (size_t)p * 6;
  float lin[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) lin[k] = srgb_decode(L[k]);
  const float D = a.c.guide[(size_t)p * 3 + 2];
  V3 rel = v3(0.0f, 0.0f, 0.0f);
  if (D > 0.0f) {
    V3 o, d;
    camera_ray(a.cam, i, j, &o, &d);
    rel = v3(o.x + D * d.x - a.origin[0], o.y + D * d.y - a.origin[1], o.z + D * d.z - a.origin[2]);
  }
  const float scale = (float)a.S / (2.0f * a.E);
  float r = 0.f, g = 0.f, b = 0.f;
  for (int k = 0; k < a.c.n_lights; ++k) {
    float vis = 1.0f;
    if (D > 0.0f && a.depth[k] != nullptr) {
      const float u = dot3(rel, v3(a.e1[k][0], a.e1[k][1], a.e1[k][2]));
      const float w = dot3(rel, v3(a.e2[k][0], a.e2[k][1], a.e2[k][2]));
      const float z = dot3(rel, v3(a.lw[k][0], a.lw[k][1], a.lw[k][2]));
      const float fu = floorf((u + a.E) * scale), fw = floorf((w + a.E) * scale);
      if (fu >= 0.0f && fu < (float)a.S && fw >= 0.0f && fw < (float)a.S &&
          a.depth[k][(size_t)fw * a.S + (int)fu] > z + a.bias)
        vis = 0.0f;
    }
    if (a.vis) a.vis[(size_t)k * a.c.P + p] = vis;
    float s = 0.f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float c = a.c.l[k][ax];
      s += fabsf(c) * (c >= 0.0f ? lin[2 * ax] : lin[2 * ax + 1]);
    }
    s *= vis;  // same arithmetic as the unshadowed shading when vis = 1
    r += a.c.rgb[k][0] * s;
    g += a.c.rgb[k][1] * s;
    b += a.c.rgb[k][2] * s;
  }
  float* o = a.c.rgba + (size_t)p * 4;
  o[0] = r;
  o[1] = g;
  o[2] = b;
  o[3] = 1.0f - a.c.guide[(size_t)p * 3 + 1];
}

}  // namespace

hipError_t launch_shadow_map_sphere(int S, float E, float cu, float cv, float cz, float r2, float* depth,
                                    hipStream_t s) {
  const long n = (long)S * S;
  hipLaunchKernelGGL(shadow_map_sphere_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, E, cu, cv, cz,
                     r2, depth);
  return hipGetLastError();
}

hipError_t launch_composite_shadowed(const ShadowArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(composite_shadowed_kernel, dim3((a.c.P + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lnm
