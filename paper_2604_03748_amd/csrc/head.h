// Six-way shading of a pixel and the 1x1 head finished from LDS, shared by
// the shading kernels and the conv kernels that apply the head in their last
// layer's epilogue (device code only).
#pragma once
#include "internal.h"

namespace lnm {

__device__ __forceinline__ float srgb_decode(float s) {
  return s <= 0.04045f ? s / 12.92f : powf((s + 0.055f) / 1.055f, 2.4f);
}

// Six-way shading of one pixel from its six lightmap values with lights
// [k0, k1) of the tables l (camera frame) and rgb:
// rgb = sum_l c_l sum_p |l_p| lin(L_p^{sign l_p}), alpha = 1 - T.
__device__ __forceinline__ void shade_lights(const float (*l)[3], const float (*rgb)[3], int k0, int k1,
                                             const float* guide, float* rgba, size_t p, const float (&L)[6]) {
  float lin[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) lin[q] = srgb_decode(L[q]);
  float r = 0.f, gg = 0.f, bb = 0.f;
  for (int k = k0; k < k1; ++k) {
    float s = 0.f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float c = l[k][ax];
      s += fabsf(c) * (c >= 0.0f ? lin[2 * ax] : lin[2 * ax + 1]);
    }
    r += rgb[k][0] * s;
    gg += rgb[k][1] * s;
    bb += rgb[k][2] * s;
  }
  float* o = rgba + p * 4;
  o[0] = r;
  o[1] = gg;
  o[2] = bb;
  o[3] = 1.0f - guide[p * 3 + 1];
}

__device__ __forceinline__ void shade_pixel(const CompositeArgs& a, int p, const float (&L)[6]) {
  shade_lights(a.l, a.rgb, 0, a.n_lights, a.guide, a.rgba, (size_t)p, L);
}

// Head epilogue of a conv layer (one 32-channel output tile): the tile's
// stored-precision activations are in sh[pixel][33] (pixels of the TH x 16
// tile in row order) and the head weights in shw[6][32] (zero past the
// layer's channels), after a barrier.  Thread t < TH * 16 finishes pixel t:
// the six sums in channel order (as the separate head kernel forms them),
// the sigmoid, the lightmap store and, when asked, the shading.
template <int TH>
__device__ __forceinline__ void head_finish(const HeadFuse& hf, const float* sh, const float* shw, int b, int H,
                                            int W, int y0, int x0) {
  constexpr int kTileW = 16, kPP = 33;
  const int t = threadIdx.x;
  if (t >= TH * kTileW) return;
  const int y = y0 + t / kTileW, x = x0 + t % kTileW;
  if (y >= H || x >= W) return;
  const float* v = sh + t * kPP;
  float z[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) z[o] = hf.b[o];
  for (int c = 0; c < 32; c += 4) {
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      const float* w = shw + o * 32 + c;
      z[o] += w[0] * v[c] + w[1] * v[c + 1] + w[2] * v[c + 2] + w[3] * v[c + 3];
    }
  }
  const size_t pix = (size_t)(b * H + y) * W + x;
  float L[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    L[o] = 1.0f / (1.0f + expf(-z[o]));
    hf.lm[pix * 6 + o] = L[o];
  }
  if (hf.comp.rgba) shade_pixel(hf.comp, (int)pix, L);
}

// Head weights into LDS: shw[o][n] = w[o][n] for n < co, else 0.
__device__ __forceinline__ void head_weights(const HeadFuse& hf, int co, float* shw) {
  for (int q = threadIdx.x; q < 6 * 32; q += blockDim.x) shw[q] = (q % 32) < co ? hf.w[(q / 32) * co + q % 32] : 0.0f;
}

}  // namespace lnm
