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
// shade_lights_lin takes the six values already decoded to linear.
__device__ __forceinline__ void shade_lights_lin(const float (*l)[3], const float (*rgb)[3], int k0, int k1,
                                                 const float* guide, float* rgba, size_t p, const float (&lin)[6]) {
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
__device__ __forceinline__ void shade_lights(const float (*l)[3], const float (*rgb)[3], int k0, int k1,
                                             const float* guide, float* rgba, size_t p, const float (&L)[6]) {
  float lin[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) lin[q] = srgb_decode(L[q]);
  shade_lights_lin(l, rgb, k0, k1, guide, rgba, p, lin);
}

__device__ __forceinline__ void shade_pixel(const CompositeArgs& a, int p, const float (&L)[6]) {
  shade_lights(a.l, a.rgb, 0, a.n_lights, a.guide, a.rgba, (size_t)p, L);
}

// Head epilogue of a conv layer (one 32-channel output tile): the tile's
// stored-precision activations are in sh[pixel][33] (pixels of the TH x 16
// tile in row order) and the head weights in shw[6][32] (zero past the
// layer's channels), after a barrier.  Two lanes finish each pixel, lane
// t < TH * 16 outputs 0..2 and lane t + TH * 16 outputs 3..5: the sums in
// channel order (as the separate head kernel forms them), the sigmoid, the
// lightmap store and, when asked, the decode to linear; the first lane then
// shades the pixel from the six linear values, exchanged through sh.  Every
// lane of the workgroup calls it (it has barriers).
template <int TH>
__device__ __forceinline__ void head_finish(const HeadFuse& hf, float* sh, const float* shw, int b, int H, int W,
                                            int y0, int x0) {
  constexpr int kTileW = 16, kPP = 33, NP = TH * kTileW;
  static_assert(2 * NP <= 256, "two lanes per pixel");
  const int t = threadIdx.x, tp = t % NP, half = t / NP;
  const bool act = t < 2 * NP;
  const int y = y0 + tp / kTileW, x = x0 + tp % kTileW;
  const bool ok = act && y < H && x < W;
  const size_t pix = (size_t)(b * H + y) * W + x;
  float lin[3];
  if (act) {
    const float* v = sh + tp * kPP;
    float z[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) z[j] = hf.b[3 * half + j];
    for (int c = 0; c < 32; c += 4) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float* w = shw + (3 * half + j) * 32 + c;
        z[j] += w[0] * v[c] + w[1] * v[c + 1] + w[2] * v[c + 2] + w[3] * v[c + 3];
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float L = 1.0f / (1.0f + expf(-z[j]));
      if (ok) hf.lm[pix * 6 + 3 * half + j] = L;
      lin[j] = srgb_decode(L);
    }
  }
  if (!hf.comp.rgba) return;
  __syncthreads();  // every lane is done reading the activations
  if (act) {
#pragma unroll
    for (int j = 0; j < 3; ++j) sh[tp * 8 + 3 * half + j] = lin[j];
  }
  __syncthreads();
  if (ok && half == 0) {
    float l6[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) l6[q] = sh[tp * 8 + q];
    shade_lights_lin(hf.comp.l, hf.comp.rgb, 0, hf.comp.n_lights, hf.comp.guide, hf.comp.rgba, pix, l6);
  }
}

// Head weights into LDS: shw[o][n] = w[o][n] for n < co, else 0.
__device__ __forceinline__ void head_weights(const HeadFuse& hf, int co, float* shw) {
  for (int q = threadIdx.x; q < 6 * 32; q += blockDim.x) shw[q] = (q % 32) < co ? hf.w[(q / 32) * co + q % 32] : 0.0f;
}

}  // namespace lnm
