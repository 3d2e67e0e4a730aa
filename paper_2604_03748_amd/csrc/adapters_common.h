// Device helpers shared by the channel adapters' inference and training
// kernels (Section 4.3: four NAFBlocks on the decoder output, one per output
// group).  See adapters.hip for the operand layout of the 1x1 convolutions
// on the matrix cores.
#pragma once

#include "internal.h"

namespace lnm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// offsets of one adapter's tensors (parameter-file order) for width C
template <int C>
struct Off {
  static constexpr int ln1w = 0, ln1b = C, c1w = 2 * C, c1b = c1w + 2 * C * C, dww = c1b + 2 * C, dwb = dww + 18 * C,
                       scaw = dwb + 2 * C, scab = scaw + C * C, c3w = scab + C, c3b = c3w + C * C, beta = c3b + C,
                       ln2w = beta + C, ln2b = ln2w + C, c4w = ln2b + C, c4b = c4w + 2 * C * C, c5w = c4b + 2 * C,
                       c5b = c5w + C * C, gamma = c5b + C, hw = gamma + C, hb = hw + 2 * C, total = hb + 2;
};

__device__ __forceinline__ float bf16f(uint32_t h) { return __uint_as_float(h << 16); }

// four floats from global memory (a group's parameters start 4-byte aligned)
__device__ __forceinline__ f4 ld4(const float* p) { return f4{p[0], p[1], p[2], p[3]}; }

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// sum over the four lanes holding one pixel's channels (every lane of the
// four gets the same value: the two additions are commutative pairings)
__device__ __forceinline__ float pixel_sum(float s) {
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

__device__ __forceinline__ float hsum(f4 v) { return (v.x + v.y) + (v.z + v.w); }

// channels c0 .. c0 + 3 of feature pixel p as fp32 (IN: 0 fp32, 1 bf16,
// 2 e4m3 x scale); c0 is a multiple of 4
template <int C, int IN>
__device__ __forceinline__ f4 feat4(const AdapterArgs& a, size_t p, int c0) {
  if constexpr (IN == 0) {
    return *reinterpret_cast<const f4*>(static_cast<const float*>(a.feat) + p * C + c0);
  } else if constexpr (IN == 1) {
    const uint2 q = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.feat) + p * C + c0);
    return f4{bf16f(q.x & 0xffffu), bf16f(q.x >> 16), bf16f(q.y & 0xffffu), bf16f(q.y >> 16)};
  } else {
    const int q = *reinterpret_cast<const int*>(static_cast<const uint8_t*>(a.feat) + p * C + c0);
    return f4{__builtin_amdgcn_cvt_f32_fp8(q, 0), __builtin_amdgcn_cvt_f32_fp8(q, 1),
              __builtin_amdgcn_cvt_f32_fp8(q, 2), __builtin_amdgcn_cvt_f32_fp8(q, 3)} *
           a.feat_scale;
  }
}

// front tile: kAdaptTileY x kAdaptTileX (8 x 32) interior pixels and a
// one-pixel halo around them (10 x 34 = 340 pixels, 22 MFMA column blocks of
// 16), 32 conv1 channels per pass in LDS at 36 floats per halo pixel (the
// pad keeps the 16-byte accesses of neighbouring pixels on distinct banks)
constexpr int kTY = kAdaptTileY, kTX = kAdaptTileX;
constexpr int kHX = kTX + 2, kHalo = (kTY + 2) * kHX;
constexpr int kHaloCols = (kHalo + 15) / 16;
constexpr int kUPitch = 36;
static_assert(kTY == 8 && kTX == 32, "the depthwise stages map 256 threads onto 8 x 32 pixels x 4 channel quads");

// Layer norm 1 and the conv1 rows {16 j + i, C + 16 j + i} (i < 16) of the
// front tile's halo pixels into us[halo pixel][32] (zero outside the image,
// where the depthwise conv pads with zeros).  Wavefront w takes column
// blocks w, w + 4, ...  With n1 set (training), the layer norm's output of
// the tile's interior pixels also goes to n1[pixel][C].
template <int C, int IN>
__device__ __forceinline__ void front_conv1(const AdapterArgs& a, const float* P, size_t img, int y0, int x0, int j,
                                            const f4 (&lw)[C / 16], const f4 (&lb)[C / 16], float* us, float* n1) {
  using O = Off<C>;
  constexpr int KB = C / 16;
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4, wave = threadIdx.x >> 6;
  f4 wa[2][KB];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) wa[m][kb] = ld4(P + O::c1w + (size_t)(m * C + 16 * j + li) * C + 16 * kb + 4 * G);
  const f4 bias0 = ld4(P + O::c1b + 16 * j + 4 * G), bias1 = ld4(P + O::c1b + C + 16 * j + 4 * G);
#pragma unroll 1
  for (int nb = wave; nb < kHaloCols; nb += 4) {  // uniform per wavefront: the MFMAs see every lane
    const int hp = nb * 16 + li;
    const int hy = hp / kHX, hx = hp - hy * kHX;
    const int y = y0 + hy - 1, x = x0 + hx - 1;
    const bool in = hp < kHalo && y >= 0 && y < a.H && x >= 0 && x < a.W;
    const size_t p = img + (size_t)min(max(y, 0), a.H - 1) * a.W + min(max(x, 0), a.W - 1);
    f4 xv[KB];
    float s = 0.0f;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      xv[kb] = feat4<C, IN>(a, p, 16 * kb + 4 * G);
      s += hsum(xv[kb]);
    }
    const float mu = pixel_sum(s) * (1.0f / (float)C);
    float sq = 0.0f;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      xv[kb] -= mu;
      sq += hsum(xv[kb] * xv[kb]);
    }
    const float rs = 1.0f / sqrtf(pixel_sum(sq) * (1.0f / (float)C) + 1e-6f);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) xv[kb] = xv[kb] * rs * lw[kb] + lb[kb];
    if (n1 && in && hy >= 1 && hy <= kTY && hx >= 1 && hx <= kTX) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) *reinterpret_cast<f4*>(n1 + p * C + 16 * kb + 4 * G) = xv[kb];
    }
    f4 acc0 = bias0, acc1 = bias1;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc0 = mfma(wa[0][kb][r], xv[kb][r], acc0);
        acc1 = mfma(wa[1][kb][r], xv[kb][r], acc1);
      }
    const f4 zero = f4{0.0f, 0.0f, 0.0f, 0.0f};
    float* dst = us + hp * kUPitch + 4 * G;
    *reinterpret_cast<f4*>(dst) = in ? acc0 : zero;
    *reinterpret_cast<f4*>(dst + 16) = in ? acc1 : zero;
  }
}

// The conv1 operands of a wavefront's halo column blocks (w, w + 4, ...: at
// most kHaloUnits of them), layer norm 1 applied, kept in registers across
// the channel passes (the norm is the same for every pass), with each
// column's in-image flag.
constexpr int kHaloUnits = (kHaloCols + 3) / 4;
template <int C>
struct FrontOperands {
  f4 xv[kHaloUnits][C / 16];
  bool in[kHaloUnits];
};

template <int C, int IN>
__device__ __forceinline__ void front_operands(const AdapterArgs& a, size_t img, int y0, int x0,
                                               const f4 (&lw)[C / 16], const f4 (&lb)[C / 16], FrontOperands<C>& fo) {
  constexpr int KB = C / 16;
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4, wave = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < kHaloUnits; ++u) {
    const int hp = (wave + 4 * u) * 16 + li;
    const int hy = hp / kHX, hx = hp - hy * kHX;
    const int y = y0 + hy - 1, x = x0 + hx - 1;
    fo.in[u] = hp < kHalo && y >= 0 && y < a.H && x >= 0 && x < a.W;
    const size_t p = img + (size_t)min(max(y, 0), a.H - 1) * a.W + min(max(x, 0), a.W - 1);
    float s = 0.0f;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      fo.xv[u][kb] = feat4<C, IN>(a, p, 16 * kb + 4 * G);
      s += hsum(fo.xv[u][kb]);
    }
    const float mu = pixel_sum(s) * (1.0f / (float)C);
    float sq = 0.0f;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      fo.xv[u][kb] -= mu;
      sq += hsum(fo.xv[u][kb] * fo.xv[u][kb]);
    }
    const float rs = 1.0f / sqrtf(pixel_sum(sq) * (1.0f / (float)C) + 1e-6f);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) fo.xv[u][kb] = fo.xv[u][kb] * rs * lw[kb] + lb[kb];
  }
}

// front_conv1 on operands from front_operands: the same products in the
// same order, without recomputing the norm
template <int C>
__device__ __forceinline__ void front_conv1_cached(const float* P, int j, const FrontOperands<C>& fo, float* us) {
  using O = Off<C>;
  constexpr int KB = C / 16;
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4, wave = threadIdx.x >> 6;
  f4 wa[2][KB];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) wa[m][kb] = ld4(P + O::c1w + (size_t)(m * C + 16 * j + li) * C + 16 * kb + 4 * G);
  const f4 bias0 = ld4(P + O::c1b + 16 * j + 4 * G), bias1 = ld4(P + O::c1b + C + 16 * j + 4 * G);
#pragma unroll
  for (int u = 0; u < kHaloUnits; ++u) {
    const int nb = wave + 4 * u;
    if (nb >= kHaloCols) break;  // uniform per wavefront
    f4 acc0 = bias0, acc1 = bias1;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc0 = mfma(wa[0][kb][r], fo.xv[u][kb][r], acc0);
        acc1 = mfma(wa[1][kb][r], fo.xv[u][kb][r], acc1);
      }
    const f4 zero = f4{0.0f, 0.0f, 0.0f, 0.0f};
    float* dst = us + (nb * 16 + li) * kUPitch + 4 * G;
    *reinterpret_cast<f4*>(dst) = fo.in[u] ? acc0 : zero;
    *reinterpret_cast<f4*>(dst + 16) = fo.in[u] ? acc1 : zero;
  }
}

// output channels of each group: lightmaps (+Z, -Z), (+X, -X), (+Y, -Y); extra (alpha, emissive)
__constant__ int kDst[4][2] = {{4, 5}, {0, 1}, {2, 3}, {-1, -2}};

}  // namespace
}  // namespace lnm
