// The network's first two 3x3 layers in one launch (device code only).
//
// A workgroup of the second layer (a TH x 16 pixel tile) needs the first
// layer's outputs on its (TH + 2) x 18 halo.  It stages the guide over the
// tile and a two-pixel border in LDS and forms those outputs per input chunk
// of the second layer, as a matrix-core product over the first layer's 27
// (tap, guide channel) pairs: 16-pixel blocks of the halo spread over the
// four waves, then bias, ReLU and the second layer's input format.  The
// first layer's output is then neither stored nor read.
#pragma once
#include "internal.h"

namespace lnm {
namespace first {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

constexpr int kTileW = 16, kHaloW = kTileW + 2, kGuideW = kTileW + 4;

template <int TH>
struct Tile {
  static constexpr int NG = (TH + 4) * kGuideW;  // staged guide pixels
  static constexpr int HP = (TH + 2) * kHaloW;   // halo pixels
  static constexpr int HB = (HP + 15) / 16;      // 16-pixel blocks of the halo
  static constexpr int BPW = (HB + 3) / 4;       // blocks per wave
};

// The guide (fp32, 3 channels) over rows y0 - 2 .. y0 + TH + 1 and columns
// x0 - 2 .. x0 + 17 of image b, one 16-byte entry per pixel, zero outside
// the image.
template <int TH>
__device__ __forceinline__ void stage_guide(const ConvArgs& a, int b, int y0, int x0, f4v* s_g) {
  const float* gs = static_cast<const float*>(a.src0);
  for (int p = threadIdx.x; p < Tile<TH>::NG; p += 256) {
    const int y = y0 + p / kGuideW - 2, x = x0 + p % kGuideW - 2;
    f4v v = f4v{0.f, 0.f, 0.f, 0.f};
    if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
      const float* q = gs + ((size_t)(b * a.H + y) * a.W + x) * 3;
      v = f4v{q[0], q[1], q[2], 0.0f};
    }
    s_g[p] = v;
  }
}

// Staged guide value of K slot k (tap k / 3, channel k % 3; 0 for k >= 27)
// for halo pixel p.
__device__ __forceinline__ float guide_slot(const f4v* s_g, int p, int k) {
  if (k >= 27) return 0.0f;
  const int py = p / kHaloW, px = p - py * kHaloW, tap = k / 3;
  return reinterpret_cast<const float*>(s_g)[((py + tap / 3) * kGuideW + px + tap % 3) * 4 + k % 3];
}

// Whether halo pixel q of the tile at (y0, x0) lies in the image.
__device__ __forceinline__ bool halo_inside(const ConvArgs& a, int y0, int x0, int q) {
  const int py = q / kHaloW, y = y0 + py - 1, x = x0 + q - py * kHaloW - 1;
  return y >= 0 && y < a.H && x >= 0 && x < a.W;
}

__device__ __forceinline__ __bf16 bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __builtin_bit_cast(__bf16, (uint16_t)(u >> 16));
}

// The bf16 first layer (bf16 and fp8 networks; packed weights
// [n-tile][n (32)][k = 3 tap + c (32)] bf16, fp32 bias): chunk ch's 32
// channels at this wave's halo blocks, one K = 32 product per block and 16
// channels with the first layer's own operands in its own K slots.
// emit(bb, nf, r, v) receives v = acc + bias of halo pixel 16 blk + 4g + r
// (blk = wave * BPW + bb) and channel 16 nf + li.
template <int TH, class Emit>
__device__ __forceinline__ void first_layer_bf16(const ConvArgs& a, int ch, const f4v* s_g, Emit emit) {
  using T = Tile<TH>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
  const uint16_t* w0 = static_cast<const uint16_t*>(a.w0) + (size_t)ch * kBN * 32;
  bf16x8v bv[2];
  float bias[2];
#pragma unroll
  for (int nf = 0; nf < 2; ++nf) {
    bv[nf] = *reinterpret_cast<const bf16x8v*>(w0 + (nf * 16 + li) * 32 + 8 * g);
    bias[nf] = a.b0[ch * kBN + nf * 16 + li];
  }
#pragma unroll
  for (int bb = 0; bb < T::BPW; ++bb) {
    const int blk = wave * T::BPW + bb;
    if (blk >= T::HB) break;
    // A: row li of the block is halo pixel p (clamped into the halo)
    const int p = min(blk * 16 + li, T::HP - 1);
    bf16x8v av;
#pragma unroll
    for (int s = 0; s < 8; ++s) av[s] = bf16_rne(guide_slot(s_g, p, 8 * g + s));
#pragma unroll
    for (int nf = 0; nf < 2; ++nf) {
      const f4v d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nf], f4v{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) emit(bb, nf, r, 1.0f * d[r] + bias[nf]);
    }
  }
}

}  // namespace first
}  // namespace lnm
