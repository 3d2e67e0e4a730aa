// U-Net 3x3 convolutions (Section 4.3) in bf16 on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16, fp32 accumulation).  Activations and weights
// are bf16 (round to nearest even), bias and ReLU are applied to the fp32
// accumulator, and the result is rounded to bf16 once.
//
// Same tiling as the fp32 kernel: a workgroup of 4 wavefronts computes a
// TH x 16 pixel tile x 32 output channels; per 32-channel input chunk the
// (TH+2) x 18 halo and the 9 x 32 x 32 weight slab are staged in LDS and read
// by all nine taps; the halo gather fuses zero padding, 2x2 max-pooling and the
// decoder's upsample + skip concatenation.  Large layers take an 8-row x
// 64-channel form (two n-tiles per workgroup, one LDS buffer), which sums
// every output in the same order and so gives the same values.
//
// K-slot permutation: lane group g (= lane / 16) supplies input channels
// 8g .. 8g+7 of the chunk to both MFMA operands, one 16-byte LDS read each.
// The 3-channel input layer packs all 27 (tap, channel) pairs of its 3x3
// window into one 32-wide K step instead of padding each tap to 32 channels.
#include "internal.h"
#include "first_layer.h"
#include "head.h"

namespace lnm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
// 16 bytes as a native vector: arrays of these stay in registers (arrays of
// the u32x4 struct are copied member-wise through memory and were kept in
// scratch)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kTW = 16;
constexpr int kHW = kTW + 2;
constexpr int kCK = 32;   // input channels per chunk
constexpr int kPad = 40;  // bf16 per LDS row (32 + 8 to spread banks)

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// fp32 -> bf16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t max_bf16x2(uint32_t a, uint32_t b) {
  const float lo = fmaxf(bf2f(a & 0xffff), bf2f(b & 0xffff));
  const float hi = fmaxf(bf2f(a >> 16), bf2f(b >> 16));
  // the maximum is one of the inputs, so the bf16 conversion is exact
  return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
}

// Raw loads of eight consecutive channels [c, c+8) of the (virtual) input at
// pixel (y, x), all three clamped to valid positions: the pooled mode keeps
// its four source pixels, the others one value.  They are combined and
// masked only when written to LDS, so a chunk's loads are all in flight
// together and nothing waits on them before the current chunk's matrix work.
template <int MODE>
struct Halo {
  u32x4 v[MODE == G_POOL ? 4 : 1];
};

template <int MODE>
__device__ __forceinline__ Halo<MODE> halo_load(const ConvArgs& a, int b, int y, int x, int c) {
  const uint16_t* s0 = static_cast<const uint16_t*>(a.src0);
  Halo<MODE> h;
  if constexpr (MODE == G_FIRST) {
    h.v[0] = u32x4{0u, 0u, 0u, 0u};
  } else if constexpr (MODE == G_PLAIN) {
    h.v[0] = *reinterpret_cast<const u32x4*>(s0 + ((size_t)(b * a.H + y) * a.W + x) * a.c0 + c);
  } else if constexpr (MODE == G_POOL) {
    const size_t W2 = 2 * (size_t)a.W, c0 = (size_t)a.c0;
    const uint16_t* p = s0 + ((size_t)(b * 2 * a.H + 2 * y) * W2 + 2 * x) * c0 + c;
    h.v[0] = *reinterpret_cast<const u32x4*>(p);
    h.v[1] = *reinterpret_cast<const u32x4*>(p + c0);
    h.v[2] = *reinterpret_cast<const u32x4*>(p + W2 * c0);
    h.v[3] = *reinterpret_cast<const u32x4*>(p + W2 * c0 + c0);
  } else {  // G_CONCAT_UP: channels [0, c0) from the skip, then the upsampled low-res tensor
    const int Hl = a.H >> 1, Wl = a.W >> 1;
    const uint16_t* skip = s0 + ((size_t)(b * a.H + y) * a.W + x) * a.c0 + c;
    const uint16_t* up = static_cast<const uint16_t*>(a.src1) +
                         ((size_t)(b * Hl + (y >> 1)) * Wl + (x >> 1)) * a.c1 + max(c - a.c0, 0);
    h.v[0] = *reinterpret_cast<const u32x4*>(c < a.c0 ? skip : up);
  }
  return h;
}

template <int MODE>
__device__ __forceinline__ u32x4 halo_value(const Halo<MODE>& h, bool ok) {
  u32x4 r = h.v[0];
  if constexpr (MODE == G_POOL) {
    r.x = max_bf16x2(max_bf16x2(h.v[0].x, h.v[1].x), max_bf16x2(h.v[2].x, h.v[3].x));
    r.y = max_bf16x2(max_bf16x2(h.v[0].y, h.v[1].y), max_bf16x2(h.v[2].y, h.v[3].y));
    r.z = max_bf16x2(max_bf16x2(h.v[0].z, h.v[1].z), max_bf16x2(h.v[2].z, h.v[3].z));
    r.w = max_bf16x2(max_bf16x2(h.v[0].w, h.v[1].w), max_bf16x2(h.v[2].w, h.v[3].w));
  }
  return ok ? r : u32x4{0u, 0u, 0u, 0u};
}

template <int TH, int NF = 2>
__device__ __forceinline__ void store_tile(const ConvArgs& a, const f4 (&acc)[TH / 4][NF], int b, int y0, int x0,
                                           int wrow, int g, int li, int nt, int ks) {
  uint16_t* out = static_cast<uint16_t*>(a.out);
#pragma unroll
  for (int mf = 0; mf < TH / 4; ++mf) {
    const int y = y0 + wrow + mf;
    if (y >= a.H) continue;
#pragma unroll
    for (int nf = 0; nf < NF; ++nf) {
      const int n = nt * kBN + nf * 16 + li;
      if (n >= a.co) continue;
      const float bias = a.bias[n];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = x0 + 4 * g + r;
        if (x >= a.W) continue;
        const size_t pix = (size_t)(b * a.H + y) * a.W + x;
        if (a.splits > 1) {
          a.partial[((size_t)ks * a.B * a.H * a.W + pix) * a.co + n] = acc[mf][nf][r];
          continue;
        }
        float v = acc[mf][nf][r] + bias;
        if (a.relu) v = fmaxf(v, 0.0f);
        out[pix * a.co + n] = f2bf(v);
      }
    }
  }
}

// NB output-channel tiles of 32 per workgroup (NF = 2 NB 16-column MFMA
// blocks per wave) and NBUF LDS buffers: the default is one tile, double
// buffered; the large-layer form (8 rows x 64 channels, 2 x 4 blocks per
// wave: a quarter fewer LDS reads per MFMA, and the halo read once for 64
// channels) is single buffered, its next chunk prefetched into registers,
// so two workgroups share a CU.  (16 rows x 64 channels, 4 x 4 blocks, needs
// more than 256 registers per lane: one wave per SIMD, and slower.)
template <int MODE, int TH, bool HEAD, int NB = 1, int NBUF = 2>
__global__ __launch_bounds__(256) void conv3x3_bf16(ConvArgs a, HeadFuse hf) {
  constexpr int MF = TH / 4, NF = 2 * NB, BN = kBN * NB;
  __shared__ __attribute__((aligned(16))) uint16_t s_in[NBUF][(TH + 2) * kHW * kPad];
  __shared__ __attribute__((aligned(16))) uint16_t s_w[NBUF][9 * BN * kPad];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_y = (a.H + TH - 1) / TH;
  const int b = blockIdx.y / tiles_y;
  const int y0 = (blockIdx.y - b * tiles_y) * TH, x0 = blockIdx.x * kTW;
  const int g = lane >> 4, li = lane & 15, wrow = wave * MF;
  const int groups = (a.n_tiles + NB - 1) / NB;
  const int nt = (blockIdx.z % groups) * NB, ks = blockIdx.z / groups;
  const int nchunks = a.ci_pad / kCK;
  const int ch_lo = ks * nchunks / a.splits, ch_hi = (ks + 1) * nchunks / a.splits;
  const int ci = a.c0 + a.c1;  // real input channels (the rest of ci_pad is zero padding)
  const size_t tile_elems = (size_t)nchunks * 9 * kBN * kCK;  // one n-tile's packed weights
  const uint16_t* wblk = static_cast<const uint16_t*>(a.w) + (size_t)nt * tile_elems;

  f4 acc[MF][NF];
#pragma unroll
  for (int mf = 0; mf < MF; ++mf)
#pragma unroll
    for (int nf = 0; nf < NF; ++nf) acc[mf][nf] = f4{0.f, 0.f, 0.f, 0.f};

  // G_FIRST: the first layer's outputs on the halo, formed from the staged
  // guide as the first layer's own kernel forms them (the same bf16
  // operands in the same K slots, bias, ReLU, one rounding to bf16), so the
  // result is the same bit for bit
  using FT = first::Tile<TH>;
  __shared__ f4 s_g[MODE == G_FIRST ? FT::NG : 1];
  uint16_t fr[MODE == G_FIRST ? 8 * FT::BPW : 1];
  auto first_layer = [&](int ch) {
    first::first_layer_bf16<TH>(a, ch, s_g, [&](int bb, int nf, int r, float v) {
      fr[8 * bb + 4 * nf + r] = f2bf(fmaxf(v, 0.0f));
    });
  };

  constexpr int NQ = (TH + 2) * kHW * (kCK / 8), NW = 9 * BN * kCK / 8;
  constexpr int RQ = (NQ + 255) / 256, RW = (NW + 255) / 256;
  Halo<MODE> rq[RQ];
  u32x4 rw[RW];
  unsigned ok = 0;
  auto fetch = [&](int ch) {
    ok = 0;
#pragma unroll
    for (int r = 0; r < (MODE == G_FIRST ? 0 : RQ); ++r) {
      const int q = min(tid + 256 * r, NQ - 1);
      const int c8 = q & 3, p = q >> 2;
      const int y = y0 + p / kHW - 1, x = x0 + p % kHW - 1, c = ch * kCK + 8 * c8;
      const bool in = tid + 256 * r < NQ && y >= 0 && y < a.H && x >= 0 && x < a.W && c < ci;
      ok |= (unsigned)in << r;
      rq[r] = halo_load<MODE>(a, b, min(max(y, 0), a.H - 1), min(max(x, 0), a.W - 1), c < ci ? c : 0);
    }
    const uint16_t* wsrc = wblk + (size_t)ch * 9 * kBN * kCK;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      // LDS row (tap, n of BN) <- n-tile nt + n / 32's slab [tap][n % 32][c]
      // (past the last tile of an odd count: the last tile again, its
      // outputs are not stored)
      const int q = min(tid + 256 * r, NW - 1);
      const int row = q >> 2, tap = row / BN, n = row - tap * BN;
      const int tsel = min(nt + n / kBN, a.n_tiles - 1) - nt;
      rw[r] = *reinterpret_cast<const u32x4*>(wsrc + (size_t)tsel * tile_elems +
                                              ((tap * kBN + n % kBN) * kCK + 8 * (q & 3)));
    }
    if constexpr (MODE == G_FIRST) first_layer(ch);
  };
  auto commit = [&](int buf) {
    if constexpr (MODE == G_FIRST) {
      // this lane's first-layer outputs: channels 16 nf + li at halo pixels
      // 16 blk + 4g + r (zero padding outside the image)
#pragma unroll
      for (int bb = 0; bb < FT::BPW; ++bb) {
        const int blk = wave * FT::BPW + bb;
        if (blk >= FT::HB) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = blk * 16 + 4 * g + r;
          if (q >= FT::HP) continue;
          const bool in = first::halo_inside(a, y0, x0, q);
#pragma unroll
          for (int nf = 0; nf < 2; ++nf) s_in[buf][q * kPad + nf * 16 + li] = in ? fr[8 * bb + 4 * nf + r] : 0;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < (MODE == G_FIRST ? 0 : RQ); ++r) {
      const int q = tid + 256 * r;
      if (q < NQ)
        *reinterpret_cast<u32x4*>(&s_in[buf][(q >> 2) * kPad + 8 * (q & 3)]) = halo_value<MODE>(rq[r], (ok >> r) & 1u);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int q = tid + 256 * r;
      if (q < NW) *reinterpret_cast<u32x4*>(&s_w[buf][(q >> 2) * kPad + 8 * (q & 3)]) = rw[r];
    }
  };

  if constexpr (MODE == G_FIRST) {
    first::stage_guide<TH>(a, b, y0, x0, s_g);
    __syncthreads();
  }
  if (ch_lo < ch_hi) {
    fetch(ch_lo);
    commit(0);
  }
  __syncthreads();
  for (int ch = ch_lo; ch < ch_hi; ++ch) {
    const int cur = NBUF == 2 ? (ch - ch_lo) & 1 : 0;
    const bool more = ch + 1 < ch_hi;
    if (more) fetch(ch + 1);
    const uint16_t* si = s_in[cur];
    const uint16_t* sw = s_w[cur];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap - 3 * (tap / 3);
      bf16x8 av[MF], bv[NF];
#pragma unroll
      for (int mf = 0; mf < MF; ++mf)
        av[mf] = *reinterpret_cast<const bf16x8*>(&si[((wrow + mf + dy) * kHW + li + dx) * kPad + 8 * g]);
#pragma unroll
      for (int nf = 0; nf < NF; ++nf)
        bv[nf] = *reinterpret_cast<const bf16x8*>(&sw[(tap * BN + nf * 16 + li) * kPad + 8 * g]);
#pragma unroll
      for (int mf = 0; mf < MF; ++mf)
#pragma unroll
        for (int nf = 0; nf < NF; ++nf)
          acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mf], bv[nf], acc[mf][nf], 0, 0, 0);
    }
    if constexpr (NBUF == 2) {
      if (more) commit(cur ^ 1);
      __syncthreads();
    } else {  // one buffer: every wave is done reading it before it is refilled
      __syncthreads();
      if (more) {
        commit(0);
        __syncthreads();
      }
    }
  }
  if constexpr (HEAD) {
    // head epilogue: the activations as they would be stored (bf16 of
    // bias + ReLU) and the head weights in LDS (the weight buffer is free
    // after the last chunk's barrier), then one thread per pixel
    static_assert((TH * kTW * 33 + 6 * kBN) * 4 <= 9 * kBN * kPad * 2, "head tile must fit the weight buffer");
    float* sh = reinterpret_cast<float*>(s_w[0]);
    float* shw = sh + TH * kTW * 33;
    head_weights(hf, a.co, shw);
#pragma unroll
    for (int mf = 0; mf < MF; ++mf)
#pragma unroll
      for (int nf = 0; nf < 2; ++nf) {
        const int n = nf * 16 + li;
        const float bias = n < a.co ? a.bias[n] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sh[((wrow + mf) * kTW + 4 * g + r) * 33 + n] = bf2f(f2bf(fmaxf(acc[mf][nf][r] + bias, 0.0f)));
      }
    __syncthreads();
    head_finish<TH>(hf, sh, shw, b, a.H, a.W, y0, x0);
    return;
  }
  store_tile<TH, NF>(a, acc, b, y0, x0, wrow, g, li, nt, ks);
}

// First layer: 3 fp32 input channels; K slot k = 3 tap + c for k < 27.
// Packed weights per n-tile: [n (32)][k (32)] bf16.
template <int TH>
__global__ __launch_bounds__(256) void conv3x3_bf16_guide(ConvArgs a) {
  constexpr int MF = TH / 4;
  __shared__ __attribute__((aligned(16))) float s_in[(TH + 2) * kHW * 4];
  __shared__ __attribute__((aligned(16))) uint16_t s_w[kBN * kPad];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_y = (a.H + TH - 1) / TH;
  const int b = blockIdx.y / tiles_y;
  const int y0 = (blockIdx.y - b * tiles_y) * TH, x0 = blockIdx.x * kTW;
  const int g = lane >> 4, li = lane & 15, wrow = wave * MF;
  const float* gsrc = static_cast<const float*>(a.src0);
  for (int p = tid; p < (TH + 2) * kHW; p += 256) {
    const int hx = p % kHW, hy = p / kHW, y = y0 + hy - 1, x = x0 + hx - 1;
    f4 v = f4{0.f, 0.f, 0.f, 0.f};
    if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
      const float* q = gsrc + ((size_t)(b * a.H + y) * a.W + x) * 3;
      v = f4{q[0], q[1], q[2], 0.0f};
    }
    *reinterpret_cast<f4*>(&s_in[4 * p]) = v;
  }
  const uint16_t* wsrc = static_cast<const uint16_t*>(a.w) + (size_t)blockIdx.z * kBN * kCK;
  for (int q = tid; q < kBN * kCK / 8; q += 256) {
    const int c8 = q & 3, row = q >> 2;
    *reinterpret_cast<u32x4*>(&s_w[row * kPad + 8 * c8]) = *reinterpret_cast<const u32x4*>(wsrc + 8 * q);
  }
  __syncthreads();
  f4 acc[MF][2];
  bf16x8 bv[2];
#pragma unroll
  for (int nf = 0; nf < 2; ++nf) bv[nf] = *reinterpret_cast<const bf16x8*>(&s_w[(nf * 16 + li) * kPad + 8 * g]);
#pragma unroll
  for (int mf = 0; mf < MF; ++mf) {
    bf16x8 av;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 8 * g + s;
      float v = 0.0f;
      if (k < 27) {
        const int tap = k / 3, c = k - 3 * tap;
        v = s_in[((wrow + mf + tap / 3) * kHW + li + (tap - 3 * (tap / 3))) * 4 + c];
      }
      av[s] = __builtin_bit_cast(__bf16, f2bf(v));
    }
#pragma unroll
    for (int nf = 0; nf < 2; ++nf)
      acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nf], f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  }
  store_tile<TH>(a, acc, b, y0, x0, wrow, g, li, blockIdx.z, 0);
}

template <int MODE, int TH>
hipError_t launch_th(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  dim3 grid((a.W + kTW - 1) / kTW, ((a.H + TH - 1) / TH) * a.B, a.n_tiles * a.splits);
  if constexpr (MODE == G_GUIDE) {
    if (head) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conv3x3_bf16_guide<TH>), grid, dim3(256), 0, s, a);
  } else if constexpr (MODE == G_PLAIN) {
    if (head)
      hipLaunchKernelGGL((conv3x3_bf16<MODE, TH, true>), grid, dim3(256), 0, s, a, *head);
    else
      hipLaunchKernelGGL((conv3x3_bf16<MODE, TH, false>), grid, dim3(256), 0, s, a, HeadFuse{});
  } else {
    if (head) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conv3x3_bf16<MODE, TH, false>), grid, dim3(256), 0, s, a, HeadFuse{});
  }
  return hipGetLastError();
}
// Large-layer form: kBf16LargeRows x 16 pixels x 64 channels per workgroup,
// one LDS buffer.
template <int MODE>
hipError_t launch_large(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if (head || a.n_tiles < 2) return hipErrorInvalidValue;
  constexpr int R = kBf16LargeRows;
  dim3 grid((a.W + kTW - 1) / kTW, ((a.H + R - 1) / R) * a.B, ((a.n_tiles + 1) / 2) * a.splits);
  hipLaunchKernelGGL((conv3x3_bf16<MODE, R, false, 2, 1>), grid, dim3(256), 0, s, a, HeadFuse{});
  return hipGetLastError();
}
// 8-row tiles, 4-row tiles or the large-layer form when the layer asks for
// them (not the input layer)
template <int MODE>
hipError_t launch_tile(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if constexpr (MODE != G_GUIDE) {
    if (a.th == 4) return launch_th<MODE, 4>(a, s, head);
    if (a.th == kBf16Large) return launch_large<MODE>(a, s, head);
  }
  return launch_th<MODE, 8>(a, s, head);
}

}  // namespace

hipError_t launch_conv3x3_bf16(int mode, const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if (head && (a.n_tiles != 1 || a.splits != 1 || a.co > kBN || !a.relu)) return hipErrorInvalidValue;
  switch (mode) {
    case G_FIRST:
      if (!a.w0 || !a.b0 || head || a.th == kBf16Large) return hipErrorInvalidValue;
      return launch_tile<G_FIRST>(a, s, head);
    case G_GUIDE: return launch_tile<G_GUIDE>(a, s, head);
    case G_PLAIN: return launch_tile<G_PLAIN>(a, s, head);
    case G_POOL: return launch_tile<G_POOL>(a, s, head);
    case G_CONCAT_UP: return launch_tile<G_CONCAT_UP>(a, s, head);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lnm
