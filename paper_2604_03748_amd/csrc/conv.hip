// U-Net layers (Section 4.3) for gfx950, fp32.
//
// 3x3 convolution as an implicit GEMM on the fp32 matrix cores
// (v_mfma_f32_16x16x4_f32): M = output pixels, N = output channels,
// K = 9 taps x input channels.  Activations are NHWC.
//
// Workgroup = 4 wavefronts computing a TH x 16 pixel tile x 32 output
// channels.  Per 16-channel input chunk the (TH+2) x 18 input halo and the
// 9 x 32 x 16 weight slab are staged in LDS once and every tap reads them
// from there.  The gather that fills the halo fuses the zero padding, the
// 2x2 max-pool of the encoder (pooled input mode) and the decoder's nearest
// 2x upsample + skip concatenation (two-source mode), so none of those
// tensors is materialised.  The epilogue adds the bias and applies ReLU; in
// the network's last layer it can instead apply the 1x1 head (and the
// frame's shading) without storing the layer.  Layers with few tiles are
// split over K and finished by splitk_reduce; conv_layer_tiling picks each
// layer's tile height and split.
//
// K-slot permutation: MFMA step jj pairs lane group g (= lane / 16) with input
// channel 4g + jj for both operands, so each lane fetches its four channels of
// A and of B with one 16-byte LDS read.
#include "internal.h"
#include "first_layer.h"
#include "head.h"

namespace lnm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTW = 16;        // tile width in pixels (= MFMA M)
constexpr int kHW = kTW + 2;   // halo width

template <int CK>
struct Pad {
  static constexpr int in = CK == 16 ? 20 : 4;  // LDS floats per halo pixel
  static constexpr int w = CK == 16 ? 20 : 4;   // LDS floats per weight row
};

// Raw loads of one halo entry (four channels at pixel (y, x), both clamped
// into the image): the pooled mode keeps its four source pixels, the others
// one value.  They are combined and masked only when written to LDS, so the
// loads of a chunk are all in flight together and nothing waits on them
// before the matrix work of the current chunk.
template <int MODE>
struct Halo {
  f4 v[MODE == G_POOL ? 4 : 1];
};

template <int MODE>
__device__ __forceinline__ Halo<MODE> halo_load(const ConvArgs& a, int b, int y, int x, int c) {
  const float* s0 = static_cast<const float*>(a.src0);
  Halo<MODE> h;
  if constexpr (MODE == G_FIRST) {
    h.v[0] = f4{0.f, 0.f, 0.f, 0.f};
  } else if constexpr (MODE == G_GUIDE) {
    const float* g = s0 + ((size_t)(b * a.H + y) * a.W + x) * 3;
    h.v[0] = f4{g[0], g[1], g[2], 0.0f};
  } else if constexpr (MODE == G_PLAIN) {
    h.v[0] = *reinterpret_cast<const f4*>(s0 + ((size_t)(b * a.H + y) * a.W + x) * a.c0 + c);
  } else if constexpr (MODE == G_POOL) {
    const size_t W2 = 2 * (size_t)a.W, c0 = (size_t)a.c0;
    const float* p = s0 + ((size_t)(b * 2 * a.H + 2 * y) * W2 + 2 * x) * c0 + c;
    h.v[0] = *reinterpret_cast<const f4*>(p);
    h.v[1] = *reinterpret_cast<const f4*>(p + c0);
    h.v[2] = *reinterpret_cast<const f4*>(p + W2 * c0);
    h.v[3] = *reinterpret_cast<const f4*>(p + W2 * c0 + c0);
  } else {  // G_CONCAT_UP: channels [0, c0) from the skip, then the upsampled low-res tensor
    const int Hl = a.H >> 1, Wl = a.W >> 1;
    const float* skip = s0 + ((size_t)(b * a.H + y) * a.W + x) * a.c0 + c;
    const float* up = static_cast<const float*>(a.src1) + ((size_t)(b * Hl + (y >> 1)) * Wl + (x >> 1)) * a.c1 +
                      max(c - a.c0, 0);
    h.v[0] = *reinterpret_cast<const f4*>(c < a.c0 ? skip : up);
  }
  return h;
}

template <int MODE>
__device__ __forceinline__ f4 halo_value(const Halo<MODE>& h, bool ok) {
  f4 v = h.v[0];
  if constexpr (MODE == G_POOL) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = fmaxf(fmaxf(h.v[0][e], h.v[1][e]), fmaxf(h.v[2][e], h.v[3][e]));
  }
  return ok ? v : f4{0.f, 0.f, 0.f, 0.f};
}

template <int CK, int MODE, int TH, bool HEAD>
__global__ __launch_bounds__(256) void conv3x3_f32(ConvArgs a, HeadFuse hf) {
  constexpr int NF = kBN / 16;
  constexpr int MF = TH / 4;
  constexpr int PIN = Pad<CK>::in, PW = Pad<CK>::w;
  // two LDS buffers: the next chunk is fetched into registers while the
  // matrix cores work on the current one
  __shared__ __attribute__((aligned(16))) float s_in[2][(TH + 2) * kHW * PIN];
  __shared__ __attribute__((aligned(16))) float s_w[2][9 * kBN * PW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_y = (a.H + TH - 1) / TH;
  const int b = blockIdx.y / tiles_y;
  const int y0 = (blockIdx.y - b * tiles_y) * TH, x0 = blockIdx.x * kTW;
  const int nt = blockIdx.z % a.n_tiles, ks = blockIdx.z / a.n_tiles;
  const int nchunks = a.ci_pad / CK;
  const int ch_lo = ks * nchunks / a.splits, ch_hi = (ks + 1) * nchunks / a.splits;
  const float* wblk = static_cast<const float*>(a.w) + (size_t)nt * nchunks * 9 * kBN * CK;
  const int g = lane >> 4, li = lane & 15;
  const int wrow = wave * MF;

  f4 acc[MF][NF];
#pragma unroll
  for (int mf = 0; mf < MF; ++mf)
#pragma unroll
    for (int nf = 0; nf < NF; ++nf) acc[mf][nf] = f4{0.f, 0.f, 0.f, 0.f};

  // G_FIRST: per chunk, the first layer's outputs at the halo pixels are a
  // K = 27 product on the matrix cores (A: the pixels' 3x3 x 3 staged guide
  // values, B: the chunk's 16 channels of first-layer weights), then bias
  // and ReLU.  The products are taken in the first layer's own K order (tap,
  // then guide channel), and the outputs matched the separate first layer's
  // bit for bit wherever they were compared.
  using FT = first::Tile<TH>;
  __shared__ f4 s_g[MODE == G_FIRST ? FT::NG : 1];
  float fr[MODE == G_FIRST ? 4 * FT::BPW : 1];
  auto first_layer = [&](int ch) {
    // B: W0[k][n] for k = 4 s + g, n = ch * 16 + li, from the packed
    // [n / 32][tap][n % 32][c (4)]
    const int n = ch * CK + li;
    const float* w = static_cast<const float*>(a.w0) + (size_t)(n / kBN) * 9 * kBN * 4 + (n % kBN) * 4;
    float bk[7];
#pragma unroll
    for (int st = 0; st < 7; ++st) {
      const int k = 4 * st + g;
      bk[st] = k < 27 ? w[(k / 3) * kBN * 4 + k % 3] : 0.0f;
    }
    const float bias = a.b0[n];
#pragma unroll
    for (int bb = 0; bb < FT::BPW; ++bb) {
      const int blk = wave * FT::BPW + bb;
      if (blk >= FT::HB) break;
      // A: row li of the block is halo pixel p (clamped into the halo)
      const int p = min(blk * 16 + li, FT::HP - 1);
      f4 d = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < 7; ++st)
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(first::guide_slot(s_g, p, 4 * st + g), bk[st], d, 0, 0, 0);
      // D: rows 4g + r of the block (pixels), column li (channel)
#pragma unroll
      for (int r = 0; r < 4; ++r) fr[4 * bb + r] = fmaxf(d[r] + bias, 0.0f);
    }
  };

  // per chunk: the (TH+2) x 18 input halo and the weight slab [tap][n][c];
  // every load is unconditional (clamped index), masks apply at commit
  constexpr int NQ = (TH + 2) * kHW * (CK / 4), NW = 9 * kBN * CK / 4;
  constexpr int RQ = (NQ + 255) / 256, RW = (NW + 255) / 256;
  Halo<MODE> rq[RQ];
  f4 rw[RW];
  unsigned ok = 0;
  auto fetch_w = [&](int ch) {
    const float* wsrc = wblk + (size_t)ch * 9 * kBN * CK;
#pragma unroll
    for (int r = 0; r < RW; ++r) rw[r] = *reinterpret_cast<const f4*>(wsrc + 4 * min(tid + 256 * r, NW - 1));
  };
  auto fetch = [&](int ch) {
    ok = 0;
#pragma unroll
    for (int r = 0; r < (MODE == G_FIRST ? 0 : RQ); ++r) {
      const int q = min(tid + 256 * r, NQ - 1);
      const int c4 = q % (CK / 4), p = q / (CK / 4);
      const int y = y0 + p / kHW - 1, x = x0 + p % kHW - 1;
      const bool in = tid + 256 * r < NQ && y >= 0 && y < a.H && x >= 0 && x < a.W;
      ok |= (unsigned)in << r;
      rq[r] = halo_load<MODE>(a, b, min(max(y, 0), a.H - 1), min(max(x, 0), a.W - 1), ch * CK + 4 * c4);
    }
    fetch_w(ch);
    if constexpr (MODE == G_FIRST) first_layer(ch);
  };
  auto commit = [&](int buf) {
    if constexpr (MODE == G_FIRST) {
      // this lane's first-layer outputs: channel li at halo pixels
      // 16 blk + 4g + r (zero padding outside the image)
#pragma unroll
      for (int bb = 0; bb < FT::BPW; ++bb) {
        const int blk = wave * FT::BPW + bb;
        if (blk >= FT::HB) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = blk * 16 + 4 * g + r;
          if (q < FT::HP) s_in[buf][q * PIN + li] = first::halo_inside(a, y0, x0, q) ? fr[4 * bb + r] : 0.0f;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < (MODE == G_FIRST ? 0 : RQ); ++r) {
      const int q = tid + 256 * r;
      if (q < NQ)
        *reinterpret_cast<f4*>(&s_in[buf][(q / (CK / 4)) * PIN + 4 * (q % (CK / 4))]) =
            halo_value<MODE>(rq[r], (ok >> r) & 1u);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int q = tid + 256 * r;
      if (q < NW) *reinterpret_cast<f4*>(&s_w[buf][(q / (CK / 4)) * PW + 4 * (q % (CK / 4))]) = rw[r];
    }
  };

  if constexpr (MODE == G_FIRST) {
    // the first chunk's weights in flight while the guide is staged
    if (ch_lo < ch_hi) fetch_w(ch_lo);
    first::stage_guide<TH>(a, b, y0, x0, s_g);
    __syncthreads();
    if (ch_lo < ch_hi) {
      first_layer(ch_lo);
      commit(0);
    }
  } else if (ch_lo < ch_hi) {
    fetch(ch_lo);
    commit(0);
  }
  __syncthreads();
  for (int ch = ch_lo; ch < ch_hi; ++ch) {
    const int cur = (ch - ch_lo) & 1;
    const bool more = ch + 1 < ch_hi;
    if (more) fetch(ch + 1);
    const float* si = s_in[cur];
    const float* sw = s_w[cur];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap - 3 * (tap / 3);
      if constexpr (CK == 16) {
        f4 av[MF], bv[NF];
#pragma unroll
        for (int mf = 0; mf < MF; ++mf)
          av[mf] = *reinterpret_cast<const f4*>(&si[((wrow + mf + dy) * kHW + li + dx) * PIN + 4 * g]);
#pragma unroll
        for (int nf = 0; nf < NF; ++nf)
          bv[nf] = *reinterpret_cast<const f4*>(&sw[(tap * kBN + nf * 16 + li) * PW + 4 * g]);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int mf = 0; mf < MF; ++mf)
#pragma unroll
            for (int nf = 0; nf < NF; ++nf)
              acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mf][jj], bv[nf][jj], acc[mf][nf], 0, 0, 0);
      } else {
        float av[MF], bv[NF];
#pragma unroll
        for (int mf = 0; mf < MF; ++mf) av[mf] = si[((wrow + mf + dy) * kHW + li + dx) * PIN + g];
#pragma unroll
        for (int nf = 0; nf < NF; ++nf) bv[nf] = sw[(tap * kBN + nf * 16 + li) * PW + g];
#pragma unroll
        for (int mf = 0; mf < MF; ++mf)
#pragma unroll
          for (int nf = 0; nf < NF; ++nf)
            acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mf], bv[nf], acc[mf][nf], 0, 0, 0);
      }
    }
    if (more) commit(cur ^ 1);
    __syncthreads();
  }

  if constexpr (HEAD) {
    // head epilogue (one 32-channel tile, unsplit, ReLU layer): the tile's
    // activations (bias + ReLU) and the head weights go to LDS (the weight
    // buffer is free after the last chunk's barrier), then one thread per
    // pixel finishes the head
    static_assert(TH * kTW * 33 + 6 * kBN <= 9 * kBN * PW, "head tile must fit the weight buffer");
    float* sh = s_w[0];
    float* shw = sh + TH * kTW * 33;
    head_weights(hf, a.co, shw);
#pragma unroll
    for (int mf = 0; mf < MF; ++mf)
#pragma unroll
      for (int nf = 0; nf < NF; ++nf) {
        const int n = nf * 16 + li;
        const float bias = n < a.co ? a.bias[n] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) sh[((wrow + mf) * kTW + 4 * g + r) * 33 + n] = fmaxf(acc[mf][nf][r] + bias, 0.0f);
      }
    __syncthreads();
    head_finish<TH>(hf, sh, shw, b, a.H, a.W, y0, x0);
    return;
  }
  // epilogue: lane holds rows (pixels) 4g..4g+3 of each 16x16 block, column
  // li; the stores are non-temporal (the next layer reads the tensor from
  // another XCD, so keeping it in this XCD's L2 only adds to the write-back
  // at the end of the kernel; measured 5 us per fp32 frame)
#pragma unroll
  for (int mf = 0; mf < MF; ++mf) {
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
          __builtin_nontemporal_store(acc[mf][nf][r], a.partial + ((size_t)ks * a.B * a.H * a.W + pix) * a.co + n);
          continue;
        }
        float v = acc[mf][nf][r] + bias;
        if (a.relu) v = fmaxf(v, 0.0f);
        __builtin_nontemporal_store(v, static_cast<float*>(a.out) + pix * a.co + n);
      }
    }
  }
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Finish a split-K layer: sum the splits in order, then the layer epilogue.
// One lane per four consecutive output elements (channels of one pixel: the
// channel count is a multiple of 16); the S partial loads are issued before
// the in-order sum.
template <int S>
__global__ __launch_bounds__(256) void splitk_reduce(ConvArgs a, int out_type, long total4) {
  const long i4 = (long)blockIdx.x * 256 + threadIdx.x;
  if (i4 >= total4) return;
  const size_t total = (size_t)total4 * 4;
  f4 v[S];
#pragma unroll
  for (int k = 0; k < S; ++k) v[k] = *reinterpret_cast<const f4*>(a.partial + k * total + 4 * i4);
  const int n0 = (int)((4 * i4) % a.co);
  float y[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < S; ++k) acc += v[k][e];
    const int n = n0 + e;
    if (out_type == 2) {
      float t = a.in_scale * a.w_scale[n] * acc + a.bias[n];
      t = t > 0.0f ? t * a.out_inv_scale : 0.0f;
      y[e] = fminf(t, 448.0f);
    } else if (out_type == 3) {
      y[e] = fmaxf(a.in_scale * a.w_scale[n] * acc + a.bias[n], 0.0f);
    } else {
      float t = acc + a.bias[n];
      if (a.relu) t = fmaxf(t, 0.0f);
      y[e] = t;
    }
  }
  if (out_type == 2) {
    uint32_t packed = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      packed |= ((uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y[e], 0.0f, 0, false) & 0xffu) << (8 * e);
    static_cast<uint32_t*>(a.out)[i4] = packed;
  } else if (out_type == 1 || out_type == 3) {
    static_cast<uint2*>(a.out)[i4] = make_uint2((uint32_t)f32_to_bf16(y[0]) | ((uint32_t)f32_to_bf16(y[1]) << 16),
                                                (uint32_t)f32_to_bf16(y[2]) | ((uint32_t)f32_to_bf16(y[3]) << 16));
  } else {
    static_cast<f4*>(a.out)[i4] = f4{y[0], y[1], y[2], y[3]};
  }
}

// 1x1 head C -> 6 and sigmoid, one lane per pixel; fp32 arithmetic on fp32
// (IN = 0), bf16 (IN = 1) or e4m3 (IN = 2) activations.  With COMP the
// pixel is also shaded from the lightmap values it just stored (the frame's
// head and composite in one launch; same values as the separate kernels).
template <int IN, bool COMP>
__global__ __launch_bounds__(256) void head_kernel(HeadArgs a, CompositeArgs comp) {
  __shared__ float sw[6 * 256];
  __shared__ float sb[6];
  for (int q = threadIdx.x; q < 6 * a.C; q += 256) sw[q] = a.w[q];
  if (threadIdx.x < 6) sb[threadIdx.x] = a.b[threadIdx.x];
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= a.P) return;
  float z[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) z[o] = sb[o];
  for (int c = 0; c < a.C; c += 4) {
    f4 v;
    if constexpr (IN == 0) {
      v = *reinterpret_cast<const f4*>(static_cast<const float*>(a.in) + (size_t)p * a.C + c);
    } else if constexpr (IN == 2) {
      const int q = *reinterpret_cast<const int*>(static_cast<const uint8_t*>(a.in) + (size_t)p * a.C + c);
      v = f4{__builtin_amdgcn_cvt_f32_fp8(q, 0), __builtin_amdgcn_cvt_f32_fp8(q, 1),
             __builtin_amdgcn_cvt_f32_fp8(q, 2), __builtin_amdgcn_cvt_f32_fp8(q, 3)} *
          a.in_scale;
    } else {
      const uint2 q = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.in) + (size_t)p * a.C + c);
      v = f4{bf16_to_f32(q.x & 0xffff), bf16_to_f32(q.x >> 16), bf16_to_f32(q.y & 0xffff), bf16_to_f32(q.y >> 16)};
    }
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      const float* w = sw + o * a.C + c;
      z[o] += w[0] * v.x + w[1] * v.y + w[2] * v.z + w[3] * v.w;
    }
  }
  float L[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (a.logits) a.logits[(size_t)p * 6 + o] = z[o];
    L[o] = 1.0f / (1.0f + expf(-z[o]));
    a.lm[(size_t)p * 6 + o] = L[o];
  }
  if constexpr (COMP) shade_pixel(comp, p, L);
}

// Six-way shading of stored lightmaps.
__global__ __launch_bounds__(256) void composite_kernel(CompositeArgs a) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= a.P) return;
  float L[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) L[q] = a.lm[(size_t)p * 6 + q];
  shade_pixel(a, p, L);
}

// Six-way shading of a batch of images with per-image lights.
__global__ __launch_bounds__(256) void composite_batch_kernel(CompositeBatchArgs a) {
  const long p = (long)blockIdx.x * 256 + threadIdx.x;
  if (p >= (long)a.P * a.B) return;
  const int b = (int)(p / a.P);
  float L[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) L[q] = a.lm[(size_t)p * 6 + q];
  shade_lights(a.l, a.rgb, a.light_lo[b], a.light_lo[b + 1], a.guide, a.rgba, (size_t)p, L);
}

// Weight gradient of a 3x3 layer: dW[o][c][tap] = sum_p E[p][o] X[p + tap][c]
// as an MFMA GEMM with M = output channels, N = input channels, K = pixels.
// Workgroup: 32 output channels x 16 input channels x 9 taps over a group of
// 8 x 16 pixel tiles; each wavefront takes two tile rows (32 pixels, 8 K-steps
// of 4) and keeps its own partial sums, written to partial[group * 4 + wave]
// and summed in a fixed order by wgrad_reduce.  X is gathered exactly as the
// forward pass reads it (pooled / upsampled-concatenated inputs stay virtual).
constexpr int kWTH = 8;

template <int MODE>
__global__ __launch_bounds__(256) void wgrad3x3_f32(WgradArgs a) {
  __shared__ float s_e[kWTH * kTW][33];
  __shared__ float s_x[(kWTH + 2) * kHW][17];
  const ConvArgs& x = a.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, li = lane & 15;
  const int tiles_x = (x.W + kTW - 1) / kTW, tiles_y = (x.H + kWTH - 1) / kWTH;
  const int n_tiles = x.B * tiles_x * tiles_y;
  const int o0 = blockIdx.y * kBN, c0 = blockIdx.z * 16;
  const int co_pad = gridDim.y * kBN;
  f4 acc[2][9];
#pragma unroll
  for (int of = 0; of < 2; ++of)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[of][t] = f4{0.f, 0.f, 0.f, 0.f};

  const int t_end = min(n_tiles, (int)(blockIdx.x + 1) * a.tiles_per_group);
  for (int t = blockIdx.x * a.tiles_per_group; t < t_end; ++t) {
    const int b = t / (tiles_x * tiles_y), r = t - b * tiles_x * tiles_y;
    const int y0 = (r / tiles_x) * kWTH, x0 = (r - (r / tiles_x) * tiles_x) * kTW;
    for (int q = tid; q < kWTH * kTW * 8; q += 256) {
      const int p = q >> 3, o = o0 + 4 * (q & 7);
      const int y = y0 + p / kTW, xx = x0 + p % kTW;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (y < x.H && xx < x.W && o < a.co) v = *reinterpret_cast<const f4*>(a.e + ((size_t)(b * x.H + y) * x.W + xx) * a.co + o);
      s_e[p][4 * (q & 7) + 0] = v.x;
      s_e[p][4 * (q & 7) + 1] = v.y;
      s_e[p][4 * (q & 7) + 2] = v.z;
      s_e[p][4 * (q & 7) + 3] = v.w;
    }
    for (int q = tid; q < (kWTH + 2) * kHW * 4; q += 256) {
      const int p = q >> 2, c = c0 + 4 * (q & 3);
      const int y = y0 + p / kHW - 1, xx = x0 + p % kHW - 1;
      f4 v = f4{0.f, 0.f, 0.f, 0.f};
      if (y >= 0 && y < x.H && xx >= 0 && xx < x.W && c < a.ci) v = halo_value<MODE>(halo_load<MODE>(x, b, y, xx, c), true);
      s_x[p][4 * (q & 3) + 0] = v.x;
      s_x[p][4 * (q & 3) + 1] = v.y;
      s_x[p][4 * (q & 3) + 2] = v.z;
      s_x[p][4 * (q & 3) + 3] = v.w;
    }
    __syncthreads();
#pragma unroll 1
    for (int ks = 0; ks < 8; ++ks) {
      const int row = 2 * wave + (ks >> 2), col = 4 * (ks & 3) + g;
      const float a0 = s_e[row * kTW + col][li], a1 = s_e[row * kTW + col][16 + li];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const float bv = s_x[(row + tap / 3) * kHW + col + tap % 3][li];
        acc[0][tap] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv, acc[0][tap], 0, 0, 0);
        acc[1][tap] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv, acc[1][tap], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const size_t part = (size_t)blockIdx.x * 4 + wave;
#pragma unroll
  for (int of = 0; of < 2; ++of)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int o = o0 + of * 16 + 4 * g + rr, c = c0 + li;
        a.partial[((part * co_pad + o) * a.ci_pad16 + c) * 9 + tap] = acc[of][tap][rr];
      }
}

__global__ __launch_bounds__(256) void wgrad_reduce(const float* __restrict__ partial, int n_partials, int co, int ci,
                                                     int co_pad, int ci_pad16, float* __restrict__ grad_w) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)co * ci * 9) return;
  const int tap = i % 9, c = (i / 9) % ci, o = i / (9 * ci);
  const size_t stride = (size_t)co_pad * ci_pad16 * 9, base = ((size_t)o * ci_pad16 + c) * 9 + tap;
  float s = 0.0f;
  for (int p = 0; p < n_partials; ++p) s += partial[p * stride + base];
  grad_w[i] = s;
}

template <int CK, int MODE, int TH>
hipError_t launch_th(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  dim3 grid((a.W + kTW - 1) / kTW, ((a.H + TH - 1) / TH) * a.B, a.n_tiles * a.splits);
  if constexpr (CK == 16 && MODE == G_PLAIN) {
    if (head) {
      hipLaunchKernelGGL((conv3x3_f32<CK, MODE, TH, true>), grid, dim3(256), 0, s, a, *head);
      return hipGetLastError();
    }
  }
  if (head) return hipErrorInvalidValue;
  hipLaunchKernelGGL((conv3x3_f32<CK, MODE, TH, false>), grid, dim3(256), 0, s, a, HeadFuse{});
  return hipGetLastError();
}
template <int CK, int MODE>
hipError_t launch_tile(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if (CK == 16 && a.th == 4) return launch_th<CK, MODE, 4>(a, s, head);
  return launch_th<CK, MODE, 8>(a, s, head);
}

}  // namespace

hipError_t launch_conv3x3_f32(int mode, int ck, const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if (head && (a.n_tiles != 1 || a.splits != 1 || a.co > kBN || !a.relu)) return hipErrorInvalidValue;
  if (mode == G_GUIDE && ck == 4) return launch_tile<4, G_GUIDE>(a, s, head);
  if (ck != 16) return hipErrorInvalidValue;
  switch (mode) {
    case G_FIRST:
      if (!a.w0 || !a.b0) return hipErrorInvalidValue;
      return launch_tile<16, G_FIRST>(a, s, head);
    case G_PLAIN: return launch_tile<16, G_PLAIN>(a, s, head);
    case G_POOL: return launch_tile<16, G_POOL>(a, s, head);
    case G_CONCAT_UP: return launch_tile<16, G_CONCAT_UP>(a, s, head);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_splitk_reduce(const ConvArgs& a, int out_type, hipStream_t s) {
  if (a.co % 4) return hipErrorInvalidValue;
  const long total4 = (long)a.B * a.H * a.W * a.co / 4;
  const dim3 grid((unsigned)((total4 + 255) / 256));
  switch (a.splits) {
    case 2: hipLaunchKernelGGL(splitk_reduce<2>, grid, dim3(256), 0, s, a, out_type, total4); break;
    case 4: hipLaunchKernelGGL(splitk_reduce<4>, grid, dim3(256), 0, s, a, out_type, total4); break;
    case 8: hipLaunchKernelGGL(splitk_reduce<8>, grid, dim3(256), 0, s, a, out_type, total4); break;
    case 16: hipLaunchKernelGGL(splitk_reduce<16>, grid, dim3(256), 0, s, a, out_type, total4); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wgrad3x3(int mode, const WgradArgs& a, int* n_partials, hipStream_t s) {
  const int tiles = a.x.B * ((a.x.W + kTW - 1) / kTW) * ((a.x.H + kWTH - 1) / kWTH);
  const int groups = (tiles + a.tiles_per_group - 1) / a.tiles_per_group;
  dim3 grid(groups, (a.co + kBN - 1) / kBN, a.ci_pad16 / 16);
  *n_partials = groups * 4;
  switch (mode) {
    case G_GUIDE: hipLaunchKernelGGL(wgrad3x3_f32<G_GUIDE>, grid, dim3(256), 0, s, a); break;
    case G_PLAIN: hipLaunchKernelGGL(wgrad3x3_f32<G_PLAIN>, grid, dim3(256), 0, s, a); break;
    case G_POOL: hipLaunchKernelGGL(wgrad3x3_f32<G_POOL>, grid, dim3(256), 0, s, a); break;
    case G_CONCAT_UP: hipLaunchKernelGGL(wgrad3x3_f32<G_CONCAT_UP>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const float* partial, int n_partials, int co, int ci, int co_pad, int ci_pad16,
                               float* grad_w, hipStream_t s) {
  const long n = (long)co * ci * 9;
  hipLaunchKernelGGL(wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, s, partial, n_partials, co, ci, co_pad,
                     ci_pad16, grad_w);
  return hipGetLastError();
}

hipError_t launch_head(const HeadArgs& a, hipStream_t s, const CompositeArgs* comp) {
  if (a.C > 256 || (a.C & 3) || a.in_type < 0 || a.in_type > 2) return hipErrorInvalidValue;
  const dim3 grid((a.P + 255) / 256);
  const CompositeArgs c = comp ? *comp : CompositeArgs{};
  if (comp) {
    if (a.in_type == 0) hipLaunchKernelGGL((head_kernel<0, true>), grid, dim3(256), 0, s, a, c);
    if (a.in_type == 1) hipLaunchKernelGGL((head_kernel<1, true>), grid, dim3(256), 0, s, a, c);
    if (a.in_type == 2) hipLaunchKernelGGL((head_kernel<2, true>), grid, dim3(256), 0, s, a, c);
  } else {
    if (a.in_type == 0) hipLaunchKernelGGL((head_kernel<0, false>), grid, dim3(256), 0, s, a, c);
    if (a.in_type == 1) hipLaunchKernelGGL((head_kernel<1, false>), grid, dim3(256), 0, s, a, c);
    if (a.in_type == 2) hipLaunchKernelGGL((head_kernel<2, false>), grid, dim3(256), 0, s, a, c);
  }
  return hipGetLastError();
}

hipError_t launch_composite(const CompositeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(composite_kernel, dim3((a.P + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_composite_batch(const CompositeBatchArgs& a, hipStream_t s) {
  const long n = (long)a.P * a.B;
  hipLaunchKernelGGL(composite_batch_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lnm
