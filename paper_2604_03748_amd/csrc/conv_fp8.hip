// U-Net 3x3 convolutions (Section 4.3) in FP8 e4m3 (OCP) on the gfx950
// matrix cores (v_mfma_f32_16x16x32_fp8_fp8, fp32 accumulation).
//
// Quantisation: weights per output channel, q_w = rne(W / s_w[o]) with
// s_w[o] = max|W[o]| / 448; activations per stored tensor, q = rne(y / s_t)
// saturated to 448.  A layer computes y = s_in s_w[o] sum q_in q_w + b,
// applies ReLU and stores rne(y / s_out) for its consumers.  The two inputs
// of a decoder concatenation share one scale, so the K-sum factors.
//
// Tiling as in the bf16 kernel (TH x 16 pixels x 32 output channels per
// workgroup, 32-channel input chunks staged in LDS, lane group g supplying
// channels 8g..8g+7 of a chunk to both operands with one 8-byte read).  The
// 3-channel input layer runs in bf16 (27 taps x channels in one K step) and
// writes fp8.
#include "internal.h"
#include "first_layer.h"
#include "head.h"

namespace lnm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTW = 16;
constexpr int kHW = kTW + 2;
constexpr int kCK = 32;      // input channels per chunk (bytes per pixel row)
constexpr int kRow = 40;     // LDS bytes per halo pixel / weight row (32 + 8)
constexpr int kRowBf = 40;   // bf16 elements per weight row of the guide layer

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// fp32 -> e4m3 byte, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint32_t f2fp8(float v) {
  v = fminf(fmaxf(v, -448.0f), 448.0f);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xffu;
}

__device__ __forceinline__ uint32_t max_u8x4(uint32_t a, uint32_t b) {
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t x = (a >> (8 * k)) & 0xffu, y = (b >> (8 * k)) & 0xffu;
    r |= (x > y ? x : y) << (8 * k);
  }
  return r;
}

// Raw loads of eight channels [c, c+8) of the virtual input at (y, x) as 8
// e4m3 bytes, all three clamped to valid positions; the pooled mode keeps
// its four source pixels.  Combined and masked when written to LDS, so a
// chunk's loads are in flight together.  Stored activations are ReLU outputs
// (non-negative, +0 encoded as 0), whose e4m3 encodings order like unsigned
// bytes, so max-pooling compares bytes.
template <int MODE>
struct Halo {
  uint2 v[MODE == G_POOL ? 4 : 1];
};

template <int MODE>
__device__ __forceinline__ Halo<MODE> halo_load(const ConvArgs& a, int b, int y, int x, int c) {
  const uint8_t* s0 = static_cast<const uint8_t*>(a.src0);
  Halo<MODE> h;
  if constexpr (MODE == G_FIRST) {
    h.v[0] = make_uint2(0u, 0u);
  } else if constexpr (MODE == G_PLAIN) {
    h.v[0] = *reinterpret_cast<const uint2*>(s0 + ((size_t)(b * a.H + y) * a.W + x) * a.c0 + c);
  } else if constexpr (MODE == G_POOL) {
    const size_t W2 = 2 * (size_t)a.W, c0 = (size_t)a.c0;
    const uint8_t* p = s0 + ((size_t)(b * 2 * a.H + 2 * y) * W2 + 2 * x) * c0 + c;
    h.v[0] = *reinterpret_cast<const uint2*>(p);
    h.v[1] = *reinterpret_cast<const uint2*>(p + c0);
    h.v[2] = *reinterpret_cast<const uint2*>(p + W2 * c0);
    h.v[3] = *reinterpret_cast<const uint2*>(p + W2 * c0 + c0);
  } else {  // G_CONCAT_UP
    const int Hl = a.H >> 1, Wl = a.W >> 1;
    const uint8_t* skip = s0 + ((size_t)(b * a.H + y) * a.W + x) * a.c0 + c;
    const uint8_t* up = static_cast<const uint8_t*>(a.src1) +
                        ((size_t)(b * Hl + (y >> 1)) * Wl + (x >> 1)) * a.c1 + max(c - a.c0, 0);
    h.v[0] = *reinterpret_cast<const uint2*>(c < a.c0 ? skip : up);
  }
  return h;
}

template <int MODE>
__device__ __forceinline__ uint2 halo_value(const Halo<MODE>& h, bool ok) {
  uint2 r = h.v[0];
  if constexpr (MODE == G_POOL) {
    r.x = max_u8x4(max_u8x4(h.v[0].x, h.v[1].x), max_u8x4(h.v[2].x, h.v[3].x));
    r.y = max_u8x4(max_u8x4(h.v[0].y, h.v[1].y), max_u8x4(h.v[2].y, h.v[3].y));
  }
  return ok ? r : make_uint2(0, 0);
}

// y = scale[o] * acc + bias (scale = s_in s_w[o], or 1 for the bf16 layer),
// ReLU, stored as e4m3 of y * out_inv_scale (bf16 of y when the consumer is
// the network's bf16 last layer).
template <int TH>
__device__ __forceinline__ void store_fp8(const ConvArgs& a, const f4 (&acc)[TH / 4][2], int b, int y0, int x0,
                                          int wrow, int g, int li, bool scaled, int nt, int ks) {
  uint8_t* out = static_cast<uint8_t*>(a.out);
#pragma unroll
  for (int nf = 0; nf < 2; ++nf) {
    const int n = nt * kBN + nf * 16 + li;
    if (n >= a.co) continue;
    const float bias = a.bias[n];
    const float sc = scaled ? a.in_scale * a.w_scale[n] : 1.0f;
#pragma unroll
    for (int mf = 0; mf < TH / 4; ++mf) {
      const int y = y0 + wrow + mf;
      if (y >= a.H) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = x0 + 4 * g + r;
        if (x >= a.W) continue;
        const size_t pix = (size_t)(b * a.H + y) * a.W + x;
        if (a.splits > 1) {
          a.partial[((size_t)ks * a.B * a.H * a.W + pix) * a.co + n] = acc[mf][nf][r];
          continue;
        }
        float v = sc * acc[mf][nf][r] + bias;
        if (a.out_bf16) {  // for a bf16 consumer: unscaled
          static_cast<uint16_t*>(a.out)[pix * a.co + n] = f2bf(fmaxf(v, 0.0f));
          continue;
        }
        v = v > 0.0f ? v * a.out_inv_scale : 0.0f;
        out[pix * a.co + n] = (uint8_t)f2fp8(v);
      }
    }
  }
}

template <int MODE, int TH, bool HEAD>
__global__ __launch_bounds__(256) void conv3x3_fp8(ConvArgs a, HeadFuse hf) {
  constexpr int MF = TH / 4;
  // two LDS buffers: the next chunk is fetched into registers while the
  // matrix cores work on the current one
  __shared__ __attribute__((aligned(16))) uint8_t s_in[2][(TH + 2) * kHW * kRow];
  __shared__ __attribute__((aligned(16))) uint8_t s_w[2][9 * kBN * kRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_y = (a.H + TH - 1) / TH;
  const int b = blockIdx.y / tiles_y;
  const int y0 = (blockIdx.y - b * tiles_y) * TH, x0 = blockIdx.x * kTW;
  const int g = lane >> 4, li = lane & 15, wrow = wave * MF;
  const int nt = blockIdx.z % a.n_tiles, ks = blockIdx.z / a.n_tiles;
  const int nchunks = a.ci_pad / kCK;
  const int ch_lo = ks * nchunks / a.splits, ch_hi = (ks + 1) * nchunks / a.splits;
  const int ci = a.c0 + a.c1;
  const uint8_t* wblk = static_cast<const uint8_t*>(a.w) + (size_t)nt * nchunks * 9 * kBN * kCK;

  f4 acc[MF][2];
#pragma unroll
  for (int mf = 0; mf < MF; ++mf) acc[mf][0] = acc[mf][1] = f4{0.f, 0.f, 0.f, 0.f};

  // G_FIRST: the first layer's outputs on the halo, formed from the staged
  // guide as the first layer's own kernel forms them (the same bf16
  // operands in the same K slots, bias, ReLU, e4m3 of the value times the
  // first layer's output scale), so the result is the same bit for bit
  using FT = first::Tile<TH>;
  __shared__ f4 s_g[MODE == G_FIRST ? FT::NG : 1];
  uint8_t fr[MODE == G_FIRST ? 8 * FT::BPW : 1];
  auto first_layer = [&](int ch) {
    first::first_layer_bf16<TH>(a, ch, s_g, [&](int bb, int nf, int r, float v) {
      fr[8 * bb + 4 * nf + r] = (uint8_t)f2fp8(v > 0.0f ? v * a.w0_out_inv : 0.0f);
    });
  };

  constexpr int NQ = (TH + 2) * kHW * (kCK / 8), NW = 9 * kBN * kCK / 16;
  constexpr int RQ = (NQ + 255) / 256, RW = (NW + 255) / 256;
  Halo<MODE> rq[RQ];
  uint4 rw[RW];
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
    const uint8_t* wsrc = wblk + (size_t)ch * 9 * kBN * kCK;
#pragma unroll
    for (int r = 0; r < RW; ++r) rw[r] = *reinterpret_cast<const uint4*>(wsrc + 16 * min(tid + 256 * r, NW - 1));
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
          for (int nf = 0; nf < 2; ++nf) s_in[buf][q * kRow + nf * 16 + li] = in ? fr[8 * bb + 4 * nf + r] : 0;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < (MODE == G_FIRST ? 0 : RQ); ++r) {
      const int q = tid + 256 * r;
      if (q < NQ) *reinterpret_cast<uint2*>(&s_in[buf][(q >> 2) * kRow + 8 * (q & 3)]) = halo_value<MODE>(rq[r], (ok >> r) & 1u);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int q = tid + 256 * r;
      if (q < NW) {
        uint8_t* dst = &s_w[buf][(q >> 1) * kRow + 16 * (q & 1)];
        *reinterpret_cast<uint2*>(dst) = make_uint2(rw[r].x, rw[r].y);
        *reinterpret_cast<uint2*>(dst + 8) = make_uint2(rw[r].z, rw[r].w);
      }
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
    const int cur = (ch - ch_lo) & 1;
    const bool more = ch + 1 < ch_hi;
    if (more) fetch(ch + 1);
    const uint8_t* si = s_in[cur];
    const uint8_t* sw = s_w[cur];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap - 3 * (tap / 3);
      long av[MF], bv[2];
#pragma unroll
      for (int mf = 0; mf < MF; ++mf)
        av[mf] = *reinterpret_cast<const long*>(&si[((wrow + mf + dy) * kHW + li + dx) * kRow + 8 * g]);
#pragma unroll
      for (int nf = 0; nf < 2; ++nf)
        bv[nf] = *reinterpret_cast<const long*>(&sw[(tap * kBN + nf * 16 + li) * kRow + 8 * g]);
#pragma unroll
      for (int mf = 0; mf < MF; ++mf)
#pragma unroll
        for (int nf = 0; nf < 2; ++nf)
          acc[mf][nf] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[mf], bv[nf], acc[mf][nf], 0, 0, 0);
    }
    if (more) commit(cur ^ 1);
    __syncthreads();
  }
  if constexpr (HEAD) {
    // head epilogue: the activations as they would be stored (e4m3 of the
    // scaled bias + ReLU, read back with the tensor's scale) and the head
    // weights in LDS (both weight buffers are free after the last chunk's
    // barrier), then one thread per pixel
    static_assert((TH * kTW * 33 + 6 * kBN) * 4 <= 2 * 9 * kBN * kRow, "head tile must fit the weight buffers");
    float* sh = reinterpret_cast<float*>(&s_w[0][0]);
    float* shw = sh + TH * kTW * 33;
    head_weights(hf, a.co, shw);
#pragma unroll
    for (int mf = 0; mf < MF; ++mf)
#pragma unroll
      for (int nf = 0; nf < 2; ++nf) {
        const int n = nf * 16 + li;
        const float bias = n < a.co ? a.bias[n] : 0.0f, sc = n < a.co ? a.in_scale * a.w_scale[n] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = sc * acc[mf][nf][r] + bias;
          v = v > 0.0f ? v * a.out_inv_scale : 0.0f;
          sh[((wrow + mf) * kTW + 4 * g + r) * 33 + n] = __builtin_amdgcn_cvt_f32_fp8((int)f2fp8(v), 0) * hf.in_scale;
        }
      }
    __syncthreads();
    head_finish<TH>(hf, sh, shw, b, a.H, a.W, y0, x0);
    return;
  }
  store_fp8<TH>(a, acc, b, y0, x0, wrow, g, li, true, nt, ks);
}

// The 3-channel input layer in bf16 (as in the bf16 network), fp8 output.
template <int TH>
__global__ __launch_bounds__(256) void conv3x3_guide_to_fp8(ConvArgs a) {
  constexpr int MF = TH / 4;
  __shared__ __attribute__((aligned(16))) float s_in[(TH + 2) * kHW * 4];
  __shared__ __attribute__((aligned(16))) uint16_t s_w[kBN * kRowBf];
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
  const uint16_t* wsrc = static_cast<const uint16_t*>(a.w) + (size_t)blockIdx.z * kBN * 32;
  for (int q = tid; q < kBN * 32 / 8; q += 256) {
    const int c8 = q & 3, row = q >> 2;
    *reinterpret_cast<uint4*>(&s_w[row * kRowBf + 8 * c8]) = *reinterpret_cast<const uint4*>(wsrc + 8 * q);
  }
  __syncthreads();
  f4 acc[MF][2];
  bf16x8 bv[2];
#pragma unroll
  for (int nf = 0; nf < 2; ++nf) bv[nf] = *reinterpret_cast<const bf16x8*>(&s_w[(nf * 16 + li) * kRowBf + 8 * g]);
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
  store_fp8<TH>(a, acc, b, y0, x0, wrow, g, li, false, blockIdx.z, 0);
}

// Per-block maximum of |x| over a fixed range, then the maximum of those.
__global__ __launch_bounds__(256) void amax_partial(const float* __restrict__ x, long n, float* __restrict__ part) {
  __shared__ float sh[256];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * per, hi = min(n, lo + per);
  float m = 0.0f;
  for (long i = lo + threadIdx.x; i < hi; i += 256) m = fmaxf(m, fabsf(x[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void amax_finish(const float* __restrict__ part, int n, float* __restrict__ out) {
  __shared__ float sh[256];
  float m = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) m = fmaxf(m, part[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

template <int MODE, int TH>
hipError_t launch_th(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  dim3 grid((a.W + kTW - 1) / kTW, ((a.H + TH - 1) / TH) * a.B, a.n_tiles * a.splits);
  if constexpr (MODE == G_GUIDE) {
    if (head) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conv3x3_guide_to_fp8<TH>), grid, dim3(256), 0, s, a);
  } else if constexpr (MODE == G_PLAIN) {
    if (head)
      hipLaunchKernelGGL((conv3x3_fp8<MODE, TH, true>), grid, dim3(256), 0, s, a, *head);
    else
      hipLaunchKernelGGL((conv3x3_fp8<MODE, TH, false>), grid, dim3(256), 0, s, a, HeadFuse{});
  } else {
    if (head) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conv3x3_fp8<MODE, TH, false>), grid, dim3(256), 0, s, a, HeadFuse{});
  }
  return hipGetLastError();
}
// 8-row tiles, or 4-row tiles when the layer asks for them (not the input layer)
template <int MODE>
hipError_t launch_tile(const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if (MODE != G_GUIDE && a.th == 4) return launch_th<MODE == G_GUIDE ? G_PLAIN : MODE, 4>(a, s, head);
  return launch_th<MODE, 8>(a, s, head);
}

}  // namespace

hipError_t launch_conv3x3_fp8(int mode, const ConvArgs& a, hipStream_t s, const HeadFuse* head) {
  if (head && (a.n_tiles != 1 || a.splits != 1 || a.co > kBN || !a.w_scale)) return hipErrorInvalidValue;
  switch (mode) {
    case G_FIRST:
      if (!a.w0 || !a.b0 || head) return hipErrorInvalidValue;
      return launch_tile<G_FIRST>(a, s, head);
    case G_GUIDE: return launch_tile<G_GUIDE>(a, s, head);
    case G_PLAIN: return launch_tile<G_PLAIN>(a, s, head);
    case G_POOL: return launch_tile<G_POOL>(a, s, head);
    case G_CONCAT_UP: return launch_tile<G_CONCAT_UP>(a, s, head);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_amax(const float* x, long n, float* partial, float* out, hipStream_t s) {
  hipLaunchKernelGGL(amax_partial, dim3(kAmaxBlocks), dim3(256), 0, s, x, n, partial);
  hipLaunchKernelGGL(amax_finish, dim3(1), dim3(256), 0, s, partial, kAmaxBlocks, out);
  return hipGetLastError();
}

}  // namespace lnm
