// Channel adapters on the U-Net decoder output (Section 4.3): four NAFBlocks
// (Chen et al. 2022), one per output group (front/back, left/right,
// up/down, alpha/emissive), each followed by a 1x1 head to its two channels
// and a sigmoid.  fp32 arithmetic.
//
// Four kernels, because the block's channel attention needs the mean of the
// gated features over the whole image between its two halves:
//   adapt_expand    lane per pixel: layer norm 1, 1x1 conv c -> 2c for all
//                   four groups -> u[g][2c][P] (channel planes, so lanes write
//                   coalesced rows);
//   adapt_dw_gate   lane per (pixel, group, channel pair): 3x3 depthwise conv
//                   of channels ch and ch + c, their product -> v[g][c][P],
//                   and per 256-pixel block partial sums for the attention;
//   adapt_attend    workgroup per (image, group): the image mean of v (partial
//                   sums added in a fixed order) and the attention's 1x1 conv
//                   -> s[b][g][c];
//   adapt_out       lane per pixel, one group at a time: v * s, 1x1 conv,
//                   residual with beta, layer norm 2, 1x1 c -> 2c, gate,
//                   1x1 c -> c, residual with gamma, head, sigmoid.
// Weights are staged in LDS and read as broadcasts; every lane keeps its
// pixel's channels in registers (c is a template parameter).
#include <cmath>

#include "internal.h"

namespace lnm {
namespace {

// offsets of one adapter's tensors (parameter-file order) for width C
template <int C>
struct Off {
  static constexpr int ln1w = 0, ln1b = C, c1w = 2 * C, c1b = c1w + 2 * C * C, dww = c1b + 2 * C, dwb = dww + 18 * C,
                       scaw = dwb + 2 * C, scab = scaw + C * C, c3w = scab + C, c3b = c3w + C * C, beta = c3b + C,
                       ln2w = beta + C, ln2b = ln2w + C, c4w = ln2b + C, c4b = c4w + 2 * C * C, c5w = c4b + 2 * C,
                       c5b = c5w + C * C, gamma = c5b + C, hw = gamma + C, hb = hw + 2 * C, total = hb + 2;
};

__device__ __forceinline__ float bf16f(uint32_t h) { return __uint_as_float(h << 16); }

// feature channel i of pixel p as fp32 (IN: 0 fp32, 1 bf16, 2 e4m3 x scale)
template <int C, int IN>
__device__ __forceinline__ void load_feat(const AdapterArgs& a, size_t p, float (&x)[C]) {
  if constexpr (IN == 0) {
    const float4* s = reinterpret_cast<const float4*>(static_cast<const float*>(a.feat) + p * C);
#pragma unroll
    for (int i = 0; i < C / 4; ++i) {
      const float4 v = s[i];
      x[4 * i] = v.x;
      x[4 * i + 1] = v.y;
      x[4 * i + 2] = v.z;
      x[4 * i + 3] = v.w;
    }
  } else if constexpr (IN == 1) {
    const uint2* s = reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.feat) + p * C);
#pragma unroll
    for (int i = 0; i < C / 4; ++i) {
      const uint2 q = s[i];
      x[4 * i] = bf16f(q.x & 0xffffu);
      x[4 * i + 1] = bf16f(q.x >> 16);
      x[4 * i + 2] = bf16f(q.y & 0xffffu);
      x[4 * i + 3] = bf16f(q.y >> 16);
    }
  } else {
    const int* s = reinterpret_cast<const int*>(static_cast<const uint8_t*>(a.feat) + p * C);
#pragma unroll
    for (int i = 0; i < C / 4; ++i) {
      const int q = s[i];
      x[4 * i] = __builtin_amdgcn_cvt_f32_fp8(q, 0) * a.feat_scale;
      x[4 * i + 1] = __builtin_amdgcn_cvt_f32_fp8(q, 1) * a.feat_scale;
      x[4 * i + 2] = __builtin_amdgcn_cvt_f32_fp8(q, 2) * a.feat_scale;
      x[4 * i + 3] = __builtin_amdgcn_cvt_f32_fp8(q, 3) * a.feat_scale;
    }
  }
}

// the same into the LDS column [channel][lane]
template <int C, int IN, int T>
__device__ __forceinline__ void load_feat(const AdapterArgs& a, size_t p, float (&col)[C][T], int lane) {
  float x[C];
  load_feat<C, IN>(a, p, x);
#pragma unroll
  for (int i = 0; i < C; ++i) col[i][lane] = x[i];
}

// (x - mean) / sqrt(var + 1e-6) over the C channels, biased variance
template <int C>
__device__ __forceinline__ void normalise(float (&x)[C]) {
  float mu = 0.0f;
#pragma unroll
  for (int i = 0; i < C; ++i) mu += x[i];
  mu *= 1.0f / (float)C;
  float var = 0.0f;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    x[i] -= mu;
    var += x[i] * x[i];
  }
  const float r = 1.0f / sqrtf(var * (1.0f / (float)C) + 1e-6f);
#pragma unroll
  for (int i = 0; i < C; ++i) x[i] *= r;
}

// out = b + W x for one output row o: W row-major [o][C] in LDS
template <int C>
__device__ __forceinline__ float row_dot(const float* __restrict__ w, float b, const float (&x)[C]) {
  float s = b;
#pragma unroll
  for (int i = 0; i < C; i += 4) {
    const float4 q = *reinterpret_cast<const float4*>(w + i);
    s += q.x * x[i] + q.y * x[i + 1] + q.z * x[i + 2] + q.w * x[i + 3];
  }
  return s;
}

template <int C, int IN>
__global__ __launch_bounds__(256) void adapt_expand(AdapterArgs a) {
  using O = Off<C>;
  __shared__ __attribute__((aligned(16))) float sw[2 * C * C + 4 * C];  // conv1 W, conv1 b, ln1 w, ln1 b
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = p < a.P;
  float xh[C], t[C];
  if (live) {
    load_feat<C, IN>(a, p, xh);
    normalise<C>(xh);
  }
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const float* P = a.prm + (size_t)g * O::total;
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * C * C; q += 256) sw[q] = P[O::c1w + q];
    for (int q = threadIdx.x; q < 2 * C; q += 256) sw[2 * C * C + q] = P[O::c1b + q];
    for (int q = threadIdx.x; q < C; q += 256) {
      sw[2 * C * C + 2 * C + q] = P[O::ln1w + q];
      sw[2 * C * C + 3 * C + q] = P[O::ln1b + q];
    }
    __syncthreads();
    if (!live) continue;
#pragma unroll
    for (int i = 0; i < C; ++i) t[i] = xh[i] * sw[2 * C * C + 2 * C + i] + sw[2 * C * C + 3 * C + i];
    float* u = a.u + (size_t)g * 2 * C * a.P + p;
#pragma unroll 4
    for (int o = 0; o < 2 * C; ++o) u[(size_t)o * a.P] = row_dot<C>(sw + o * C, sw[2 * C * C + o], t);
  }
}

// grid: (ceil(HW / 256), 4 C, B); block (bx, g * C + ch, b)
template <int C>
__global__ __launch_bounds__(256) void adapt_dw_gate(AdapterArgs a) {
  using O = Off<C>;
  __shared__ float red[4];
  const int HW = a.H * a.W;
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y / C, ch = blockIdx.y - g * C, b = blockIdx.z;
  const float* P = a.prm + (size_t)g * O::total;
  float v = 0.0f;
  if (q < HW) {
    const int y = q / a.W, x = q - y * a.W;
    const size_t base = (size_t)b * HW;
    const float* u1 = a.u + ((size_t)g * 2 * C + ch) * a.P + base;
    const float* u2 = u1 + (size_t)C * a.P;
    float s1 = P[O::dwb + ch], s2 = P[O::dwb + C + ch];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int yy = y + dy - 1;
      if (yy < 0 || yy >= a.H) continue;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int xx = x + dx - 1;
        if (xx < 0 || xx >= a.W) continue;
        const int nb = yy * a.W + xx;
        s1 += P[O::dww + ch * 9 + dy * 3 + dx] * u1[nb];
        s2 += P[O::dww + (C + ch) * 9 + dy * 3 + dx] * u2[nb];
      }
    }
    v = s1 * s2;
    a.v[((size_t)g * C + ch) * a.P + base + q] = v;
  }
  // block sum of v in a fixed order: a butterfly within each wavefront, then
  // the four wavefront sums in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    a.part[(((size_t)b * 4 + g) * C + ch) * a.n_blk + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// grid: (4, B); image mean of v per channel (thread (slice, ch) sums the
// block partials slice, slice + S, ... in order, then the S slices are added
// in order), then the attention's 1x1 conv
template <int C>
__global__ __launch_bounds__(256) void adapt_attend(AdapterArgs a) {
  using O = Off<C>;
  constexpr int S = 256 / C;
  __shared__ float red[S][C];
  __shared__ float pooled[C];
  const int g = blockIdx.x, b = blockIdx.y;
  const int ch = threadIdx.x % C, slice = threadIdx.x / C;
  const float* P = a.prm + (size_t)g * O::total;
  if (slice < S) {
    const float* src = a.part + (((size_t)b * 4 + g) * C + ch) * a.n_blk;
    float s = 0.0f;
    for (int k = slice; k < a.n_blk; k += S) s += src[k];
    red[slice][ch] = s;
  }
  __syncthreads();
  if (threadIdx.x < C) {
    float s = 0.0f;
    for (int q = 0; q < S; ++q) s += red[q][threadIdx.x];
    pooled[threadIdx.x] = s / (float)(a.H * a.W);
  }
  __syncthreads();
  if (threadIdx.x < C) {
    float s = P[O::scab + threadIdx.x];
    for (int i = 0; i < C; ++i) s += P[O::scaw + threadIdx.x * C + i] * pooled[i];
    a.sca[((size_t)b * 4 + g) * C + threadIdx.x] = s;
  }
}

// output channels of each group: lightmaps (+Z, -Z), (+X, -X), (+Y, -Y); extra (alpha, emissive)
__constant__ int kDst[4][2] = {{4, 5}, {0, 1}, {2, 3}, {-1, -2}};

// Outputs of a dense layer are produced one channel at a time (a runtime
// loop, so code size and registers stay bounded) into per-lane LDS columns
// [channel][lane]; inputs are loaded back into registers for the next layer.
constexpr int kOutThreads = 128;

template <int C, int IN>
__global__ __launch_bounds__(kOutThreads) void adapt_out(AdapterArgs a) {
  using O = Off<C>;
  // conv3 W, conv4 W, conv5 W, head W, then the vectors
  constexpr int W3 = 0, W4 = C * C, W5 = 3 * C * C, WH = 4 * C * C, V = WH + 2 * C;
  constexpr int B3 = V, BETA = V + C, L2W = V + 2 * C, L2B = V + 3 * C, B4 = V + 4 * C, B5 = V + 6 * C,
                GAM = V + 7 * C, HB = V + 8 * C, NW = V + 8 * C + 4;
  __shared__ __attribute__((aligned(16))) float sw[NW];
  __shared__ float ys[C][kOutThreads];  // y = in + beta conv3(.), then + gamma conv5(.)
  __shared__ float hs[C][kOutThreads];  // gated conv4 output
  const int tid = threadIdx.x;
  const size_t p = (size_t)blockIdx.x * kOutThreads + tid;
  const bool live = p < a.P;
  const int b = live ? (int)(p / ((size_t)a.H * a.W)) : 0;
  float t[C];
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const float* P = a.prm + (size_t)g * O::total;
    __syncthreads();
    for (int q = tid; q < C * C; q += kOutThreads) {
      sw[W3 + q] = P[O::c3w + q];
      sw[W5 + q] = P[O::c5w + q];
    }
    for (int q = tid; q < 2 * C * C; q += kOutThreads) sw[W4 + q] = P[O::c4w + q];
    for (int q = tid; q < 2 * C; q += kOutThreads) {
      sw[WH + q] = P[O::hw + q];
      sw[B4 + q] = P[O::c4b + q];
    }
    for (int q = tid; q < C; q += kOutThreads) {
      sw[B3 + q] = P[O::c3b + q];
      sw[BETA + q] = P[O::beta + q];
      sw[L2W + q] = P[O::ln2w + q];
      sw[L2B + q] = P[O::ln2b + q];
      sw[B5 + q] = P[O::c5b + q];
      sw[GAM + q] = P[O::gamma + q];
    }
    if (tid < 2) sw[HB + tid] = P[O::hb + tid];
    __syncthreads();
    if (!live) continue;  // no barrier below this point
    // attended gate output
    const float* s = a.sca + ((size_t)b * 4 + g) * C;
#pragma unroll
    for (int i = 0; i < C; ++i) t[i] = a.v[((size_t)g * C + i) * a.P + p] * s[i];
    // y = in + beta * conv3(t)
    load_feat<C, IN>(a, p, ys, tid);
#pragma unroll 2
    for (int o = 0; o < C; ++o) ys[o][tid] += sw[BETA + o] * row_dot<C>(sw + W3 + o * C, sw[B3 + o], t);
    // t = LN2(y)
#pragma unroll
    for (int i = 0; i < C; ++i) t[i] = ys[i][tid];
    normalise<C>(t);
#pragma unroll
    for (int i = 0; i < C; ++i) t[i] = t[i] * sw[L2W + i] + sw[L2B + i];
    // h = gate(conv4(t))
#pragma unroll 2
    for (int o = 0; o < C; ++o)
      hs[o][tid] =
          row_dot<C>(sw + W4 + o * C, sw[B4 + o], t) * row_dot<C>(sw + W4 + (C + o) * C, sw[B4 + C + o], t);
    // y += gamma * conv5(h)
#pragma unroll
    for (int i = 0; i < C; ++i) t[i] = hs[i][tid];
#pragma unroll 2
    for (int o = 0; o < C; ++o) ys[o][tid] += sw[GAM + o] * row_dot<C>(sw + W5 + o * C, sw[B5 + o], t);
#pragma unroll
    for (int i = 0; i < C; ++i) t[i] = ys[i][tid];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float z = row_dot<C>(sw + WH + k * C, sw[HB + k], t);
      const float sig = 1.0f / (1.0f + expf(-z));
      const int d = kDst[g][k];
      if (d >= 0)
        a.lm[p * 6 + d] = sig;
      else if (a.extra)
        a.extra[p * 2 + (-1 - d)] = sig;
    }
  }
}

template <int C>
hipError_t launch_c(const AdapterArgs& a, int in_type, hipStream_t s) {
  const unsigned blk = (unsigned)((a.P + 255) / 256);
  switch (in_type) {
    case 0: hipLaunchKernelGGL((adapt_expand<C, 0>), dim3(blk), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((adapt_expand<C, 1>), dim3(blk), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((adapt_expand<C, 2>), dim3(blk), dim3(256), 0, s, a); break;
  }
  hipLaunchKernelGGL(adapt_dw_gate<C>, dim3(a.n_blk, 4 * C, a.B), dim3(256), 0, s, a);
  hipLaunchKernelGGL(adapt_attend<C>, dim3(4, a.B), dim3(256), 0, s, a);
  const unsigned oblk = (unsigned)((a.P + kOutThreads - 1) / kOutThreads);
  switch (in_type) {
    case 0: hipLaunchKernelGGL((adapt_out<C, 0>), dim3(oblk), dim3(kOutThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL((adapt_out<C, 1>), dim3(oblk), dim3(kOutThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((adapt_out<C, 2>), dim3(oblk), dim3(kOutThreads), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace

bool adapter_width_supported(int c) { return c == 16 || c == 32 || c == 48 || c == 64; }

hipError_t launch_adapters(int c, const AdapterArgs& a, int in_type, hipStream_t s) {
  switch (c) {
    case 16: return launch_c<16>(a, in_type, s);
    case 32: return launch_c<32>(a, in_type, s);
    case 48: return launch_c<48>(a, in_type, s);
    case 64: return launch_c<64>(a, in_type, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lnm
