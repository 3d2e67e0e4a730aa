// Backward-pass and optimiser kernels for training the fp32 U-Net on the GPU
// (Section 4.4 pixel loss in sRGB space, Section 5 Adam).  Every reduction
// has a fixed assignment of terms to lanes and blocks and a fixed combination
// order, so a gradient does not depend on scheduling.
#include "internal.h"

namespace lnm {
namespace {

// Block-wide sum in a fixed tree order (256 lanes).
__device__ __forceinline__ float block_sum(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

// e = y - t; dz = 2 e y (1 - y) / n (mean-squared error through the sigmoid);
// partial[block] = sum of e^2 over the block's fixed element range.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                    float* __restrict__ dz, float* __restrict__ partial, long n) {
  __shared__ float sh[256];
  const float scale = 2.0f / (float)n;
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * per, hi = min(n, lo + per);
  float acc = 0.0f;
  for (long i = lo + threadIdx.x; i < hi; i += 256) {
    const float yy = y[i], e = yy - t[i];
    acc += e * e;
    dz[i] = scale * e * yy * (1.0f - yy);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void finish_sum(const float* __restrict__ partial, int n, float scale,
                                                   float* __restrict__ out) {
  __shared__ float sh[256];
  float acc = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = acc * scale;
}

// Column sums of E[P][C] in two fixed stages: partial[block][c] over a fixed
// pixel range, then out[c] = sum over blocks in order.
__global__ __launch_bounds__(256) void colsum_partial(const float* __restrict__ e, long P, int C,
                                                       float* __restrict__ partial) {
  const long per = (P + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * per, hi = min(P, lo + per);
  for (int c = threadIdx.x; c < C; c += 256) {
    float acc = 0.0f;
    for (long p = lo; p < hi; ++p) acc += e[p * C + c];
    partial[(long)blockIdx.x * C + c] = acc;
  }
}

__global__ __launch_bounds__(256) void colsum_finish(const float* __restrict__ partial, int nb, int C,
                                                      float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= C) return;
  float acc = 0.0f;
  for (int b = 0; b < nb; ++b) acc += partial[(long)b * C + c];
  out[c] = acc;
}

__global__ __launch_bounds__(256) void relu_mask(float* __restrict__ g, const float* __restrict__ y, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n && !(y[i] > 0.0f)) g[i] = 0.0f;
}

// Head (1x1, C -> 6) backward, data part fused with the ReLU mask of its
// input: E[p][c] = (sum_o W[o][c] dz[p][o]) * (X[p][c] > 0).
__global__ __launch_bounds__(256) void head_bwd_data(const float* __restrict__ dz, const float* __restrict__ w,
                                                      const float* __restrict__ x, long P, int C,
                                                      float* __restrict__ e) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= P * C) return;
  const long p = i / C;
  const int c = i - p * C;
  float s = 0.0f;
#pragma unroll
  for (int o = 0; o < 6; ++o) s += w[o * C + c] * dz[p * 6 + o];
  e[i] = x[i] > 0.0f ? s : 0.0f;
}

// Head weight/bias gradient: block (o, c) reduces over all pixels in a fixed
// order; c == C gives the bias.
__global__ __launch_bounds__(256) void head_bwd_weight(const float* __restrict__ dz, const float* __restrict__ x,
                                                        long P, int C, float* __restrict__ gw,
                                                        float* __restrict__ gb) {
  __shared__ float sh[256];
  const int o = blockIdx.x / (C + 1), c = blockIdx.x % (C + 1);
  float acc = 0.0f;
  for (long p = threadIdx.x; p < P; p += 256) acc += dz[p * 6 + o] * (c < C ? x[p * C + c] : 1.0f);
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (c < C)
      gw[o * C + c] = acc;
    else
      gb[o] = acc;
  }
}

// Gradient of concat(skip, upsample2(low)): the first c0 channels go to the
// skip, the rest are summed over each 2x2 block into the low-resolution map.
__global__ __launch_bounds__(256) void route_concat_skip(const float* __restrict__ dx, long P, int c0, int c1,
                                                          float* __restrict__ g_skip) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= P * c0) return;
  const long p = i / c0;
  g_skip[i] = dx[p * (c0 + c1) + (i - p * c0)];
}

__global__ __launch_bounds__(256) void route_concat_low(const float* __restrict__ dx, int B, int H, int W, int c0,
                                                         int c1, float* __restrict__ g_low) {
  const int h = H >> 1, w = W >> 1;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)B * h * w * c1) return;
  const int c = i % c1;
  const long q = i / c1;
  const int xx = q % w, yy = (q / w) % h, b = q / ((long)w * h);
  const int ct = c0 + c1;
  float s = 0.0f;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx2 = 0; dx2 < 2; ++dx2)
      s += dx[((size_t)(b * H + 2 * yy + dy) * W + 2 * xx + dx2) * ct + c0 + c];
  g_low[i] = s;
}

// 2x2 max-pool backward: the gradient of each pooled element is added at the
// first maximum of its window in raster order.
__global__ __launch_bounds__(256) void route_pool(const float* __restrict__ dx, const float* __restrict__ y, int B,
                                                   int h, int w, int C, float* __restrict__ g) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)B * h * w * C) return;
  const int c = i % C;
  const long q = i / C;
  const int xx = q % w, yy = (q / w) % h, b = q / ((long)w * h);
  const int W2 = 2 * w;
  size_t best = ((size_t)(b * 2 * h + 2 * yy) * W2 + 2 * xx) * C + c;
  float m = y[best];
  const size_t cand[3] = {best + C, best + (size_t)W2 * C, best + (size_t)W2 * C + C};
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (y[cand[k]] > m) {
      m = y[cand[k]];
      best = cand[k];
    }
  g[best] += dx[i];
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                    float* __restrict__ m, float* __restrict__ v, long n, float lr,
                                                    float b1, float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Packed fp32 layout [n_tile][chunk][tap][n (32)][c (ck)] from flat
// W[co][ci][3][3].  dgrad = 1: the layout of the convolution that propagates
// gradients, whose input channels are the layer's outputs and whose output
// channels are the layer's inputs, taps mirrored (8 - tap).
__global__ __launch_bounds__(256) void pack_f32(const float* __restrict__ w, const float* __restrict__ bsrc,
                                                 LayerDesc d, int dgrad, float* __restrict__ dst,
                                                 float* __restrict__ bdst, int src_ci, int src_co) {
  const long total = (long)d.co_pad * d.ci_pad * 9;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < total) {
    const int cc = i % d.ck;
    long r = i / d.ck;
    const int n = r % kBN;
    r /= kBN;
    const int tap = r % 9;
    r /= 9;
    const int nch = d.ci_pad / d.ck;
    const int ch = r % nch, t = r / nch;
    const int oc = t * kBN + n, ic = ch * d.ck + cc;  // output / input channel of this convolution
    float v = 0.0f;
    if (oc < d.co && ic < d.ci) {
      if (dgrad)
        v = w[((size_t)ic * src_ci + oc) * 9 + (8 - tap)];
      else
        v = w[((size_t)oc * src_ci + ic) * 9 + tap];
    }
    dst[i] = v;
  }
  if (bdst && i < d.co_pad) bdst[i] = (!dgrad && i < d.co) ? bsrc[i] : 0.0f;
  (void)src_co;
}

}  // namespace

hipError_t launch_loss(const float* y, const float* t, float* dz, float* partial, long n, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(kLossBlocks), dim3(256), 0, s, y, t, dz, partial, n);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, s, partial, kLossBlocks, 1.0f / (float)n, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* e, long P, int C, float* partial, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_partial, dim3(kColsumBlocks), dim3(256), 0, s, e, P, C, partial);
  hipLaunchKernelGGL(colsum_finish, dim3((C + 255) / 256), dim3(256), 0, s, partial, kColsumBlocks, C, out);
  return hipGetLastError();
}

hipError_t launch_relu_mask(float* g, const float* y, long n, hipStream_t s) {
  hipLaunchKernelGGL(relu_mask, dim3((n + 255) / 256), dim3(256), 0, s, g, y, n);
  return hipGetLastError();
}

hipError_t launch_head_bwd(const float* dz, const float* w, const float* x, long P, int C, float* e_out,
                           float* grad_w, float* grad_b, float* partial, hipStream_t s) {
  (void)partial;
  hipLaunchKernelGGL(head_bwd_data, dim3((P * C + 255) / 256), dim3(256), 0, s, dz, w, x, P, C, e_out);
  hipLaunchKernelGGL(head_bwd_weight, dim3(6 * (C + 1)), dim3(256), 0, s, dz, x, P, C, grad_w, grad_b);
  return hipGetLastError();
}

hipError_t launch_route_concat(const float* dx, int B, int H, int W, int c0, int c1, float* g_skip, float* g_low,
                               hipStream_t s) {
  const long P = (long)B * H * W;
  hipLaunchKernelGGL(route_concat_skip, dim3((P * c0 + 255) / 256), dim3(256), 0, s, dx, P, c0, c1, g_skip);
  const long nl = (long)B * (H / 2) * (W / 2) * c1;
  hipLaunchKernelGGL(route_concat_low, dim3((nl + 255) / 256), dim3(256), 0, s, dx, B, H, W, c0, c1, g_low);
  return hipGetLastError();
}

hipError_t launch_route_pool(const float* dx, const float* y, int B, int h, int w, int c, float* g, hipStream_t s) {
  const long n = (long)B * h * w * c;
  hipLaunchKernelGGL(route_pool, dim3((n + 255) / 256), dim3(256), 0, s, dx, y, B, h, w, c, g);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_f32(const float* flat_w, const float* flat_b, const LayerDesc& d, int dgrad, char* dst,
                           size_t w_off, size_t b_off, hipStream_t s) {
  // src_ci: input channels of the original layer (row length of flat W)
  const int src_ci = dgrad ? d.co : d.ci;
  const long total = (long)d.co_pad * d.ci_pad * 9;
  const long n = std::max<long>(total, d.co_pad);
  hipLaunchKernelGGL(pack_f32, dim3((n + 255) / 256), dim3(256), 0, s, flat_w, flat_b, d, dgrad,
                     reinterpret_cast<float*>(dst + w_off), dgrad ? nullptr : reinterpret_cast<float*>(dst + b_off),
                     src_ci, 0);
  return hipGetLastError();
}

}  // namespace lnm
