// Channel adapters on the U-Net decoder output (Section 4.3): four NAFBlocks
// (Chen et al. 2022), one per output group (front/back, left/right,
// up/down, alpha/emissive), each followed by a 1x1 head to its two channels
// and a sigmoid.  fp32 arithmetic; the 1x1 convolutions run on the fp32
// matrix cores (v_mfma_f32_16x16x4_f32).
//
// Every 1x1 convolution is computed transposed, out[channel][pixel] =
// W[channel][:] x[:][pixel]: channels are the MFMA rows and 16 pixels its
// columns.  A lane then holds four consecutive channels (16 mb + 4 (lane /
// 16) + r, r < 4, of each 16-channel block mb) of one pixel (lane % 16).
// That is the operand layout the next product reads when its K step (kb, r)
// takes input channel 16 kb + 4 (lane / 16) + r in both operands, so a chain
// of 1x1 convolutions stays in registers.  Per-pixel reductions over the
// channels (the layer norms, the head) add a lane's own channels and then
// the four lanes of the pixel (shuffles across 16 and 32 lanes).
//
// Three kernels, because the block's channel attention needs the mean of
// the gated features over the whole image between its two halves:
//   adapt_front  workgroup per (8 x 32 pixel tile, group, image): layer norm
//                1 and the 1x1 conv c -> 2c on the tile and a one-pixel halo
//                (recomputed, so the 2c-channel tensor never goes to
//                memory), 32 of the 2c channels at a time into LDS; then the
//                3x3 depthwise conv and the gate of those 16 channel pairs ->
//                v[g][P][c], and the tile's sum of v per channel;
//   adapt_attend workgroup per (group, image): the image mean of v (tile
//                sums added in a fixed order) and the attention's 1x1 conv
//                -> s[b][g][c];
//   adapt_tail   workgroup per (256 pixels, group): v * s, 1x1 conv c -> c,
//                residual with beta, layer norm 2, 1x1 c -> 2c, gate, 1x1
//                c -> c, residual with gamma, head, sigmoid; the three
//                weight matrices staged in LDS.
#include <cmath>

#include "adapters_common.h"
#include "internal.h"

namespace lnm {
namespace {

template <int C, int IN>
__global__ __launch_bounds__(256) void adapt_front(AdapterArgs a) {
  using O = Off<C>;
  constexpr int KB = C / 16;
  __shared__ __attribute__((aligned(16))) float us[kHaloCols * 16 * kUPitch];
  __shared__ __attribute__((aligned(16))) float wdw[2][9][16];  // the pass's depthwise taps [half][tap][channel]
  __shared__ f4 red[256];
  const int tid = threadIdx.x, lane = tid & 63, G = lane >> 4;
  const int g = blockIdx.y, b = blockIdx.z;
  const int tiles_x = (a.W + kTX - 1) / kTX;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
  const int y0 = ty * kTY, x0 = tx * kTX;
  const float* P = a.prm + (size_t)g * O::total;
  const size_t img = (size_t)b * a.H * a.W;
  // layer norm 1 weight and bias of this lane's channels 16 kb + 4 G + r
  f4 lw[KB], lb[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    lw[kb] = ld4(P + O::ln1w + 16 * kb + 4 * G);
    lb[kb] = ld4(P + O::ln1b + 16 * kb + 4 * G);
  }
  // depthwise stage: thread (quad qd, column xc, half hh) takes interior rows
  // 4 hh .. 4 hh + 3 of column xc and gate channels 16 j + 4 qd + (0..3)
  const int qd = tid & 3, xc = (tid >> 2) & 31, hh = tid >> 7;
  // up to width 32 the normed conv1 operands stay in registers across the
  // passes; wider blocks recompute them per pass (register budget)
  constexpr bool kCache = C <= 32;
  FrontOperands<kCache ? C : 16> fo;
  if constexpr (kCache) front_operands<C, IN>(a, img, y0, x0, lw, lb, fo);

#pragma unroll 1
  for (int j = 0; j < KB; ++j) {
    for (int q = tid; q < 2 * 9 * 16; q += 256) {
      const int h = q / 144, t = (q / 16) % 9, c = q % 16;
      wdw[h][t][c] = P[O::dww + (h * C + 16 * j + c) * 9 + t];
    }
    if constexpr (kCache)
      front_conv1_cached<C>(P, j, fo, us);
    else
      front_conv1<C, IN>(a, P, img, y0, x0, j, lw, lb, us, nullptr);
    __syncthreads();
    {
      const int ch = 16 * j + 4 * qd;
      const f4 d1 = ld4(P + O::dwb + ch), d2 = ld4(P + O::dwb + C + ch);
      f4 s1[4], s2[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        s1[i] = d1;
        s2[i] = d2;
      }
      // halo rows 4 hh + hr feed interior rows 4 hh + i at tap row hr - i
      // (a loop, not unrolled: unrolled, the compiler hoists all 36 LDS
      // loads and the kernel runs one wavefront per SIMD)
#pragma unroll 1
      for (int hr = 0; hr < 6; ++hr) {
        f4 ua[3], ub[3];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const float* src = us + ((4 * hh + hr) * kHX + xc + dx) * kUPitch + 4 * qd;
          ua[dx] = *reinterpret_cast<const f4*>(src);
          ub[dx] = *reinterpret_cast<const f4*>(src + 16);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int dy = hr - i;
          if (dy < 0 || dy > 2) continue;
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            s1[i] += *reinterpret_cast<const f4*>(&wdw[0][dy * 3 + dx][4 * qd]) * ua[dx];
            s2[i] += *reinterpret_cast<const f4*>(&wdw[1][dy * 3 + dx][4 * qd]) * ub[dx];
          }
        }
      }
      f4 part = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int y = y0 + 4 * hh + i, x = x0 + xc;
        if (y < a.H && x < a.W) {
          const size_t p = img + (size_t)y * a.W + x;
          const f4 v = s1[i] * s2[i];
          *reinterpret_cast<f4*>(a.v + ((size_t)g * a.P + p) * C + ch) = v;
          part += v;
          if (a.dsave) {  // training keeps the depthwise outputs for the backward pass
            *reinterpret_cast<f4*>(a.dsave + ((size_t)g * a.P + p) * 2 * C + ch) = s1[i];
            *reinterpret_cast<f4*>(a.dsave + ((size_t)g * a.P + p) * 2 * C + C + ch) = s2[i];
          }
        }
      }
      red[tid] = part;
    }
    __syncthreads();  // LDS u of this pass consumed; the sums in red complete
    if (tid < 16) {
      // channel 16 j + 4 q + r: the 64 threads of quad q, in thread order
      const int q = tid >> 2, r = tid & 3;
      float s = 0.0f;
      for (int t = 0; t < 64; ++t) s += red[(t << 2) | q][r];
      a.part[(((size_t)b * 4 + g) * a.n_blk + blockIdx.x) * C + 16 * j + 4 * q + r] = s;
    }
  }
}

// grid: (4, B); image mean of v per channel (thread (slice, ch) sums the
// tile sums slice, slice + S, ... in order, then the S slices are added in
// order), then the attention's 1x1 conv
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
    // tile sums [tile][C]: the lanes of a slice read one tile's row together
    const float* src = a.part + ((size_t)b * 4 + g) * a.n_blk * C + ch;
    float s = 0.0f;
#pragma unroll 4
    for (int k = slice; k < a.n_blk; k += S) s += src[(size_t)k * C];
    red[slice][ch] = s;
  }
  __syncthreads();
  if (threadIdx.x < C) {
    float s = 0.0f;
    for (int q = 0; q < S; ++q) s += red[q][threadIdx.x];
    pooled[threadIdx.x] = s / (float)(a.H * a.W);
    if (a.msave) a.msave[((size_t)b * 4 + g) * C + threadIdx.x] = pooled[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x < C) {
    float s = P[O::scab + threadIdx.x];
#pragma unroll 8
    for (int i = 0; i < C; ++i) s += P[O::scaw + threadIdx.x * C + i] * pooled[i];
    a.sca[((size_t)b * 4 + g) * C + threadIdx.x] = s;
  }
}


constexpr int kTailPix = 256;  // pixels per tail workgroup (64 per wavefront)

// Wide adapters: keep the scheduler from moving one output block's weight
// loads above the previous block's products (hoisted, they take every
// register of the wavefront)
template <int C>
__device__ __forceinline__ void fence_schedule() {
  if constexpr (C > 32) __builtin_amdgcn_sched_barrier(0);
}

// Width 32 asks for four wavefronts per SIMD (128 registers, a few spilled):
// the chain is latency-bound and the fourth wavefront hides more of it than
// the spill costs (40 -> 36 us per 256x256 frame).
template <int C, int IN>
__global__ __launch_bounds__(256, C == 32 ? 4 : 1) void adapt_tail(AdapterArgs a, int n_tiles) {
  using O = Off<C>;
  constexpr int KB = C / 16;
  constexpr int NB = C <= 32 ? 4 : 2;  // 16-pixel column blocks per MFMA batch (register budget)
  constexpr int WP = C + 4;            // LDS row pitch of the weight matrices (bank spread)
  constexpr int W3 = 0, W4 = C * WP, W5 = 3 * C * WP, VEC = 4 * C * WP;
  constexpr int B3 = VEC, BETA = B3 + C, L2W = BETA + C, L2B = L2W + C, B4 = L2B + C, B5 = B4 + 2 * C,
                GAM = B5 + C, HWT = GAM + C, HB = HWT + 2 * C, NW = HB + 4;
  __shared__ __attribute__((aligned(16))) float sw[NW];
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, G = lane >> 4, wave = tid >> 6;
  // the four groups of a tile are blocks 8 apart: round-robin placement puts
  // them on one XCD, whose L2 then serves the tile's features to all four
  const int id = blockIdx.x;
  const int g = (id >> 3) & 3, tile = ((id >> 5) << 3) | (id & 7);
  if (tile >= n_tiles) return;  // whole workgroup, before any barrier
  const float* P = a.prm + (size_t)g * O::total;
  for (int q = tid; q < C * C; q += 256) {
    const int r = q / C, col = q - r * C;
    sw[W3 + r * WP + col] = P[O::c3w + q];
    sw[W5 + r * WP + col] = P[O::c5w + q];
  }
  for (int q = tid; q < 2 * C * C; q += 256) {
    const int r = q / C, col = q - r * C;
    sw[W4 + r * WP + col] = P[O::c4w + q];
  }
  for (int q = tid; q < C; q += 256) {
    sw[B3 + q] = P[O::c3b + q];
    sw[BETA + q] = P[O::beta + q];
    sw[L2W + q] = P[O::ln2w + q];
    sw[L2B + q] = P[O::ln2b + q];
    sw[B5 + q] = P[O::c5b + q];
    sw[GAM + q] = P[O::gamma + q];
  }
  for (int q = tid; q < 2 * C; q += 256) {
    sw[B4 + q] = P[O::c4b + q];
    sw[HWT + q] = P[O::hw + q];
  }
  if (tid < 2) sw[HB + tid] = P[O::hb + tid];
  __syncthreads();
  // this lane's four channels of a vector, and of weight row `row` at K block kb
  auto vec = [&](int off) { return *reinterpret_cast<const f4*>(sw + off + 4 * G); };
  auto wrow = [&](int off, int row, int kb) {
    return *reinterpret_cast<const f4*>(sw + off + row * WP + 16 * kb + 4 * G);
  };
  const size_t HWn = (size_t)a.H * a.W;

#pragma unroll 1
  for (int sub = 0; sub < 64 / (16 * NB); ++sub) {
    const size_t pbase = (size_t)tile * kTailPix + (size_t)wave * 64 + (size_t)sub * 16 * NB;
    size_t pix[NB];
    bool ok[NB];
    f4 t[KB][NB];
    // t = v * s
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const size_t p = pbase + 16 * nb + li;
      ok[nb] = p < a.P;
      pix[nb] = ok[nb] ? p : a.P - 1;
      const float* s = a.sca + ((size_t)(pix[nb] / HWn) * 4 + g) * C;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        t[kb][nb] = *reinterpret_cast<const f4*>(a.v + ((size_t)g * a.P + pix[nb]) * C + 16 * kb + 4 * G) *
                    *reinterpret_cast<const f4*>(s + 16 * kb + 4 * G);
    }
    // y = in + beta (W3 t + b3)
    f4 y[KB][NB];
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      f4 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = vec(B3 + 16 * mb);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const f4 w = wrow(W3, 16 * mb + li, kb);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(w[r], t[kb][nb][r], acc[nb]);
      }
      const f4 beta = vec(BETA + 16 * mb);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) y[mb][nb] = feat4<C, IN>(a, pix[nb], 16 * mb + 4 * G) + beta * acc[nb];
      fence_schedule<C>();
    }
    // t = LN2(y) w + b over each pixel's C channels
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float s = 0.0f;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) s += hsum(y[mb][nb]);
      const float mu = pixel_sum(s) * (1.0f / (float)C);
      float sq = 0.0f;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) {
        t[mb][nb] = y[mb][nb] - mu;
        sq += hsum(t[mb][nb] * t[mb][nb]);
      }
      const float rs = 1.0f / sqrtf(pixel_sum(sq) * (1.0f / (float)C) + 1e-6f);
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) t[mb][nb] = t[mb][nb] * rs * vec(L2W + 16 * mb) + vec(L2B + 16 * mb);
    }
    // h = gate(W4 t + b4): output rows 16 mb + i and C + 16 mb + i multiply
    f4 h[KB][NB];
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      f4 a1[NB], a2[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        a1[nb] = vec(B4 + 16 * mb);
        a2[nb] = vec(B4 + C + 16 * mb);
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const f4 w1 = wrow(W4, 16 * mb + li, kb), w2 = wrow(W4, C + 16 * mb + li, kb);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            a1[nb] = mfma(w1[r], t[kb][nb][r], a1[nb]);
            a2[nb] = mfma(w2[r], t[kb][nb][r], a2[nb]);
          }
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) h[mb][nb] = a1[nb] * a2[nb];
      fence_schedule<C>();
    }
    // y += gamma (W5 h + b5)
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      f4 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = vec(B5 + 16 * mb);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const f4 w = wrow(W5, 16 * mb + li, kb);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(w[r], h[kb][nb][r], acc[nb]);
      }
      const f4 gam = vec(GAM + 16 * mb);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) y[mb][nb] += gam * acc[nb];
      fence_schedule<C>();
    }
    // head and sigmoid
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float z0 = 0.0f, z1 = 0.0f;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) {
        z0 += hsum(vec(HWT + 16 * mb) * y[mb][nb]);
        z1 += hsum(vec(HWT + C + 16 * mb) * y[mb][nb]);
      }
      z0 = pixel_sum(z0) + sw[HB];
      z1 = pixel_sum(z1) + sw[HB + 1];
      if (G == 0 && ok[nb]) {
        const float o[2] = {1.0f / (1.0f + expf(-z0)), 1.0f / (1.0f + expf(-z1))};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int d = kDst[g][k];
          if (d >= 0)
            a.lm[pix[nb] * 6 + d] = o[k];
          else if (a.extra)
            a.extra[pix[nb] * 2 + (-1 - d)] = o[k];
        }
      }
    }
  }
}

template <int C>
void launch_front_c(const AdapterArgs& a, int in_type, hipStream_t s) {
  const dim3 fgrid((unsigned)a.n_blk, 4, (unsigned)a.B);
  switch (in_type) {
    case 0: hipLaunchKernelGGL((adapt_front<C, 0>), fgrid, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((adapt_front<C, 1>), fgrid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((adapt_front<C, 2>), fgrid, dim3(256), 0, s, a); break;
  }
  hipLaunchKernelGGL(adapt_attend<C>, dim3(4, a.B), dim3(256), 0, s, a);
}

template <int C>
hipError_t launch_c(const AdapterArgs& a, int in_type, hipStream_t s) {
  launch_front_c<C>(a, in_type, s);
  const int n_tiles = (int)((a.P + kTailPix - 1) / kTailPix);
  const unsigned tblk = 32u * (unsigned)((n_tiles + 7) / 8);
  switch (in_type) {
    case 0: hipLaunchKernelGGL((adapt_tail<C, 0>), dim3(tblk), dim3(256), 0, s, a, n_tiles); break;
    case 1: hipLaunchKernelGGL((adapt_tail<C, 1>), dim3(tblk), dim3(256), 0, s, a, n_tiles); break;
    default: hipLaunchKernelGGL((adapt_tail<C, 2>), dim3(tblk), dim3(256), 0, s, a, n_tiles); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adapters_front(int c, const AdapterArgs& a, int in_type, hipStream_t s) {
  switch (c) {
    case 16: launch_front_c<16>(a, in_type, s); break;
    case 32: launch_front_c<32>(a, in_type, s); break;
    case 48: launch_front_c<48>(a, in_type, s); break;
    case 64: launch_front_c<64>(a, in_type, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

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
