// Training of the channel adapters with the network: their backward pass
// (Section 4.3 puts four NAFBlocks on the decoder output; Section 5 trains
// the model on the lightmap loss).  The adapters' lightmaps replace the
// plain head's; the alpha/emissive group has no target, takes no gradient
// and is skipped.  fp32; the 1x1 products on the matrix cores in the layout
// of adapters.hip (channels as rows, 16 pixels as columns).
//
// The forward pass for training is the inference one keeping two more
// tensors (the depthwise outputs d and the image means m).  The backward
// pass recomputes the rest from them:
//   adapt_bwd_tail    workgroup per (256 pixels of one image, group): the
//                     tail chain again, the loss on the group's two lightmap
//                     channels and its gradient back to the gate output;
//                     writes the deltas and inputs of conv3/4/5 (their
//                     weight gradients), the features' gradient through the
//                     first residual, the gate's gradient and per-workgroup
//                     sums of every vector gradient;
//   adapt_bwd_attend  workgroup per group: the attention scale's gradient per
//                     image, its weights' gradient, the image-mean term of
//                     the gate gradient, and the tail's vector gradients;
//   adapt_bwd_front   workgroup per (8 x 32 tile, group, image): conv1 on
//                     tile + halo again, the gate's and depthwise conv's
//                     backward (mirrored taps), conv1's input gradient
//                     accumulated over the channel passes, layer norm 1's
//                     backward -> the features' gradient from this side;
//   adapt_bwd_finish  workgroup per group: the front's vector gradients (and
//                     zeros for the alpha/emissive group);
//   wgrad_1x1         dW = sum over pixels of delta x^T, K = pixels on the
//                     matrix cores, per chunk of pixels; chunk sums added in
//                     order by sum_chunks;
//   adapt_feat_grad   the features' gradient (the parts of the three groups
//                     added in a fixed order) through the decoder's ReLU, and
//                     the loss.
// Every sum runs in a fixed order, so results do not depend on scheduling.
#include <cmath>

#include "adapters_common.h"
#include "internal.h"

namespace lnm {
namespace {

constexpr int kTrainGroups = 3;  // groups with a lightmap target

// slots of the tail workgroups' sums
template <int C>
struct TailSlots {
  static constexpr int ds = 0, b3 = C, beta = 2 * C, l2w = 3 * C, l2b = 4 * C, b4 = 5 * C, b5 = 7 * C, gam = 8 * C,
                       hw = 9 * C, hb = 11 * C, loss = 11 * C + 2, n = 11 * C + 4;
};
// slots of the front workgroups' sums
template <int C>
struct FrontSlots {
  static constexpr int l1w = 0, l1b = C, b1 = 2 * C, dwb = 4 * C, dww = 6 * C, n = 24 * C;
};

template <int C>
__device__ __forceinline__ void fence_schedule() {
  if constexpr (C > 32) __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ f4 shfl_xor4(f4 v, int o) {
  return f4{__shfl_xor(v.x, o), __shfl_xor(v.y, o), __shfl_xor(v.z, o), __shfl_xor(v.w, o)};
}

// Adds v (this lane's channels 16 kb + 4 G + r of its NB pixels) summed over
// the wavefront's pixels to row[off + channel]: over nb in the lane, over the
// 16 pixel lanes by a butterfly, then lane li == 0 of each channel quad adds
// to the wavefront's own LDS row (one writer per row, in program order).
template <int KB, int NB>
__device__ __forceinline__ void row_add(float* row, int off, const f4 (&v)[KB][NB]) {
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    f4 s = v[kb][0];
#pragma unroll
    for (int nb = 1; nb < NB; ++nb) s += v[kb][nb];
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) s += shfl_xor4(s, o);
    if (li == 0) {
      float* d = row + off + 16 * kb + 4 * G;
      d[0] += s.x;
      d[1] += s.y;
      d[2] += s.z;
      d[3] += s.w;
    }
  }
}

// sum of a lane value over the wavefront (every lane gets it)
__device__ __forceinline__ float wave_sum(float s) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o);
  return s;
}

// out = bias + W[row0 + i][:] x over K = C (forward rows from LDS, pitch WP)
template <int C, int NB, int WP>
__device__ __forceinline__ void gemm_rows(const float* sw, int w_off, int row0, int b_off, const f4 (&x)[C / 16][NB],
                                          f4 (&out)[C / 16][NB]) {
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4;
#pragma unroll
  for (int mb = 0; mb < C / 16; ++mb) {
    const f4 bias = *reinterpret_cast<const f4*>(sw + b_off + 16 * mb + 4 * G);
    f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = bias;
#pragma unroll
    for (int kb = 0; kb < C / 16; ++kb) {
      const f4 w = *reinterpret_cast<const f4*>(sw + w_off + (row0 + 16 * mb + li) * WP + 16 * kb + 4 * G);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(w[r], x[kb][nb][r], acc[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) out[mb][nb] = acc[nb];
    fence_schedule<C>();
  }
}

// out (+)= W^T d: out[i] = sum_o W[row0 + o][i] d[o] over the 16 KBI rows o
// (A operand read transposed from the forward rows in LDS)
template <int C, int NB, int WP, int KBI>
__device__ __forceinline__ void gemm_t(const float* sw, int w_off, int row0, const f4 (&d)[KBI][NB],
                                       f4 (&out)[C / 16][NB], bool accumulate) {
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4;
#pragma unroll
  for (int mb = 0; mb < C / 16; ++mb) {
    f4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = accumulate ? out[mb][nb] : f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KBI; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float w = sw[w_off + (row0 + 16 * kb + 4 * G + r) * WP + 16 * mb + li];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(w, d[kb][nb][r], acc[nb]);
      }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) out[mb][nb] = acc[nb];
    fence_schedule<C>();
  }
}

__device__ __forceinline__ void st4(float* p, f4 v) { *reinterpret_cast<f4*>(p) = v; }
__device__ __forceinline__ f4 ldv(const float* p) { return *reinterpret_cast<const f4*>(p); }

template <int C>
__global__ __launch_bounds__(256) void adapt_bwd_tail(AdapterTrainArgs t) {
  using O = Off<C>;
  using S = TailSlots<C>;
  const AdapterArgs& a = t.f;
  constexpr int KB = C / 16;
  constexpr int NB = C <= 16 ? 4 : C <= 32 ? 2 : 1;  // register budget of the longer chain
  constexpr int WP = C + 4;
  constexpr int W3 = 0, W4 = C * WP, W5 = 3 * C * WP, VEC = 4 * C * WP;
  constexpr int B3 = VEC, BETA = B3 + C, L2W = BETA + C, L2B = L2W + C, B4 = L2B + C, B5 = B4 + 2 * C,
                GAM = B5 + C, HWT = GAM + C, HB = HWT + 2 * C, NW = HB + 4;
  __shared__ __attribute__((aligned(16))) float sw[NW];
  __shared__ float rows[4][S::n];
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, G = lane >> 4, wave = tid >> 6;
  const int g = blockIdx.y, blk = blockIdx.x, b = blk / t.tpi, tb = blk - b * t.tpi;
  const size_t HWn = (size_t)a.H * a.W;
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
  for (int q = tid; q < 4 * S::n; q += 256) rows[q / S::n][q % S::n] = 0.0f;
  __syncthreads();
  auto vec = [&](int off) { return ldv(sw + off + 4 * G); };
  float* row = rows[wave];
  const float* sv = a.sca + ((size_t)b * 4 + g) * C;
  const int dst0 = kDst[g][0], dst1 = kDst[g][1];
  const size_t gP = (size_t)g * a.P;

#pragma unroll 1
  for (int sub = 0; sub < 64 / (16 * NB); ++sub) {
    const size_t q0 = (size_t)tb * 256 + (size_t)wave * 64 + (size_t)sub * 16 * NB;  // pixel within the image
    size_t pix[NB];
    bool ok[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const size_t qi = q0 + 16 * nb + li;
      ok[nb] = qi < HWn;
      pix[nb] = (size_t)b * HWn + (ok[nb] ? qi : HWn - 1);
    }
    // ---- the forward chain again
    f4 x[KB][NB];  // a = v s (conv3's input)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        x[kb][nb] = ldv(a.v + (gP + pix[nb]) * C + 16 * kb + 4 * G) * ldv(sv + 16 * kb + 4 * G);
        if (ok[nb]) st4(t.x3 + (gP + pix[nb]) * C + 16 * kb + 4 * G, x[kb][nb]);
      }
    f4 t3[KB][NB];
    gemm_rows<C, NB, WP>(sw, W3, 0, B3, x, t3);
    f4 y[KB][NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        y[kb][nb] = feat4<C, 0>(a, pix[nb], 16 * kb + 4 * G) + vec(BETA + 16 * kb) * t3[kb][nb];
    // layer norm 2: xh and 1 / sigma
    f4 xh[KB][NB];
    float r2[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float s = 0.0f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) s += hsum(y[kb][nb]);
      const float mu = pixel_sum(s) * (1.0f / (float)C);
      float sq = 0.0f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        xh[kb][nb] = y[kb][nb] - mu;
        sq += hsum(xh[kb][nb] * xh[kb][nb]);
      }
      r2[nb] = 1.0f / sqrtf(pixel_sum(sq) * (1.0f / (float)C) + 1e-6f);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) xh[kb][nb] *= r2[nb];
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        x[kb][nb] = xh[kb][nb] * vec(L2W + 16 * kb) + vec(L2B + 16 * kb);  // n2 (conv4's input)
        if (ok[nb]) st4(t.x4 + (gP + pix[nb]) * C + 16 * kb + 4 * G, x[kb][nb]);
      }
    f4 e1[KB][NB], e2[KB][NB];
    gemm_rows<C, NB, WP>(sw, W4, 0, B4, x, e1);
    gemm_rows<C, NB, WP>(sw, W4, C, B4 + C, x, e2);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        x[kb][nb] = e1[kb][nb] * e2[kb][nb];  // h (conv5's input)
        if (ok[nb]) st4(t.x5 + (gP + pix[nb]) * C + 16 * kb + 4 * G, x[kb][nb]);
      }
    f4 t5[KB][NB];
    gemm_rows<C, NB, WP>(sw, W5, 0, B5, x, t5);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) y[kb][nb] += vec(GAM + 16 * kb) * t5[kb][nb];  // z
    // ---- head, sigmoid, loss and its gradient at the two outputs
    float do0[NB], do1[NB];
    float lsum = 0.0f, hsum0 = 0.0f, hsum1 = 0.0f;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float z0 = 0.0f, z1 = 0.0f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        z0 += hsum(vec(HWT + 16 * kb) * y[kb][nb]);
        z1 += hsum(vec(HWT + C + 16 * kb) * y[kb][nb]);
      }
      const float o0 = 1.0f / (1.0f + expf(-(pixel_sum(z0) + sw[HB])));
      const float o1 = 1.0f / (1.0f + expf(-(pixel_sum(z1) + sw[HB + 1])));
      float g0 = 0.0f, g1 = 0.0f;
      if (ok[nb]) {
        const float e0 = o0 - t.target[pix[nb] * 6 + dst0], ee1 = o1 - t.target[pix[nb] * 6 + dst1];
        if (G == 0) lsum += e0 * e0 + ee1 * ee1;
        g0 = 2.0f * e0 * t.inv_n * o0 * (1.0f - o0);
        g1 = 2.0f * ee1 * t.inv_n * o1 * (1.0f - o1);
        if (G == 0) {
          hsum0 += g0;
          hsum1 += g1;
        }
      }
      do0[nb] = g0;
      do1[nb] = g1;
    }
    {
      const float l = wave_sum(lsum), h0 = wave_sum(hsum0), h1 = wave_sum(hsum1);
      if (lane == 0) {
        row[S::loss] += l;
        row[S::hb] += h0;
        row[S::hb + 1] += h1;
      }
    }
    // head weights: dhw[k][ch] += do_k z[ch]; then dz = hw^T do
    {
      f4 tmp[KB][NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) tmp[kb][nb] = y[kb][nb] * do0[nb];
      row_add<KB, NB>(row, S::hw, tmp);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) tmp[kb][nb] = y[kb][nb] * do1[nb];
      row_add<KB, NB>(row, S::hw + C, tmp);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        y[kb][nb] = vec(HWT + 16 * kb) * do0[nb] + vec(HWT + C + 16 * kb) * do1[nb];  // dz = dy so far
    // z = y + gamma t5: dgamma += dz t5; dt5 = gamma dz
    {
      f4 tmp[KB][NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          tmp[kb][nb] = y[kb][nb] * t5[kb][nb];
          t5[kb][nb] = vec(GAM + 16 * kb) * y[kb][nb];  // dt5
          if (ok[nb]) st4(t.d5 + (gP + pix[nb]) * C + 16 * kb + 4 * G, t5[kb][nb]);
        }
      row_add<KB, NB>(row, S::gam, tmp);
      row_add<KB, NB>(row, S::b5, t5);
    }
    // dh = W5^T dt5; de = (dh e2, dh e1)
    gemm_t<C, NB, WP, KB>(sw, W5, 0, t5, x, false);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const f4 e1v = e1[kb][nb];
        e1[kb][nb] = x[kb][nb] * e2[kb][nb];
        e2[kb][nb] = x[kb][nb] * e1v;
        if (ok[nb]) {
          st4(t.d4 + (gP + pix[nb]) * 2 * C + 16 * kb + 4 * G, e1[kb][nb]);
          st4(t.d4 + (gP + pix[nb]) * 2 * C + C + 16 * kb + 4 * G, e2[kb][nb]);
        }
      }
    row_add<KB, NB>(row, S::b4, e1);
    row_add<KB, NB>(row, S::b4 + C, e2);
    // dn2 = W4^T de (K = 2C)
    gemm_t<C, NB, WP, KB>(sw, W4, 0, e1, x, false);
    gemm_t<C, NB, WP, KB>(sw, W4, C, e2, x, true);
    // layer norm 2's weights and its input gradient: dy += r (dxh - mean(dxh) - xh mean(dxh xh))
    {
      f4 tmp[KB][NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) tmp[kb][nb] = x[kb][nb] * xh[kb][nb];
      row_add<KB, NB>(row, S::l2w, tmp);
      row_add<KB, NB>(row, S::l2b, x);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float m1 = 0.0f, m2 = 0.0f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        x[kb][nb] *= vec(L2W + 16 * kb);  // dxh
        m1 += hsum(x[kb][nb]);
        m2 += hsum(x[kb][nb] * xh[kb][nb]);
      }
      m1 = pixel_sum(m1) * (1.0f / (float)C);
      m2 = pixel_sum(m2) * (1.0f / (float)C);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        y[kb][nb] += r2[nb] * (x[kb][nb] - m1 - xh[kb][nb] * m2);
        if (ok[nb]) st4(t.dyf + (gP + pix[nb]) * C + 16 * kb + 4 * G, y[kb][nb]);
      }
    }
    // y = feat + beta t3: dbeta += dy t3; dt3 = beta dy
    {
      f4 tmp[KB][NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          tmp[kb][nb] = y[kb][nb] * t3[kb][nb];
          t3[kb][nb] = vec(BETA + 16 * kb) * y[kb][nb];  // dt3
          if (ok[nb]) st4(t.d3 + (gP + pix[nb]) * C + 16 * kb + 4 * G, t3[kb][nb]);
        }
      row_add<KB, NB>(row, S::beta, tmp);
      row_add<KB, NB>(row, S::b3, t3);
    }
    // da = W3^T dt3; the gate's gradient from this side da s, and ds += da v
    gemm_t<C, NB, WP, KB>(sw, W3, 0, t3, x, false);
    {
      f4 tmp[KB][NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const f4 vv = ldv(a.v + (gP + pix[nb]) * C + 16 * kb + 4 * G);
          tmp[kb][nb] = x[kb][nb] * vv;
          if (ok[nb]) st4(t.dgt + (gP + pix[nb]) * C + 16 * kb + 4 * G, x[kb][nb] * ldv(sv + 16 * kb + 4 * G));
        }
      row_add<KB, NB>(row, S::ds, tmp);
    }
  }
  __syncthreads();
  float* out = t.tpart + ((size_t)g * gridDim.x + blk) * S::n;
  for (int q = tid; q < S::n; q += 256) out[q] = ((rows[0][q] + rows[1][q]) + rows[2][q]) + rows[3][q];
}

// grid: (3 groups).  ds per image (its tail workgroups' sums in order), the
// attention weights' gradient (images in order), dmh = Wsca^T ds / HW, and
// the tail's other vector gradients (all tail workgroups in order)
template <int C>
__global__ __launch_bounds__(256) void adapt_bwd_attend(AdapterTrainArgs t) {
  using O = Off<C>;
  using S = TailSlots<C>;
  const AdapterArgs& a = t.f;
  __shared__ float dss[C];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int nblk = a.B * t.tpi;
  const float* part = t.tpart + (size_t)g * nblk * S::n;
  const float* P = a.prm + (size_t)g * O::total;
  float* Gr = t.grad + (size_t)g * O::total;
  const float inv_hw = 1.0f / (float)(a.H * a.W);
  float gb = 0.0f, gw[C];
#pragma unroll
  for (int i = 0; i < C; ++i) gw[i] = 0.0f;
  for (int b = 0; b < a.B; ++b) {
    if (tid < C) {
      float ds = 0.0f;
      for (int k = 0; k < t.tpi; ++k) ds += part[(size_t)(b * t.tpi + k) * S::n + S::ds + tid];
      dss[tid] = ds;
      gb += ds;
      const float* m = a.msave + ((size_t)b * 4 + g) * C;
#pragma unroll
      for (int i = 0; i < C; ++i) gw[i] += ds * m[i];
    }
    __syncthreads();
    if (tid < C) {
      float dm = 0.0f;
      for (int o = 0; o < C; ++o) dm += P[O::scaw + o * C + tid] * dss[o];
      t.dmh[((size_t)b * 4 + g) * C + tid] = dm * inv_hw;
    }
    __syncthreads();
  }
  if (tid < C) {
    Gr[O::scab + tid] = gb;
#pragma unroll
    for (int i = 0; i < C; ++i) Gr[O::scaw + tid * C + i] = gw[i];
  }
  for (int q = tid; q < S::n; q += 256) {
    if (q < S::b3) continue;  // ds: per image, above
    float s = 0.0f;
    for (int k = 0; k < nblk; ++k) s += part[(size_t)k * S::n + q];
    if (q < S::beta) Gr[O::c3b + (q - S::b3)] = s;
    else if (q < S::l2w) Gr[O::beta + (q - S::beta)] = s;
    else if (q < S::l2b) Gr[O::ln2w + (q - S::l2w)] = s;
    else if (q < S::b4) Gr[O::ln2b + (q - S::l2b)] = s;
    else if (q < S::b5) Gr[O::c4b + (q - S::b4)] = s;
    else if (q < S::gam) Gr[O::c5b + (q - S::b5)] = s;
    else if (q < S::hw) Gr[O::gamma + (q - S::gam)] = s;
    else if (q < S::hb) Gr[O::hw + (q - S::hw)] = s;
    else if (q < S::loss) Gr[O::hb + (q - S::hb)] = s;
    else if (q == S::loss) t.lossg[g] = s;
  }
}

template <int C>
__global__ __launch_bounds__(256) void adapt_bwd_front(AdapterTrainArgs t) {
  using O = Off<C>;
  using S = FrontSlots<C>;
  const AdapterArgs& a = t.f;
  constexpr int KB = C / 16;
  __shared__ __attribute__((aligned(16))) float us[kHaloCols * 16 * kUPitch];   // u of the pass, then du
  __shared__ __attribute__((aligned(16))) float dds[kHaloCols * 16 * kUPitch];  // the depthwise output's gradient
  __shared__ __attribute__((aligned(16))) float wdw[2][9][16];
  __shared__ float rows[4][S::n];
  __shared__ f4 red[256][2];
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, G = lane >> 4, wave = tid >> 6;
  const int g = blockIdx.y, b = blockIdx.z;
  const int tiles_x = (a.W + kTX - 1) / kTX;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
  const int y0 = ty * kTY, x0 = tx * kTX;
  const float* P = a.prm + (size_t)g * O::total;
  const size_t img = (size_t)b * a.H * a.W, gP = (size_t)g * a.P;
  for (int q = tid; q < 4 * S::n; q += 256) rows[q / S::n][q % S::n] = 0.0f;
  f4 lw[KB], lb[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    lw[kb] = ld4(P + O::ln1w + 16 * kb + 4 * G);
    lb[kb] = ld4(P + O::ln1b + 16 * kb + 4 * G);
  }
  const int qd = tid & 3, xc = (tid >> 2) & 31, hh = tid >> 7;
  // conv1's input gradient of the wavefront's interior pixel blocks 4 w .. 4 w + 3
  f4 dn1[KB][4];
#pragma unroll
  for (int mb = 0; mb < KB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) dn1[mb][nb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const float* dmh = t.dmh + ((size_t)b * 4 + g) * C;

#pragma unroll 1
  for (int j = 0; j < KB; ++j) {
    for (int q = tid; q < 2 * 9 * 16; q += 256) {
      const int h = q / 144, tp = (q / 16) % 9, c = q % 16;
      wdw[h][tp][c] = P[O::dww + (h * C + 16 * j + c) * 9 + tp];
    }
    front_conv1<C, 0>(a, P, img, y0, x0, j, lw, lb, us, j == 0 ? t.x1 + gP * C : nullptr);
    // dd on tile + halo: gate gradient (with the image-mean term) times the partner channel
    for (int q = tid; q < kHaloCols * 16 * 8; q += 256) {
      const int hp = q >> 3, qq = q & 7, half = qq >> 2, q4 = qq & 3;
      const int hy = hp / kHX, hx = hp - hy * kHX;
      const int y = y0 + hy - 1, x = x0 + hx - 1;
      f4 v = f4{0.0f, 0.0f, 0.0f, 0.0f};
      if (hp < kHalo && y >= 0 && y < a.H && x >= 0 && x < a.W) {
        const size_t p = img + (size_t)y * a.W + x;
        const int i = 16 * j + 4 * q4;
        const f4 dg = ldv(t.dgt + (gP + p) * C + i) + ldv(dmh + i);
        v = dg * ldv(a.dsave + (gP + p) * 2 * C + (half ? i : C + i));
      }
      st4(dds + hp * kUPitch + 16 * half + 4 * q4, v);
    }
    __syncthreads();
    // depthwise backward for rows 4 hh .. 4 hh + 3 of column xc, channels
    // 16 j + 4 qd (+ C): du[p] = sum over taps of w[tap] dd[p - offset(tap)]
    f4 du1[4], du2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) du1[i] = du2[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int hr = 0; hr < 6; ++hr) {
      f4 a1[3], a2[3];
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        const float* src = dds + ((4 * hh + hr) * kHX + xc + cx) * kUPitch + 4 * qd;
        a1[cx] = ldv(src);
        a2[cx] = ldv(src + 16);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int dy = i + 2 - hr;
        if (dy < 0 || dy > 2) continue;
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
          const int tp = dy * 3 + (2 - cx);
          du1[i] += ldv(&wdw[0][tp][4 * qd]) * a1[cx];
          du2[i] += ldv(&wdw[1][tp][4 * qd]) * a2[cx];
        }
      }
    }
    f4 dd1[4], dd2[4];  // the interior pixels' own dd
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool in = y0 + 4 * hh + i < a.H && x0 + xc < a.W;
      const float* src = dds + ((4 * hh + i + 1) * kHX + xc + 1) * kUPitch + 4 * qd;
      dd1[i] = ldv(src);
      dd2[i] = ldv(src + 16);
      if (!in) du1[i] = du2[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    // the tile's sums: depthwise weights (9 taps), depthwise bias, conv1 bias;
    // each reduced over the 64 threads of a channel quad in thread order
#pragma unroll 1
    for (int k = 0; k < 11; ++k) {
      f4 v1 = f4{0.0f, 0.0f, 0.0f, 0.0f}, v2 = v1;
      if (k < 9) {
        const int dy = k / 3, dx = k - 3 * (k / 3);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float* src = us + ((4 * hh + i + dy) * kHX + xc + dx) * kUPitch + 4 * qd;
          v1 += dd1[i] * ldv(src);
          v2 += dd2[i] * ldv(src + 16);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          v1 += k == 9 ? dd1[i] : du1[i];
          v2 += k == 9 ? dd2[i] : du2[i];
        }
      }
      red[tid][0] = v1;
      red[tid][1] = v2;
      __syncthreads();
      if (tid < 32) {
        const int half = tid >> 4, q = (tid >> 2) & 3, r = tid & 3;
        float s = 0.0f;
        for (int u = 0; u < 64; ++u) s += red[(u << 2) | q][half][r];
        const int ch = half * C + 16 * j + 4 * q + r;
        if (k < 9) rows[0][S::dww + ch * 9 + k] += s;
        else if (k == 9) rows[0][S::dwb + ch] += s;
        else rows[0][S::b1 + ch] += s;
      }
      __syncthreads();
    }
    // du of the interior into LDS (us is free now) and to memory (conv1's weight gradient)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ip = (4 * hh + i) * kTX + xc;
      st4(us + ip * kUPitch + 4 * qd, du1[i]);
      st4(us + ip * kUPitch + 16 + 4 * qd, du2[i]);
      const int y = y0 + 4 * hh + i, x = x0 + xc;
      if (y < a.H && x < a.W) {
        const size_t p = img + (size_t)y * a.W + x;
        st4(t.d1 + (gP + p) * 2 * C + 16 * j + 4 * qd, du1[i]);
        st4(t.d1 + (gP + p) * 2 * C + C + 16 * j + 4 * qd, du2[i]);
      }
    }
    __syncthreads();
    // dn1 += W1^T du over the pass's 32 conv1 rows (16 j + k and C + 16 j + k)
    {
      f4 wt[KB][2];
#pragma unroll
      for (int mb = 0; mb < KB; ++mb)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float* src = P + O::c1w + (size_t)(h * C + 16 * j + 4 * G) * C + 16 * mb + li;
          wt[mb][h] = f4{src[0], src[C], src[2 * C], src[3 * C]};
        }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int ip = (4 * wave + nb) * 16 + li;
        const f4 b0 = ldv(us + ip * kUPitch + 4 * G), b1 = ldv(us + ip * kUPitch + 16 + 4 * G);
#pragma unroll
        for (int mb = 0; mb < KB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            dn1[mb][nb] = mfma(wt[mb][0][r], b0[r], dn1[mb][nb]);
            dn1[mb][nb] = mfma(wt[mb][1][r], b1[r], dn1[mb][nb]);
          }
      }
    }
    __syncthreads();  // before the next pass overwrites us and dds
  }
  // layer norm 1: weights' gradient and the features' gradient from this side
  {
    f4 gw[KB][4], gb[KB][4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int ip = (4 * wave + nb) * 16 + li;
      const int y = y0 + ip / kTX, x = x0 + ip % kTX;
      const bool in = y < a.H && x < a.W;
      const size_t p = img + (size_t)min(y, a.H - 1) * a.W + min(x, a.W - 1);
      f4 xh[KB];
      float s = 0.0f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        xh[kb] = feat4<C, 0>(a, p, 16 * kb + 4 * G);
        s += hsum(xh[kb]);
      }
      const float mu = pixel_sum(s) * (1.0f / (float)C);
      float sq = 0.0f;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        xh[kb] -= mu;
        sq += hsum(xh[kb] * xh[kb]);
      }
      const float rs = 1.0f / sqrtf(pixel_sum(sq) * (1.0f / (float)C) + 1e-6f);
      float m1 = 0.0f, m2 = 0.0f;
      f4 dxh[KB];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        xh[kb] *= rs;
        const f4 d = in ? dn1[kb][nb] : f4{0.0f, 0.0f, 0.0f, 0.0f};
        gw[kb][nb] = d * xh[kb];
        gb[kb][nb] = d;
        dxh[kb] = d * lw[kb];
        m1 += hsum(dxh[kb]);
        m2 += hsum(dxh[kb] * xh[kb]);
      }
      m1 = pixel_sum(m1) * (1.0f / (float)C);
      m2 = pixel_sum(m2) * (1.0f / (float)C);
      if (in) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          st4(t.dxf + (gP + p) * C + 16 * kb + 4 * G, rs * (dxh[kb] - m1 - xh[kb] * m2));
      }
    }
    row_add<KB, 4>(rows[wave], S::l1w, gw);
    row_add<KB, 4>(rows[wave], S::l1b, gb);
  }
  __syncthreads();
  float* out = t.fpart + (((size_t)g * a.B + b) * a.n_blk + blockIdx.x) * S::n;
  for (int q = tid; q < S::n; q += 256) out[q] = ((rows[0][q] + rows[1][q]) + rows[2][q]) + rows[3][q];
}

// grid: (4 groups): the front's vector gradients summed over its
// workgroups in order; the alpha/emissive group's slice set to zero
template <int C>
__global__ __launch_bounds__(256) void adapt_bwd_finish(AdapterTrainArgs t) {
  using O = Off<C>;
  using S = FrontSlots<C>;
  const AdapterArgs& a = t.f;
  const int g = blockIdx.x, tid = threadIdx.x;
  float* Gr = t.grad + (size_t)g * O::total;
  if (g >= kTrainGroups) {
    for (int q = tid; q < O::total; q += 256) Gr[q] = 0.0f;
    return;
  }
  const int nblk = a.B * a.n_blk;
  const float* part = t.fpart + (size_t)g * nblk * S::n;
  for (int q = tid; q < S::n; q += 256) {
    float s = 0.0f;
    for (int k = 0; k < nblk; ++k) s += part[(size_t)k * S::n + q];
    if (q < S::l1b) Gr[O::ln1w + q] = s;
    else if (q < S::b1) Gr[O::ln1b + (q - S::l1b)] = s;
    else if (q < S::dwb) Gr[O::c1b + (q - S::b1)] = s;
    else if (q < S::dww) Gr[O::dwb + (q - S::dwb)] = s;
    else Gr[O::dww + (q - S::dww)] = s;
  }
}

// part[chunk][M][N] = sum over pixels q of the chunk of delta[q][o] x[q][i]
// (K = pixels: lane (li, G) feeds row o / column i = li at pixel q + G)
constexpr int kWgradChunk = kAdaptWgradChunk;
__global__ __launch_bounds__(256) void wgrad_1x1(const float* __restrict__ delta, int M, const float* __restrict__ x,
                                                 int N, size_t P, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, li = lane & 15, G = lane >> 4, wave = threadIdx.x >> 6;
  const size_t q0 = (size_t)blockIdx.x * kWgradChunk;
  const size_t q1 = min(P, q0 + kWgradChunk);
  const int tn = N / 16, tiles = (M / 16) * tn;
  for (int tile = wave; tile < tiles; tile += 4) {  // uniform per wavefront
    const int mt = tile / tn, nt = tile - mt * tn;
    f4 acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (size_t q = q0; q < q1; q += 16) {
      float av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const size_t qq = q + 4 * u + G;
        const bool ok = qq < q1;
        av[u] = ok ? delta[qq * M + 16 * mt + li] : 0.0f;
        bv[u] = ok ? x[qq * N + 16 * nt + li] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = mfma(av[u], bv[u], acc);
    }
    float* out = part + (size_t)blockIdx.x * M * N;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(size_t)(16 * mt + 4 * G + r) * N + 16 * nt + li] = acc[r];
  }
}

// out[e] = sum over chunks (in order) of part[chunk][e]
__global__ __launch_bounds__(256) void sum_chunks(const float* __restrict__ part, int n_chunks, int n,
                                                  float* __restrict__ out) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float s = 0.0f;
  for (int k = 0; k < n_chunks; ++k) s += part[(size_t)k * n + e];
  out[e] = s;
}

// gfeat[q][i] = (y[q][i] > 0) * sum over groups (in order) of (dyf + dxf);
// block 0 also finishes the loss
template <int C>
__global__ __launch_bounds__(256) void adapt_feat_grad(AdapterTrainArgs t, const float* __restrict__ y,
                                                       float* __restrict__ gfeat) {
  const AdapterArgs& a = t.f;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    *t.loss = ((t.lossg[0] + t.lossg[1]) + t.lossg[2]) * t.inv_n;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.P * C) return;
  float s = 0.0f;
#pragma unroll
  for (int g = 0; g < kTrainGroups; ++g) s += t.dyf[(size_t)g * a.P * C + e] + t.dxf[(size_t)g * a.P * C + e];
  gfeat[e] = y[e] > 0.0f ? s : 0.0f;
}

template <int C>
hipError_t launch_train_c(const AdapterTrainArgs& t, const float* y_last, float* g_last, float* wpart,
                          hipStream_t s) {
  using O = Off<C>;
  const AdapterArgs& a = t.f;
  // forward for training (v, d, m, s kept)
  hipError_t e = launch_adapters_front(C, a, 0, s);
  if (e != hipSuccess) return e;
  // backward
  hipLaunchKernelGGL(adapt_bwd_tail<C>, dim3((unsigned)(a.B * t.tpi), kTrainGroups), dim3(256), 0, s, t);
  hipLaunchKernelGGL(adapt_bwd_attend<C>, dim3(kTrainGroups), dim3(256), 0, s, t);
  hipLaunchKernelGGL(adapt_bwd_front<C>, dim3((unsigned)a.n_blk, kTrainGroups, (unsigned)a.B), dim3(256), 0, s, t);
  hipLaunchKernelGGL(adapt_bwd_finish<C>, dim3(4), dim3(256), 0, s, t);
  const int chunks = (int)((a.P + kWgradChunk - 1) / kWgradChunk);
  struct Job {
    const float *d, *x;
    int M, off;
  };
  for (int g = 0; g < kTrainGroups; ++g) {
    const size_t gc = (size_t)g * a.P * C;
    const Job jobs[4] = {{t.d5 + gc, t.x5 + gc, C, O::c5w},
                         {t.d4 + 2 * gc, t.x4 + gc, 2 * C, O::c4w},
                         {t.d3 + gc, t.x3 + gc, C, O::c3w},
                         {t.d1 + 2 * gc, t.x1 + gc, 2 * C, O::c1w}};
    for (const Job& j : jobs) {
      hipLaunchKernelGGL(wgrad_1x1, dim3((unsigned)chunks), dim3(256), 0, s, j.d, j.M, j.x, C, a.P, wpart);
      const int n = j.M * C;
      hipLaunchKernelGGL(sum_chunks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, wpart, chunks, n,
                         t.grad + (size_t)g * O::total + j.off);
    }
  }
  const size_t n = a.P * C;
  hipLaunchKernelGGL(adapt_feat_grad<C>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, y_last, g_last);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_zero(float* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

}  // namespace

hipError_t launch_fill_zero(float* p, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}


hipError_t launch_adapters_train(int c, const AdapterTrainArgs& t, const float* y_last, float* g_last, float* wpart,
                                 hipStream_t s) {
  switch (c) {
    case 16: return launch_train_c<16>(t, y_last, g_last, wpart, s);
    case 32: return launch_train_c<32>(t, y_last, g_last, wpart, s);
    case 48: return launch_train_c<48>(t, y_last, g_last, wpart, s);
    case 64: return launch_train_c<64>(t, y_last, g_last, wpart, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lnm
