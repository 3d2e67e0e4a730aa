// Guiding-map ray march (Algorithm 1, Section 4.2) and fine-step six-way
// reference lightmaps, fp32, one lane per pixel.
//
// Work mapping: a 256-lane workgroup covers a 16x16 pixel tile and each
// wavefront an 8x8 sub-tile, so the 64 rays of a wave are spatially coherent
// and their trilinear gathers hit the same cache lines.  A wave retires when
// its last ray terminates (early termination is per lane, so the wave's
// lifetime is that of its longest ray).
#include <cmath>

#include "internal.h"

namespace lnm {
namespace {

struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 scale3(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ V3 normalize3(V3 a) { return scale3(a, 1.0f / sqrtf(dot3(a, a))); }

// SplitMix64 output for state s: the finaliser applied to s + golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// sigma(p): sigma_scale x zero-border cell-centred trilinear interpolation.
// Corner indices are clamped into the grid and corners outside it get weight
// zero, so every load is in bounds.
__device__ __forceinline__ float sample_sigma(const MarchDev& m, float px, float py, float pz) {
  const float gx = px * (float)m.nx - 0.5f, gy = py * (float)m.ny - 0.5f, gz = pz * (float)m.nz - 0.5f;
  if (!(gx > -1.0f && gy > -1.0f && gz > -1.0f && gx < (float)m.nx && gy < (float)m.ny && gz < (float)m.nz))
    return 0.0f;
  const float fx0 = floorf(gx), fy0 = floorf(gy), fz0 = floorf(gz);
  const int i = (int)fx0, j = (int)fy0, k = (int)fz0;
  const float fx = gx - fx0, fy = gy - fy0, fz = gz - fz0;
  const float wx0 = i >= 0 ? 1.0f - fx : 0.0f, wx1 = i + 1 < m.nx ? fx : 0.0f;
  const float wy0 = j >= 0 ? 1.0f - fy : 0.0f, wy1 = j + 1 < m.ny ? fy : 0.0f;
  const float wz0 = k >= 0 ? 1.0f - fz : 0.0f, wz1 = k + 1 < m.nz ? fz : 0.0f;
  const int ia = max(i, 0), ib = min(i + 1, m.nx - 1);
  const size_t sy = (size_t)m.nx, sz = (size_t)m.nx * m.ny;
  const size_t ya = (size_t)max(j, 0) * sy, yb = (size_t)min(j + 1, m.ny - 1) * sy;
  const size_t za = (size_t)max(k, 0) * sz, zb = (size_t)min(k + 1, m.nz - 1) * sz;
  const float* r = m.rho;
  const float c00 = wx0 * r[za + ya + ia] + wx1 * r[za + ya + ib];
  const float c10 = wx0 * r[za + yb + ia] + wx1 * r[za + yb + ib];
  const float c01 = wx0 * r[zb + ya + ia] + wx1 * r[zb + ya + ib];
  const float c11 = wx0 * r[zb + yb + ia] + wx1 * r[zb + yb + ib];
  const float v = wz0 * (wy0 * c00 + wy1 * c10) + wz1 * (wy0 * c01 + wy1 * c11);
  return m.sigma_scale * v;
}

// Parametric exit distance of x + s l from the support box (x assumed inside);
// negative if x lies outside along some axis.
__device__ __forceinline__ float exit_distance(const MarchDev& m, V3 x, V3 l) {
  float s = INFINITY;
  const float px[3] = {x.x, x.y, x.z}, dl[3] = {l.x, l.y, l.z};
  const int n[3] = {m.nx, m.ny, m.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (dl[a] == 0.0f) continue;
    const float b = dl[a] > 0.0f ? 1.0f + 0.5f / (float)n[a] : -0.5f / (float)n[a];
    s = fminf(s, (b - px[a]) / dl[a]);
  }
  return s;
}

// Ray-box clip of o + t d against the support box, t >= 0.
__device__ __forceinline__ bool clip_support(const MarchDev& m, V3 o, V3 d, float* t0, float* t1) {
  float lo = 0.0f, hi = INFINITY;
  const float po[3] = {o.x, o.y, o.z}, pd[3] = {d.x, d.y, d.z};
  const int n[3] = {m.nx, m.ny, m.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float bmin = -0.5f / (float)n[a], bmax = 1.0f + 0.5f / (float)n[a];
    if (pd[a] == 0.0f) {
      if (po[a] < bmin || po[a] > bmax) return false;
      continue;
    }
    float ta = (bmin - po[a]) / pd[a], tb = (bmax - po[a]) / pd[a];
    if (ta > tb) {
      const float t = ta;
      ta = tb;
      tb = t;
    }
    lo = fmaxf(lo, ta);
    hi = fminf(hi, tb);
  }
  *t0 = lo;
  *t1 = hi;
  return hi >= lo;
}

// Transmittance from x toward l: exp(-h sum_k sigma(x + k h l)) over the
// points inside the support box, 0 once the optical depth passes tau_max.
__device__ __forceinline__ float light_transmittance(const MarchDev& m, V3 x, V3 l, float h, float tau_max) {
  const float s1 = exit_distance(m, x, l);
  const int kmax = s1 > 0.0f ? (int)floorf(s1 / h) : 0;
  const float lim = tau_max / h;
  float acc = 0.0f;
  // four samples' gathers are issued together; they are summed and tested
  // against the termination limit one at a time, in order
  for (int k = 1; k <= kmax; k += 4) {
    float s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float t = (float)(k + j) * h;
      s[j] = k + j <= kmax ? sample_sigma(m, x.x + t * l.x, x.y + t * l.y, x.z + t * l.z) : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc += s[j];
      if (acc > lim) return 0.0f;
    }
  }
  return expf(-acc * h);
}

__device__ __forceinline__ void camera_ray(const CamDev& c, int i, int j, V3* o, V3* d) {
  const float sx = 2.0f * ((float)i + 0.5f) / (float)c.W - 1.0f;
  const float sy = 1.0f - 2.0f * ((float)j + 0.5f) / (float)c.H;
  const V3 f = v3(c.f[0], c.f[1], c.f[2]), r = v3(c.r[0], c.r[1], c.r[2]), u = v3(c.u[0], c.u[1], c.u[2]);
  const float a = sx * c.aspect;
  if (c.proj == LNM_PERSPECTIVE) {
    *o = v3(c.eye[0], c.eye[1], c.eye[2]);
    *d = normalize3(v3(f.x + c.tan_half * (a * r.x + sy * u.x), f.y + c.tan_half * (a * r.y + sy * u.y),
                       f.z + c.tan_half * (a * r.z + sy * u.z)));
  } else {
    const float e = c.half_extent;
    *o = v3(c.eye[0] + e * (a * r.x + sy * u.x), c.eye[1] + e * (a * r.y + sy * u.y),
            c.eye[2] + e * (a * r.z + sy * u.z));
    *d = f;
  }
}

__device__ __forceinline__ void tile_pixel(int* i, int* j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  *i = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  *j = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
}

// Top surrogate light of a ray: normalize(w x z), or normalize(w x x) when w
// is parallel to z.
__device__ __forceinline__ V3 top_light(V3 d) {
  const V3 w = v3(-d.x, -d.y, -d.z);
  V3 top = cross3(w, v3(0.0f, 0.0f, 1.0f));
  if (sqrtf(dot3(top, top)) < 1e-6f) top = cross3(w, v3(1.0f, 0.0f, 0.0f));
  return normalize3(top);
}

// The march runs in three kernels so that its dominant cost, the light
// marches (two per primary sample), is spread over one lane per
// (pixel, sample, light) instead of serialised inside one lane per pixel:
//   1. march_primary: one lane per pixel walks the primary samples, writes
//      T and D, and records (t_n, A_n, T_{n-1}) of every sample with A_n != 0;
//   2. march_lights: one lane per recorded sample and light computes its
//      transmittance toward the top or bottom light;
//   3. march_accumulate: one lane per pixel sums A_n L_n in sample order.
__global__ __launch_bounds__(256) void march_primary(MarchDev m, CamDev c, MarchBuf buf, float* __restrict__ guide) {
  int i, j;
  tile_pixel(&i, &j);
  if (i >= c.W || j >= c.H) return;
  V3 o, d;
  camera_ray(c, i, j, &o, &d);
  const uint32_t pix = (uint32_t)j * (uint32_t)c.W + (uint32_t)i;
  float u = 0.0f;
  if (m.jitter_on) {
    const uint64_t key = m.seed ^ ((uint64_t)m.frame << 32) ^ (uint64_t)pix;
    u = (float)(uint32_t)(splitmix64(key) >> 40) * (1.0f / 16777216.0f);
  }
  const float h = m.h;
  float tau = 0.0f, Tprev = 1.0f, Tout = 1.0f, D = 0.0f;
  int cnt = 0;
  float t0, t1;
  if (clip_support(m, o, d, &t0, &t1)) {
    const int n0 = max(1, (int)ceilf(t0 / h - u)), n1 = (int)floorf(t1 / h - u);
    bool done = false;
    // gathers of four samples are issued together, then the samples are
    // processed one at a time in order
    for (int nb = n0; nb <= n1 && !done; nb += 4) {
      float sg[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float t = ((float)(nb + q) + u) * h;
        sg[q] = nb + q <= n1 ? sample_sigma(m, o.x + t * d.x, o.y + t * d.y, o.z + t * d.z) : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = nb + q;
        if (done || n > n1) break;
        const float t = ((float)n + u) * h;
        const float sig = sg[q];
        if (D == 0.0f && sig > m.depth_tau) D = (float)n * h;
        tau += sig * h;
        const float T = expf(-tau);
        const float A = m.quadrature == LNM_QUAD_RIEMANN ? Tprev * sig * h : Tprev * -expm1f(-sig * h);
        if (A != 0.0f && cnt < buf.K) {
          const size_t r = (size_t)cnt * buf.P + pix;
          buf.t[r] = t;
          buf.a[r] = A;
          buf.tp[r] = Tprev;
          ++cnt;
        }
        Tprev = T;
        Tout = T;
        if (tau > m.tau_max) {
          Tout = 0.0f;
          done = true;
        }
      }
    }
  }
  buf.cnt[pix] = cnt;
  float* g = guide + 3 * (size_t)pix;
  g[1] = Tout;
  g[2] = D;
}

// grid: (pixel tiles of 16x16, recorded sample index k, light 0 top / 1 bottom)
__global__ __launch_bounds__(256) void march_lights(MarchDev m, CamDev c, MarchBuf buf, int tiles_x) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int i = tx * 16 + (wave & 1) * 8 + (lane & 7), j = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
  if (i >= c.W || j >= c.H) return;
  const uint32_t pix = (uint32_t)j * (uint32_t)c.W + (uint32_t)i;
  const int k = blockIdx.y;
  if ((blockIdx.z == 0 ? m.wt : m.wb) == 0.0f || k >= buf.cnt[pix]) return;
  V3 o, d;
  camera_ray(c, i, j, &o, &d);
  V3 l = top_light(d);
  if (blockIdx.z) l = v3(-l.x, -l.y, -l.z);
  const size_t r = (size_t)k * buf.P + pix;
  const float t = buf.t[r];
  const V3 x = v3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
  buf.tl[(size_t)blockIdx.z * buf.K * buf.P + r] = light_transmittance(m, x, l, m.h, m.tau_max);
}

__global__ __launch_bounds__(256) void march_accumulate(MarchDev m, CamDev c, MarchBuf buf,
                                                        float* __restrict__ guide) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= buf.P) return;
  const int cnt = buf.cnt[p];
  float Ls = 0.0f;
  for (int k = 0; k < cnt; ++k) {
    const size_t r = (size_t)k * buf.P + p;
    // front light: marching toward w retraces the earlier primary samples,
    // so its transmittance is T_{n-1}
    float L = m.wf * buf.tp[r];
    if (m.wt != 0.0f) L += m.wt * buf.tl[r];
    if (m.wb != 0.0f) L += m.wb * buf.tl[(size_t)buf.K * buf.P + r];
    Ls += buf.a[r] * L;
  }
  guide[3 * (size_t)p] = Ls;
}

__device__ __forceinline__ float srgb_encode(float c) {
  return c <= 0.0031308f ? 12.92f * c : 1.055f * powf(c, 1.0f / 2.4f) - 0.055f;
}

__global__ __launch_bounds__(256) void reference_kernel(MarchDev m, CamDev c, int srgb, float* __restrict__ lm) {
  int i, j;
  tile_pixel(&i, &j);
  if (i >= c.W || j >= c.H) return;
  V3 o, d;
  camera_ray(c, i, j, &o, &d);
  const V3 ax[6] = {v3(c.r[0], c.r[1], c.r[2]),    v3(-c.r[0], -c.r[1], -c.r[2]),
                    v3(c.u[0], c.u[1], c.u[2]),    v3(-c.u[0], -c.u[1], -c.u[2]),
                    v3(-c.f[0], -c.f[1], -c.f[2]), v3(c.f[0], c.f[1], c.f[2])};
  const float h = m.h;
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float tau = 0.0f, Tprev = 1.0f, t0, t1;
  if (clip_support(m, o, d, &t0, &t1)) {
    const int n0 = max(1, (int)ceilf(t0 / h)), n1 = (int)floorf(t1 / h);
    for (int n = n0; n <= n1; ++n) {
      const float t = (float)n * h;
      const V3 x = v3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
      const float sig = sample_sigma(m, x.x, x.y, x.z);
      tau += sig * h;
      const float A = Tprev * -expm1f(-sig * h);
      if (A > 0.0f) {
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[a] += A * light_transmittance(m, x, ax[a], h, m.tau_max);
      }
      Tprev = expf(-tau);
      if (tau > m.tau_max) break;
    }
  }
  float* out = lm + 6 * ((size_t)j * c.W + i);
#pragma unroll
  for (int a = 0; a < 6; ++a) out[a] = srgb ? srgb_encode(acc[a]) : acc[a];
}

}  // namespace

int march_capacity(const MarchDev& m) {
  double d2 = 0.0;
  const int n[3] = {m.nx, m.ny, m.nz};
  for (int a = 0; a < 3; ++a) d2 += (1.0 + 1.0 / n[a]) * (1.0 + 1.0 / n[a]);
  return (int)std::ceil(std::sqrt(d2) / (double)m.h) + 2;
}

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }

size_t march_scratch_bytes(int K, int P) {
  const size_t plane = a256(sizeof(float) * (size_t)K * P);
  return 5 * plane + a256(sizeof(int) * (size_t)P);
}

MarchBuf march_buffers(void* ws, int K, int P) {
  char* p = static_cast<char*>(ws);
  const size_t plane = a256(sizeof(float) * (size_t)K * P);
  MarchBuf b;
  b.t = reinterpret_cast<float*>(p);
  b.a = reinterpret_cast<float*>(p + plane);
  b.tp = reinterpret_cast<float*>(p + 2 * plane);
  b.tl = reinterpret_cast<float*>(p + 3 * plane);  // two planes
  b.cnt = reinterpret_cast<int*>(p + 5 * plane);
  b.K = K;
  b.P = P;
  return b;
}

hipError_t launch_march(const MarchDev& m, const CamDev& cam, const MarchBuf& buf, float* guide, hipStream_t s) {
  const int tiles_x = (cam.W + 15) / 16, tiles_y = (cam.H + 15) / 16;
  hipLaunchKernelGGL(march_primary, dim3(tiles_x, tiles_y), dim3(256), 0, s, m, cam, buf, guide);
  if (m.wt != 0.0f || m.wb != 0.0f)
    hipLaunchKernelGGL(march_lights, dim3(tiles_x * tiles_y, buf.K, 2), dim3(256), 0, s, m, cam, buf, tiles_x);
  hipLaunchKernelGGL(march_accumulate, dim3((buf.P + 255) / 256), dim3(256), 0, s, m, cam, buf, guide);
  return hipGetLastError();
}

hipError_t launch_reference(const MarchDev& m, const CamDev& cam, int srgb, float* lm, hipStream_t s) {
  dim3 grid((cam.W + 15) / 16, (cam.H + 15) / 16);
  hipLaunchKernelGGL(reference_kernel, grid, dim3(256), 0, s, m, cam, srgb, lm);
  return hipGetLastError();
}

}  // namespace lnm
