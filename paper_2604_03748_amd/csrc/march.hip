// Guiding-map ray march (Algorithm 1, Section 4.2) and fine-step six-way
// reference lightmaps, fp32.
//
// The march first copies the density grid into 4^3-cell bricks (so the 8
// corners of a trilinear sample are one short span of one 512-byte slot) and
// then runs three kernels (see march_primary).  Pixels are handed out in
// 16x16 tiles, an 8x8 sub-tile per wavefront, so the 64 rays of a wave are
// spatially coherent and their gathers share cache lines; tiles are ordered
// so that each XCD takes one band of the screen.
#include <cmath>

#include "internal.h"
#include "ray.h"

namespace lnm {
namespace {

// SplitMix64 output for state s: the finaliser applied to s + golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// sigma(p): sigma_scale x zero-border cell-centred trilinear interpolation.
// This form reads the caller's linear grid: corner indices are clamped into
// the grid and corners outside it get weight zero, so every load is in
// bounds.
__device__ __forceinline__ float sample_sigma_linear(const MarchDev& m, float px, float py, float pz) {
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

// Bricked grid: index i' = i + 1 over [0, n + 1] (a zero layer on each side),
// cut into bricks of 4 cells per axis that also store the next layer
// (5 x 5 x 5 values in a 128-float slot).  The 8 corners of the cell holding
// a point are then in one brick at fixed offsets, and the zero layers make
// the grid's zero border explicit.  Same value as sample_sigma_linear.
constexpr int kBrickSlot = 128;
__device__ __forceinline__ float sample_sigma(const MarchDev& m, float px, float py, float pz) {
  const float gx = px * (float)m.nx - 0.5f, gy = py * (float)m.ny - 0.5f, gz = pz * (float)m.nz - 0.5f;
  if (!(gx > -1.0f && gy > -1.0f && gz > -1.0f && gx < (float)m.nx && gy < (float)m.ny && gz < (float)m.nz))
    return 0.0f;
  const float fx0 = floorf(gx), fy0 = floorf(gy), fz0 = floorf(gz);
  const int i = (int)fx0 + 1, j = (int)fy0 + 1, k = (int)fz0 + 1;  // in [0, n]
  const float fx = gx - fx0, fy = gy - fy0, fz = gz - fz0;
  const int brick = ((k >> 2) * m.nby + (j >> 2)) * m.nbx + (i >> 2);
  const float* r = m.brick + (size_t)brick * kBrickSlot + ((k & 3) * 25 + (j & 3) * 5 + (i & 3));
  const float c00 = (1.0f - fx) * r[0] + fx * r[1];
  const float c10 = (1.0f - fx) * r[5] + fx * r[6];
  const float c01 = (1.0f - fx) * r[25] + fx * r[26];
  const float c11 = (1.0f - fx) * r[30] + fx * r[31];
  const float v = (1.0f - fz) * ((1.0f - fy) * c00 + fy * c10) + fz * ((1.0f - fy) * c01 + fy * c11);
  return m.sigma_scale * v;
}

// Fill the bricked grid from the caller's linear grid (HBM-bound copy; once
// per grid).  One lane per slot entry; entries 125..127 are padding.
__global__ __launch_bounds__(256) void relayout_bricks(const float* __restrict__ rho, int nx, int ny, int nz, int nbx,
                                                       int nby, int nbz, float* __restrict__ brick) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)nbx * nby * nbz * kBrickSlot) return;
  const int s = e % kBrickSlot;
  const long b = e / kBrickSlot;
  float v = 0.0f;
  if (s < 125) {
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / ((long)nbx * nby);
    const int i = 4 * bx + s % 5 - 1, j = 4 * by + (s / 5) % 5 - 1, k = 4 * bz + s / 25 - 1;
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) v = rho[((size_t)k * ny + j) * nx + i];
  }
  brick[e] = v;
}

template <bool BRICK>
__device__ __forceinline__ float sample(const MarchDev& m, float px, float py, float pz) {
  return BRICK ? sample_sigma(m, px, py, pz) : sample_sigma_linear(m, px, py, pz);
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

__device__ __forceinline__ int light_steps(const MarchDev& m, V3 x, V3 l, float h) {
  const float s1 = exit_distance(m, x, l);
  return s1 > 0.0f ? (int)floorf(s1 / h) : 0;
}

// Transmittance from x toward l: exp(-h sum_k sigma(x + k h l)) over the
// points inside the support box, 0 once the optical depth passes tau_max.
template <bool BRICK>
__device__ __forceinline__ float light_transmittance(const MarchDev& m, V3 x, V3 l, float h, float tau_max) {
  const int kmax = light_steps(m, x, l, h);
  const float lim = tau_max / h;
  float acc = 0.0f;
  // four samples' gathers are issued together; they are summed and tested
  // against the termination limit one at a time, in order
  for (int k = 1; k <= kmax; k += 4) {
    float s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float t = (float)(k + j) * h;
      s[j] = k + j <= kmax ? sample<BRICK>(m, x.x + t * l.x, x.y + t * l.y, x.z + t * l.z) : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc += s[j];
      if (acc > lim) return 0.0f;
    }
  }
  return expf(-acc * h);
}

// The two side-light marches (+l and -l) of one point in one loop, two
// samples of each per iteration, so that four gathers are in flight.  Each
// march sums its samples in order and stops at its own termination limit;
// the results equal two calls of light_transmittance.
__device__ __forceinline__ void top_bottom_transmittance(const MarchDev& m, V3 x, V3 l, bool want_t, bool want_b,
                                                         float* Tt, float* Tb) {
  const float h = m.h, lim = m.tau_max / h;
  int kt = want_t ? light_steps(m, x, l, h) : 0;
  int kb = want_b ? light_steps(m, x, v3(-l.x, -l.y, -l.z), h) : 0;
  float at = 0.0f, ab = 0.0f;
  bool dead_t = false, dead_b = false;
  for (int k = 1; k <= kt || k <= kb; k += 2) {
    float st[2], sb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const float t = (float)(k + q) * h;
      st[q] = k + q <= kt ? sample<true>(m, x.x + t * l.x, x.y + t * l.y, x.z + t * l.z) : 0.0f;
      sb[q] = k + q <= kb ? sample<true>(m, x.x - t * l.x, x.y - t * l.y, x.z - t * l.z) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      at += st[q];
      dead_t = dead_t || at > lim;
      ab += sb[q];
      dead_b = dead_b || ab > lim;
    }
    if (dead_t) kt = 0;
    if (dead_b) kb = 0;
  }
  *Tt = dead_t ? 0.0f : expf(-at * h);
  *Tb = dead_b ? 0.0f : expf(-ab * h);
}

__device__ __forceinline__ void tile_pixel(int* i, int* j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  *i = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  *j = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
}

// Pixel of this lane under an XCD-aware tile order.  Workgroups are handed to
// the 8 XCDs round robin by their linear id, so XCD e runs the blocks with
// blockIdx.x = e (mod 8); the map gives those blocks one contiguous band of
// 16x16 tiles (of screen columns, or rows when the light marches run
// horizontally on screen), so each XCD's L2 holds the slab of the volume its
// band sees instead of the whole grid.
__device__ __forceinline__ bool banded_pixel(const TileMap& tm, int* i, int* j) {
  const int b = blockIdx.x;
  const int L = (b & 7) * tm.per_xcd + (b >> 3);
  if (L >= tm.tiles_x * tm.tiles_y) return false;
  int tx, ty;
  if (tm.band_rows) {
    ty = L / tm.tiles_x;
    tx = L - ty * tm.tiles_x;
  } else {
    tx = L / tm.tiles_y;
    ty = L - tx * tm.tiles_y;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  *i = tx * 16 + (wave & 1) * 8 + (lane & 7);
  *j = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
  return true;
}

// Top surrogate light of a ray: normalize(w x z), or normalize(w x x) when w
// is parallel to z.
__device__ __forceinline__ V3 top_light(V3 d) {
  const V3 w = v3(-d.x, -d.y, -d.z);
  V3 top = cross3(w, v3(0.0f, 0.0f, 1.0f));
  if (sqrtf(dot3(top, top)) < 1e-6f) top = cross3(w, v3(1.0f, 0.0f, 0.0f));
  return normalize3(top);
}

// First side light of the chosen set: top, or left = normalize(w x top).
__device__ __forceinline__ V3 side_light(V3 d, int light_set) {
  const V3 top = top_light(d);
  return light_set == LNM_LIGHTS_LEFT_RIGHT ? normalize3(cross3(v3(-d.x, -d.y, -d.z), top)) : top;
}

// The march runs in three kernels so that its dominant cost, the light
// marches (two per primary sample), is spread over one lane per
// (pixel, sample) instead of serialised inside one lane per pixel:
//   1. march_primary: one lane per pixel walks the primary samples, writes
//      T and D, and records (t_n, A_n, T_{n-1}) of every sample with A_n != 0;
//   2. march_lights: one lane per recorded sample marches toward the top and
//      bottom lights and stores A_n L_n;
//   3. march_accumulate: one lane per pixel sums A_n L_n in sample order.
// All three read the bricked grid filled by relayout_bricks.
__global__ __launch_bounds__(256) void march_primary(MarchDev m, CamDev c, TileMap tm, MarchBuf buf,
                                                     float* __restrict__ guide) {
  int i, j;
  if (!banded_pixel(tm, &i, &j) || i >= c.W || j >= c.H) return;
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
        sg[q] = nb + q <= n1 ? sample<true>(m, o.x + t * d.x, o.y + t * d.y, o.z + t * d.z) : 0.0f;
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

// grid: (banded pixel tiles, recorded sample index k)
__global__ __launch_bounds__(256) void march_lights(MarchDev m, CamDev c, TileMap tm, MarchBuf buf) {
  int i, j;
  if (!banded_pixel(tm, &i, &j) || i >= c.W || j >= c.H) return;
  const uint32_t pix = (uint32_t)j * (uint32_t)c.W + (uint32_t)i;
  const int k = blockIdx.y;
  if (k >= buf.cnt[pix]) return;
  const size_t r = (size_t)k * buf.P + pix;
  // front light: marching toward w retraces the earlier primary samples, so
  // its transmittance is T_{n-1}
  float L = m.wf * buf.tp[r];
  if (m.wt != 0.0f || m.wb != 0.0f) {
    V3 o, d;
    camera_ray(c, i, j, &o, &d);
    const float t = buf.t[r];
    const V3 x = v3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
    float Tt, Tb;
    top_bottom_transmittance(m, x, side_light(d, m.light_set), m.wt != 0.0f, m.wb != 0.0f, &Tt, &Tb);
    if (m.wt != 0.0f) L += m.wt * Tt;
    if (m.wb != 0.0f) L += m.wb * Tb;
  }
  buf.al[r] = buf.a[r] * L;
}

__global__ __launch_bounds__(256) void march_accumulate(MarchBuf buf, float* __restrict__ guide) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= buf.P) return;
  const int cnt = buf.cnt[p];
  const float* al = buf.al + p;
  const size_t P = (size_t)buf.P;
  float Ls = 0.0f;
  int k = 0;
  // eight loads in flight, summed in sample order
  for (; k + 8 <= cnt; k += 8) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = al[(size_t)(k + q) * P];
#pragma unroll
    for (int q = 0; q < 8; ++q) Ls += v[q];
  }
  for (; k < cnt; ++k) Ls += al[(size_t)k * P];
  guide[3 * (size_t)p] = Ls;
}

__device__ __forceinline__ float srgb_encode(float c) {
  return c <= 0.0031308f ? 12.92f * c : 1.055f * powf(c, 1.0f / 2.4f) - 0.055f;
}

// Fine-step reference: reads the caller's linear grid (it takes no scratch).
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
      const float sig = sample<false>(m, x.x, x.y, x.z);
      tau += sig * h;
      const float A = Tprev * -expm1f(-sig * h);
      if (A > 0.0f) {
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[a] += A * light_transmittance<false>(m, x, ax[a], h, m.tau_max);
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
static int bricks_along(int n) { return (n >> 2) + 1; }
static size_t brick_bytes(const MarchDev& m) {
  return sizeof(float) * kBrickSlot * (size_t)bricks_along(m.nx) * bricks_along(m.ny) * bricks_along(m.nz);
}

size_t march_scratch_bytes(const MarchDev& m, int K, int P) {
  const size_t plane = a256(sizeof(float) * (size_t)K * P);
  return 4 * plane + a256(sizeof(int) * (size_t)P) + a256(brick_bytes(m));
}

MarchBuf march_buffers(void* ws, const MarchDev& m, int K, int P) {
  char* p = static_cast<char*>(ws);
  const size_t plane = a256(sizeof(float) * (size_t)K * P);
  MarchBuf b;
  b.t = reinterpret_cast<float*>(p);
  b.a = reinterpret_cast<float*>(p + plane);
  b.tp = reinterpret_cast<float*>(p + 2 * plane);
  b.al = reinterpret_cast<float*>(p + 3 * plane);
  b.cnt = reinterpret_cast<int*>(p + 4 * plane);
  b.brick = reinterpret_cast<float*>(p + 4 * plane + a256(sizeof(int) * (size_t)P));
  b.nbx = bricks_along(m.nx);
  b.nby = bricks_along(m.ny);
  b.nbz = bricks_along(m.nz);
  b.K = K;
  b.P = P;
  return b;
}

// Band screen rows instead of columns when the top light of the central ray
// runs more horizontally than vertically on screen.
static TileMap tile_map(const CamDev& c) {
  TileMap tm;
  tm.tiles_x = (c.W + 15) / 16;
  tm.tiles_y = (c.H + 15) / 16;
  tm.per_xcd = (tm.tiles_x * tm.tiles_y + 7) / 8;
  const double w[3] = {-c.f[0], -c.f[1], -c.f[2]};
  double top[3] = {w[1], -w[0], 0.0};  // w x z
  if (std::sqrt(top[0] * top[0] + top[1] * top[1]) < 1e-6) {
    top[0] = 0.0;  // w x x
    top[1] = w[2];
    top[2] = -w[1];
  }
  const double along_r = std::fabs(top[0] * c.r[0] + top[1] * c.r[1] + top[2] * c.r[2]);
  const double along_u = std::fabs(top[0] * c.u[0] + top[1] * c.u[1] + top[2] * c.u[2]);
  tm.band_rows = along_r > along_u ? 1 : 0;
  return tm;
}

hipError_t launch_march(const MarchDev& m0, const CamDev& cam, const MarchBuf& buf, float* guide, hipStream_t s) {
  MarchDev m = m0;
  m.brick = buf.brick;
  m.nbx = buf.nbx;
  m.nby = buf.nby;
  m.nbz = buf.nbz;
  const long entries = (long)buf.nbx * buf.nby * buf.nbz * kBrickSlot;
  hipLaunchKernelGGL(relayout_bricks, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, s, m.rho, m.nx, m.ny,
                     m.nz, buf.nbx, buf.nby, buf.nbz, buf.brick);
  const TileMap tm = tile_map(cam);
  hipLaunchKernelGGL(march_primary, dim3(8 * tm.per_xcd), dim3(256), 0, s, m, cam, tm, buf, guide);
  hipLaunchKernelGGL(march_lights, dim3(8 * tm.per_xcd, buf.K), dim3(256), 0, s, m, cam, tm, buf);
  hipLaunchKernelGGL(march_accumulate, dim3((buf.P + 255) / 256), dim3(256), 0, s, buf, guide);
  return hipGetLastError();
}

hipError_t launch_reference(const MarchDev& m, const CamDev& cam, int srgb, float* lm, hipStream_t s) {
  dim3 grid((cam.W + 15) / 16, (cam.H + 15) / 16);
  hipLaunchKernelGGL(reference_kernel, grid, dim3(256), 0, s, m, cam, srgb, lm);
  return hipGetLastError();
}

}  // namespace lnm
