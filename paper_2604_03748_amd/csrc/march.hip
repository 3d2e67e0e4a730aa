// Guiding-map ray march (Algorithm 1, Section 4.2) and fine-step six-way
// reference lightmaps, fp32.
//
// The march first copies the density grid into 4^3-cell bricks (so the 8
// corners of a trilinear sample are one short span of one 512-byte slot),
// cutting the screen's 8x8 tiles into eight bands of equal estimated work on
// the way, then runs three kernels (see march_primary): the primary march
// (four lanes per pixel, one band per XCD), the light marches (one lane per
// recorded sample and light, an eighth of the records per XCD; on large
// grids after a scatter of the records into z order) and the accumulation.
// The fine-step reference kernel reads the linear grid.
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
  const float gx0 = px * (float)m.nx - 0.5f, gy0 = py * (float)m.ny - 0.5f, gz0 = pz * (float)m.nz - 0.5f;
  const bool inside = gx0 > -1.0f && gy0 > -1.0f && gz0 > -1.0f && gx0 < (float)m.nx && gy0 < (float)m.ny &&
                      gz0 < (float)m.nz;
  // branch-free: outside points are moved to the origin for the loads and give 0
  const float gx = inside ? gx0 : 0.0f, gy = inside ? gy0 : 0.0f, gz = inside ? gz0 : 0.0f;
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
  return m.sigma_scale * v * (inside ? 1.0f : 0.0f);
}

// Bricked grid (kBrickSlot): index i' = i + 1 over [0, n + 1] (a zero layer
// on each side), cut into bricks of 4 cells per axis that also store the
// next layer (5 x 5 x 5 values in a 128-float slot).  The 8 corners of the
// cell holding a point are then in one brick at fixed offsets, and the zero
// layers make the grid's zero border explicit.  Same value as
// sample_sigma_linear.
//
// The sample is branch-free so that a caller's batch of samples issues all
// its loads before waiting on any: a point outside the support box is
// moved to the grid origin for the loads and its value discarded.  Slot
// offsets are 32-bit (the bricked grid is limited to 4 GiB).

// Address and interpolation weights of one bricked sample (split from the
// loads so that callers can issue the loads of several samples together).
struct BrickTap {
  const float* r;    // corner (0,0,0) in its slot; the others at +1, +5, +6, +25, +26, +30, +31
  float fx, fy, fz;  // fractions
  float mask;        // 1 inside the support box, else 0
};

__device__ __forceinline__ BrickTap brick_tap(const MarchDev& m, float px, float py, float pz) {
  const float gx = fmaf(px, (float)m.nx, -0.5f), gy = fmaf(py, (float)m.ny, -0.5f), gz = fmaf(pz, (float)m.nz, -0.5f);
  const bool inside = gx > -1.0f && gy > -1.0f && gz > -1.0f && gx < (float)m.nx && gy < (float)m.ny &&
                      gz < (float)m.nz;
  // outside points are moved to the origin for the loads (their value is masked)
  const float cx = inside ? gx : 0.0f, cy = inside ? gy : 0.0f, cz = inside ? gz : 0.0f;
  const float fx0 = floorf(cx), fy0 = floorf(cy), fz0 = floorf(cz);
  const uint32_t i = (uint32_t)((int)fx0 + 1), j = (uint32_t)((int)fy0 + 1), k = (uint32_t)((int)fz0 + 1);
  const uint32_t brick = ((k >> 2) * (uint32_t)m.nby + (j >> 2)) * (uint32_t)m.nbx + (i >> 2);
  BrickTap t;
  t.r = m.brick + (brick * (uint32_t)kBrickSlot + ((k & 3u) * 25u + (j & 3u) * 5u + (i & 3u)));
  t.fx = cx - fx0;
  t.fy = cy - fy0;
  t.fz = cz - fz0;
  t.mask = inside ? 1.0f : 0.0f;
  return t;
}

struct BrickVals {
  float v[8];
};
__device__ __forceinline__ BrickVals brick_load(const BrickTap& t) {
  BrickVals c;
  c.v[0] = t.r[0];
  c.v[1] = t.r[1];
  c.v[2] = t.r[5];
  c.v[3] = t.r[6];
  c.v[4] = t.r[25];
  c.v[5] = t.r[26];
  c.v[6] = t.r[30];
  c.v[7] = t.r[31];
  return c;
}
// Trilinear value of the 8 corners (v[0] at (i, j, k), then +x, +y, +x+y,
// and the same at k + 1) with fractions fx, fy, fz: each linear blend
// (1 - f) a + f b written as one fused multiply-add, so that every sampler
// (bricks in global memory, grid planes in LDS) computes it identically.
__device__ __forceinline__ float lerp1(float a, float b, float f) { return fmaf(f, b, (1.0f - f) * a); }
__device__ __forceinline__ float trilerp(const float (&v)[8], float fx, float fy, float fz) {
  const float c00 = lerp1(v[0], v[1], fx), c10 = lerp1(v[2], v[3], fx);
  const float c01 = lerp1(v[4], v[5], fx), c11 = lerp1(v[6], v[7], fx);
  return lerp1(lerp1(c00, c10, fy), lerp1(c01, c11, fy), fz);
}
// sigma_scale x the trilinear value, times the inside mask (a multiply, not a
// select, which the compiler would turn back into a branch around the loads)
__device__ __forceinline__ float brick_lerp(const MarchDev& m, const BrickTap& t, const BrickVals& c) {
  return m.sigma_scale * trilerp(c.v, t.fx, t.fy, t.fz) * t.mask;
}
// The trilinear value on a flat light march, whose z fraction is the same at
// every sample: the two planes are blended first, b + fz d with
// d = above - below (one fused multiply-add per corner, the cell-order
// planes in LDS hold d), then along x and y.  Corners (below, d) at (i, j),
// (i + 1, j), (i, j + 1), (i + 1, j + 1).
__device__ __forceinline__ float flat_lerp(float b00, float d00, float b10, float d10, float b01, float d01,
                                           float b11, float d11, float fx, float fy, float fz) {
  const float e00 = fmaf(fz, d00, b00), e10 = fmaf(fz, d10, b10);
  const float e01 = fmaf(fz, d01, b01), e11 = fmaf(fz, d11, b11);
  return lerp1(lerp1(e00, e10, fx), lerp1(e01, e11, fx), fy);
}
__device__ __forceinline__ float brick_lerp_flat(const MarchDev& m, const BrickTap& t, const BrickVals& c) {
  const float(&v)[8] = c.v;
  return m.sigma_scale *
         flat_lerp(v[0], v[4] - v[0], v[1], v[5] - v[1], v[2], v[6] - v[2], v[3], v[7] - v[3], t.fx, t.fy, t.fz) *
         t.mask;
}

__device__ __forceinline__ float sample_sigma(const MarchDev& m, float px, float py, float pz) {
  const BrickTap t = brick_tap(m, px, py, pz);
  return brick_lerp(m, t, brick_load(t));
}

// N samples: all addresses, then all loads, then all interpolations.
template <int N>
__device__ __forceinline__ void sample_batch(const MarchDev& m, const float (&px)[N], const float (&py)[N],
                                             const float (&pz)[N], float (&out)[N]) {
  BrickTap t[N];
  BrickVals c[N];
#pragma unroll
  for (int q = 0; q < N; ++q) t[q] = brick_tap(m, px[q], py[q], pz[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) c[q] = brick_load(t[q]);
  // keep the scheduler from sinking the loads next to their uses
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = brick_lerp(m, t[q], c[q]);
}

// The z part of brick_tap for points that share one z (a light march whose
// direction has no z component): computed once per march, selected per
// sample (an outside point takes the origin's values, as in brick_tap), so
// the taps are the same, bit for bit.
struct FlatZ {
  bool in;        // gz inside (-1, nz)
  uint32_t zrow;  // (k >> 2) * nby for the point's cell index k
  uint32_t zoff;  // (k & 3) * 25
  float fz;
};
__device__ __forceinline__ FlatZ flat_z(const MarchDev& m, float pz) {
  const float gz = fmaf(pz, (float)m.nz, -0.5f);
  FlatZ z;
  z.in = gz > -1.0f && gz < (float)m.nz;
  const float cz = z.in ? gz : 0.0f, fz0 = floorf(cz);
  const uint32_t k = (uint32_t)((int)fz0 + 1);
  z.zrow = (k >> 2) * (uint32_t)m.nby;
  z.zoff = (k & 3u) * 25u;
  z.fz = cz - fz0;
  return z;
}
__device__ __forceinline__ BrickTap brick_tap_flat(const MarchDev& m, float px, float py, const FlatZ& z) {
  const float gx = fmaf(px, (float)m.nx, -0.5f), gy = fmaf(py, (float)m.ny, -0.5f);
  const bool inside = z.in && gx > -1.0f && gy > -1.0f && gx < (float)m.nx && gy < (float)m.ny;
  const float cx = inside ? gx : 0.0f, cy = inside ? gy : 0.0f;
  const float fx0 = floorf(cx), fy0 = floorf(cy);
  const uint32_t i = (uint32_t)((int)fx0 + 1), j = (uint32_t)((int)fy0 + 1);
  // the origin's cell index is k = 1: row 0, offset 25
  const uint32_t brick = ((inside ? z.zrow : 0u) + (j >> 2)) * (uint32_t)m.nbx + (i >> 2);
  BrickTap t;
  t.r = m.brick + (brick * (uint32_t)kBrickSlot + ((inside ? z.zoff : 25u) + (j & 3u) * 5u + (i & 3u)));
  t.fx = cx - fx0;
  t.fy = cy - fy0;
  t.fz = inside ? z.fz : 0.0f;
  t.mask = inside ? 1.0f : 0.0f;
  return t;
}
template <int N>
__device__ __forceinline__ void sample_batch_flat(const MarchDev& m, const float (&px)[N], const float (&py)[N],
                                                  const FlatZ& z, float (&out)[N]) {
  BrickTap t[N];
  BrickVals c[N];
#pragma unroll
  for (int q = 0; q < N; ++q) t[q] = brick_tap_flat(m, px[q], py[q], z);
#pragma unroll
  for (int q = 0; q < N; ++q) c[q] = brick_load(t[q]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < N; ++q) out[q] = brick_lerp_flat(m, t[q], c[q]);
}

// Fill the bricked grid from the caller's linear grid (HBM-bound copy; once
// per march, or once per grid with lnm_make_bricks).  Workgroup = up to
// kRelayBricks consecutive bricks along x in kRelayY brick rows at one bz:
// it stages the source rows they cover (4 kRelayY + 1 y rows x 5 z planes
// of 4 kRelayBricks + 1 floats) in LDS, the rows read as one flat run of
// entries so every lane issues all its loads together (out-of-grid entries
// read a valid address and are zeroed), then writes each brick row's slots
// (contiguous) with coalesced stores.  Slot entries 125..127 are zero
// padding.  Runs of 11 bricks split a row of 33 (the 128^3 grid's) evenly;
// at 128^3 the relayout took 8.4 us against 8.9 with runs of 17 (and 10.4
// with runs of 31, which left a 2-brick workgroup per row); two brick rows
// per workgroup took 9.1.
constexpr int kRelayBricks = 11, kRelayRow = 4 * kRelayBricks + 1, kRelayY = 1;
constexpr int kRelayRows = 5 * (4 * kRelayY + 1), kRelayLoads = (kRelayRows * kRelayRow + 255) / 256;
__device__ __forceinline__ void relayout_block(const float* __restrict__ rho, int nx, int ny, int nz, int nbx, int nby,
                                               float* __restrict__ brick, float (&rows)[kRelayRows][kRelayRow],
                                               int bxb, int byb, int bz) {
  constexpr int RY = 4 * kRelayY + 1;  // staged y rows per z plane
  const int bx0 = bxb * kRelayBricks, by0 = byb * kRelayY;
  float* flat = &rows[0][0];
  float v[kRelayLoads];
#pragma unroll
  for (int q = 0; q < kRelayLoads; ++q) {
    const int e = (int)threadIdx.x + 256 * q, r = e / kRelayRow, x = e - r * kRelayRow;
    const int i = 4 * bx0 + x - 1, j = 4 * by0 + r % RY - 1, k = 4 * bz + r / RY - 1;
    const bool ok = e < kRelayRows * kRelayRow && i < nx && j < ny && k < nz && i >= 0 && j >= 0 && k >= 0;
    const size_t src = ok ? ((size_t)k * ny + j) * nx + i : 0;
    v[q] = rho[src] * (ok ? 1.0f : 0.0f);
  }
#pragma unroll
  for (int q = 0; q < kRelayLoads; ++q) {
    const int e = (int)threadIdx.x + 256 * q;
    if (e < kRelayRows * kRelayRow) flat[e] = v[q];
  }
  __syncthreads();
  const int nb = min(kRelayBricks, nbx - bx0), nyb = min(kRelayY, nby - by0);
  // a thread keeps one slot entry s of every brick it writes (256 threads,
  // 128-entry slots), so its row and column in the staged rows are fixed
  static_assert(256 % kBrickSlot == 0, "slot entries per thread");
  const int s = threadIdx.x & (kBrickSlot - 1);
  const bool live = s < 125;
  const int rr = live ? (s / 25) * RY + (s / 5) % 5 : 0, cc = s % 5;
  for (int yb = 0; yb < nyb; ++yb) {
    float* out = brick + (((size_t)bz * nby + by0 + yb) * nbx + bx0) * kBrickSlot;
    for (int b = threadIdx.x / kBrickSlot; b < nb; b += 256 / kBrickSlot)
      out[b * kBrickSlot + s] = live ? rows[rr + 4 * yb][4 * b + cc] : 0.0f;
  }
}

__global__ __launch_bounds__(256) void relayout_bricks(const float* __restrict__ rho, int nx, int ny, int nz, int nbx,
                                                       int nby, float* __restrict__ brick) {
  __shared__ float rows[kRelayRows][kRelayRow];
  relayout_block(rho, nx, ny, nz, nbx, nby, brick, rows, blockIdx.x, blockIdx.y, blockIdx.z);
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
      const float v = sample<BRICK>(m, x.x + t * l.x, x.y + t * l.y, x.z + t * l.z);
      s[j] = k + j <= kmax ? v : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc += s[j];
      if (acc > lim) return 0.0f;
    }
  }
  return expf(-acc * h);
}

// Transmittance toward one light on the bricked grid: the samples of the
// march are gathered four at a time (all loads issued before any is used)
// and summed in order; the march stops at the termination limit.
// FLAT: l has no z component, so every sample has the z of x (x.z + t * 0
// is x.z exactly): the z part of the taps is computed once, and the
// interpolation blends the two planes first (flat_lerp, the same arithmetic
// as the cell order's LDS march).  Otherwise the samples are those of
// light_transmittance<true>.
template <bool FLAT>
__device__ __forceinline__ float light_transmittance_batched(const MarchDev& m, V3 x, V3 l) {
  const float h = m.h, lim = m.tau_max / h;
  const int kmax = light_steps(m, x, l, h);
  const FlatZ fz = flat_z(m, FLAT ? x.z : 0.0f);
  float acc = 0.0f;
  for (int k = 1; k <= kmax; k += 4) {
    float px[4], py[4], pz[4], sv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float t = (float)(k + q) * h;
      px[q] = fmaf(t, l.x, x.x);
      py[q] = fmaf(t, l.y, x.y);
      pz[q] = fmaf(t, l.z, x.z);
    }
    if constexpr (FLAT)
      sample_batch_flat<4>(m, px, py, fz, sv);
    else
      sample_batch<4>(m, px, py, pz, sv);
    // the depth is tested after each sample, the branch taken once per batch
    bool over = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc += k + q <= kmax ? sv[q] : 0.0f;
      over |= acc > lim;
    }
    if (over) return 0.0f;
  }
  return expf(-acc * h);
}

// The light march of a flat light (no z component) with the density of its
// sample's z cell staged in LDS: pl[ny + 3][nx + 3] pairs (value of the grid
// plane below the cell, value above minus value below), index i + 1 holding
// grid column i, with a zero border (one entry before the grid, two after),
// so one 8-byte read gives a corner of both planes.  The tap coordinates are
// clamped to [-1, n]: a point outside the grid then reads border zeros with
// weight one (and finite entries with weight zero), which is the zero the
// bricked sampler's inside mask gives it.  Inside the grid the taps, weights
// and sums are those of light_transmittance_batched<true>, so the result is
// the same bit for bit; the corners come from LDS instead of the bricks.
struct LdsTap {
  int o;  // LDS pair index of corner (i, j)
  float fx, fy;
};
__device__ __forceinline__ LdsTap lds_tap(const MarchDev& m, float px, float py, int pitch) {
  const float gx = fmaf(px, (float)m.nx, -0.5f), gy = fmaf(py, (float)m.ny, -0.5f);
  const float cx = __builtin_amdgcn_fmed3f(gx, -1.0f, (float)m.nx);
  const float cy = __builtin_amdgcn_fmed3f(gy, -1.0f, (float)m.ny);
  const float fx0 = floorf(cx), fy0 = floorf(cy);
  LdsTap t;
  // (fy0 + 1) pitch + fx0 + 1, exact in fp32 (under 2^24)
  t.o = (int)fmaf(fy0, (float)pitch, fx0) + pitch + 1;
  t.fx = cx - fx0;
  t.fy = cy - fy0;
  return t;
}
__device__ __forceinline__ float light_transmittance_lds(const MarchDev& m, V3 x, V3 l, const float2* __restrict__ pl,
                                                         int pitch) {
  const float h = m.h, lim = m.tau_max / h;
  const int kmax = light_steps(m, x, l, h);
  const FlatZ fz = flat_z(m, x.z);
  float acc = 0.0f;
  for (int k = 1; k <= kmax; k += 4) {
    LdsTap t[4];
    float2 c[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float tt = (float)(k + q) * h;
      t[q] = lds_tap(m, fmaf(tt, l.x, x.x), fmaf(tt, l.y, x.y), pitch);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float2* a = pl + t[q].o;
      c[q][0] = a[0];
      c[q][1] = a[1];
      c[q][2] = a[pitch];
      c[q][3] = a[pitch + 1];
    }
    // the depth is tested after each sample, the branch taken once per batch
    bool over = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float sv = m.sigma_scale * flat_lerp(c[q][0].x, c[q][0].y, c[q][1].x, c[q][1].y, c[q][2].x, c[q][2].y,
                                                 c[q][3].x, c[q][3].y, t[q].fx, t[q].fy, fz.fz);
      acc += k + q <= kmax ? sv : 0.0f;
      over |= acc > lim;
    }
    if (over) return 0.0f;
  }
  return expf(-acc * h);
}

__device__ __forceinline__ void tile_pixel(int* i, int* j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  *i = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  *j = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
}

// Screen tiles of 8x8 pixels are numbered in band order: L runs down the
// screen columns of tiles (or along the rows when the light marches run
// horizontally on screen), so a contiguous range of L is a screen band whose
// light marches stay inside one slab of the volume.  A workgroup of 256
// lanes covers one tile with four lanes per pixel; each wavefront an 8x2
// block.

// z bucket of a sample point: its trilinear cell k' = floor(gz) + 1 (the
// cell between grid planes k' - 1 and k'), in z order grouped by brick layer
// (the bricks hold cells in layers k' / 4), capped at the last bucket.  A
// side light has no z component, so a light march stays in its sample's
// cell (the fallback lights of a ray along z and the left/right set do not;
// the order then only loses locality).
__device__ __forceinline__ int z_bucket(const MarchDev& m, float pz) {
  const float gz = fminf(fmaxf(fmaf(pz, (float)m.nz, -0.5f), -1.0f), (float)m.nz);
  const int cell = (int)floorf(gz) + 1;
  return min(m.zorder == kOrderCells ? cell : cell >> 2, kZBuckets - 1);
}

__device__ __forceinline__ void tile_origin(const TileMap& tm, int L, int* tx, int* ty) {
  if (tm.band_rows) {
    *ty = L / tm.tiles_x;
    *tx = L - *ty * tm.tiles_x;
  } else {
    *tx = L / tm.tiles_y;
    *ty = L - *tx * tm.tiles_y;
  }
}
__device__ __forceinline__ void quad_pixel(const TileMap& tm, int L, int* i, int* j) {
  int tx, ty;
  tile_origin(tm, L, &tx, &ty);
  const int q = threadIdx.x >> 2;
  *i = tx * kTile + (q & 7);
  *j = ty * kTile + (q >> 3);
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

// Sum and maximum over the 64 lanes of a wavefront.
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// The march runs in three kernels so that its dominant cost, the light
// marches (two per primary sample), is spread over one lane per recorded
// sample and light instead of serialised inside one lane per pixel:
//   0. (relayout_balance: the bricked grid, and the band tile ranges)
//   1. march_primary: four lanes per pixel walk the primary samples, write
//      T and D, and record (t_n, A_n, T_{n-1}) of every sample with a
//      nonzero weight in [k][P] planes (in z order also the sample's z
//      bucket, or in cell order its z cell, counting the records per
//      bucket); in band and z order each wavefront then appends (pixel, k)
//      of its records, k-major, to its XCD band's work list;
//   2. (z order: zsort_records scatters the band lists' entries into z-bucket
//      order; cell order: zsort_cells scatters the records into cell order;)
//   3. march_lights: one lane per record and light (the records cut into
//      eight equal ranges, one per XCD) marches toward that light and
//      stores its transmittance at (light, k, pixel); in cell order
//      march_lights_cells does the same from the cell's density planes
//      staged in LDS;
//   4. march_accumulate: one lane per pixel sums A_n L_n in sample order.
// Band order suits grids whose bricks fit the XCDs' L2s (each XCD's screen
// band sees a slab of them); larger grids take z order, and grids whose
// planes fit in LDS take cell order for the top/bottom lights (march_order
// in plan.hip).  The work lists keep the light-march lanes dense and
// spatially coherent (a wave takes neighbouring pixels at similar depths)
// whatever the per-pixel sample counts are.
// One optical-depth step (tau_n = tau_{n-1} + sigma_n h).
__device__ __forceinline__ float depth_step(float L, float sig, float h) { return L + sig * h; }

// Primary march of tile `tile` (band order) of band `band`, whose work list
// starts at `list`, with four lanes per pixel (see below); zh: the block's
// z-bucket counts, agg: 5 ints of LDS for the block's append.  Every thread
// of the block calls it (it has block barriers).
__device__ __forceinline__ void primary_tile(const MarchDev& m, const CamDev& c, const TileMap& tm,
                                             const MarchBuf& buf, float* __restrict__ guide, int tile, int band,
                                             int2* __restrict__ list, int* zh, int* agg) {
  int i, j;
  quad_pixel(tm, tile, &i, &j);
  const int s = threadIdx.x & 3;
  const bool inside = i < c.W && j < c.H;
  const uint32_t pix = (uint32_t)j * (uint32_t)c.W + (uint32_t)i;
  const float h = m.h;
  V3 o = v3(0.0f, 0.0f, 0.0f), d = v3(0.0f, 0.0f, 1.0f);
  float u = 0.0f;
  int n0 = 1, n1 = 0;  // sample range [n0, n1] (empty by default)
  if (inside) {
    camera_ray(c, i, j, &o, &d);
    if (m.jitter_on) {
      const uint64_t key = m.seed ^ ((uint64_t)m.frame << 32) ^ (uint64_t)pix;
      u = (float)(uint32_t)(splitmix64(key) >> 40) * (1.0f / 16777216.0f);
    }
    float t0, t1;
    if (clip_support(m, o, d, &t0, &t1)) {
      n0 = max(1, (int)ceilf(t0 / h - u));
      n1 = (int)floorf(t1 / h - u);
    }
  }
  // Lane s of the quad takes samples n = n0 + 4g + s of group g, so the four
  // lanes gather four consecutive samples and a wave's loads stay in a
  // compact part of the volume.  Group by group, the optical depth runs
  // through the quad in sample order (tau_n = tau_{n-1} + sigma_n h, handed
  // from lane to lane, the same float sums as one lane walking the ray),
  // each lane forms T_{n-1}, A_n, its record index (records of the lower
  // lanes counted by a ballot) and the depth test, and the quad stops after
  // the group in which the depth first passes tau_max.  A sample is taken
  // only if the depth before it is still within tau_max.  (Issuing the loads
  // of two or four groups before their sums was slower: 19.3 and 20.9 us
  // against 18.2 per headline march, the extra groups mostly wasted past
  // the termination and their registers costing waves.)
  const bool riemann = m.quadrature == LNM_QUAD_RIEMANN;
  const int lane = threadIdx.x & 63, qbase = lane & ~3;
  float tau = 0.0f;  // depth before the current group (equal in the quad)
  int k = 0, dn = 0;  // records so far (equal in the quad), this lane's first sample over depth_tau
  bool term = false;
  for (int nb = n0; nb <= n1 && !term; nb += 4) {
    const int n = nb + s;
    const float t = ((float)n + u) * h;
    const float pz = o.z + t * d.z;
    const float sg = sample_sigma(m, o.x + t * d.x, o.y + t * d.y, pz);
    const bool valid = n <= n1;
    const float sig = valid ? sg : 0.0f;
    // running depth through the quad: lane s ends with tau_n
    float x = s == 0 ? depth_step(tau, sig, h) : 0.0f;
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      const float v = __shfl_up(x, 1, 4);
      if (s == r) x = depth_step(v, sig, h);
    }
    float before = __shfl_up(x, 1, 4);
    if (s == 0) before = tau;
    const bool active = valid && before <= m.tau_max;
    const float alpha = riemann ? sig * h : -expm1f(-sig * h);
    const bool rec = active && alpha != 0.0f;
    const unsigned quad = (unsigned)(__ballot(rec) >> qbase) & 0xfu;
    const int kr = k + __popc(quad & ((1u << s) - 1u));
    if (rec && kr < buf.K) {
      const float Tprev = expf(-before);
      const size_t r = (size_t)kr * buf.P + pix;
      buf.t[r] = t;
      buf.a[r] = Tprev * alpha;
      buf.tp[r] = Tprev;
      if (m.zorder) {
        const int zk = z_bucket(m, pz);
        buf.zb[r] = (uint8_t)zk;
        atomicAdd(&zh[zk], 1);
      }
    }
    if (active && dn == 0 && sig > m.depth_tau) dn = n;
    k = min(k + __popc(quad), buf.K);
    const unsigned over = (unsigned)(__ballot(active && x > m.tau_max) >> qbase) & 0xfu;
    tau = __shfl(x, 3, 4);
    term = over != 0u;
  }
  // quad results: records, depth, transmittance
  const int cnt = k;
  const int big = 0x7fffffff;
  int dmin = dn ? dn : big;
  dmin = min(dmin, __shfl_xor(dmin, 1, 4));
  dmin = min(dmin, __shfl_xor(dmin, 2, 4));
  if (inside && s == 0) {
    buf.cnt[pix] = cnt;
    float* g = guide + 3 * (size_t)pix;
    g[1] = term ? 0.0f : expf(-tau);
    g[2] = dmin == big ? 0.0f : (float)dmin * h;
  }
  // cell order reads the records through the per-pixel counts instead
  if (m.zorder == kOrderCells) return;
  // append the tile's records to the band's list: one atomic per block (the
  // four waves' totals summed in LDS; a wave's share follows the lower
  // waves'), then k-major order within each wave (pixels in lane order within
  // each k); lane s of a quad writes the pixel's records k = s (mod 4)
  const int total = wave_sum(s == 0 ? cnt : 0);
  const int wave = threadIdx.x >> 6;
  if (lane == 0) agg[wave] = total;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int all = agg[0] + agg[1] + agg[2] + agg[3];
    agg[4] = all ? atomicAdd(buf.ctr + band, all) : 0;
  }
  __syncthreads();
  int base = agg[4];
  for (int w = 0; w < wave; ++w) base += agg[w];
  __syncthreads();
  if (total == 0) return;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int kmax = wave_max(k);
  int off = base;
  for (int kk = 0; kk < kmax; ++kk) {
    const bool mine = (kk & 3) == s && kk < cnt;
    const unsigned long long has = __ballot(mine);
    if (mine) list[off + __popcll(has & below)] = make_int2((int)pix, kk);
    off += __popcll(has);
  }
}

// Band e = blockIdx.x % 8 (the XCD the block runs on under round-robin
// placement) owns tiles [start[e], start[e + 1]) of the band order, chosen by
// march_balance so that the bands carry equal estimated work; its work list
// starts at entry start[e] * 64 * K, room for K records of every pixel it
// owns.  The band's blocks take its tiles in turn.
// In z order the block also counts its records per z bucket in LDS and adds
// them to the global counts at the end.
__global__ __launch_bounds__(256, 4) void march_primary(MarchDev m, CamDev c, TileMap tm, MarchBuf buf,
                                                     float* __restrict__ guide) {
  __shared__ int zh[kZBuckets];
  __shared__ int agg[5];
  if (m.zorder) {
    for (int q = threadIdx.x; q < kZBuckets; q += 256) zh[q] = 0;
    __syncthreads();
  }
  const int band = blockIdx.x & 7, slots = gridDim.x >> 3;
  const int* start = buf.ctr + kBandStart;
  const int lo = start[band], hi = start[band + 1];
  int2* list = buf.rec ? buf.rec + (size_t)lo * (kTile * kTile) * (size_t)buf.K : nullptr;
  for (int L = lo + (int)(blockIdx.x >> 3); L < hi; L += slots)
    primary_tile(m, c, tm, buf, guide, L, band, list, zh, agg);
  if (m.zorder) {
    __syncthreads();
    for (int q = threadIdx.x; q < kZBuckets; q += 256)
      if (zh[q]) atomicAdd(buf.ctr + kZHist + q, zh[q]);
  }
}

// Estimated cost of tile L: the primary samples of its centre ray (every
// sample in the support box is taken, dense or empty) plus a fixed share.
__device__ __forceinline__ int tile_cost(const MarchDev& m, const CamDev& c, const TileMap& tm, int L) {
  int tx, ty;
  tile_origin(tm, L, &tx, &ty);
  const int i = min(tx * kTile + kTile / 2, c.W - 1), j = min(ty * kTile + kTile / 2, c.H - 1);
  V3 o, d;
  camera_ray(c, i, j, &o, &d);
  float t0, t1;
  const int n = clip_support(m, o, d, &t0, &t1) ? (int)fminf((t1 - t0) / m.h, 1e6f) : 0;
  return n + 2;
}

// Zero the band counters and cut the band order of tiles into 8 ranges of
// about equal estimated cost (start[0..8] after the counters).  The smoke
// often covers a small part of the screen; equal screen bands would leave
// most XCDs idle.  One workgroup of 256 lanes: per-lane sums over contiguous
// tile runs, an LDS scan, then each tile goes to range floor(8 (prefix +
// cost / 2) / total); all sums are integers, so the ranges are exact and
// contiguous.  The first kCostCache tile costs are kept in LDS for the
// second pass.
constexpr int kBalanceThreads = 256, kCostCache = 2048;
struct BalanceLds {
  long long scan[2][kBalanceThreads];
  int cost[kCostCache];
  int first[8];
};
__device__ void balance_tiles(const MarchDev& m, const CamDev& c, const TileMap& tm, int* __restrict__ ctr,
                              BalanceLds& sh) {
  const int tid = threadIdx.x, ntiles = tm.tiles_x * tm.tiles_y;
  const int per = (ntiles + kBalanceThreads - 1) / kBalanceThreads;
  const int a = min(ntiles, tid * per), b = min(ntiles, a + per);
  if (tid < 8) {
    ctr[tid] = 0;
    ctr[kUnitNext + tid] = 0;
    sh.first[tid] = ntiles;
  }
  for (int q = tid; q < 2 * kZBuckets; q += kBalanceThreads) ctr[kZHist + q] = 0;
  long long sum = 0;
  for (int L = a; L < b; ++L) {
    const int cst = tile_cost(m, c, tm, L);
    if (L < kCostCache) sh.cost[L] = cst;
    sum += cst;
  }
  sh.scan[0][tid] = sum;
  __syncthreads();
  int cur = 0;
  for (int o = 1; o < kBalanceThreads; o <<= 1) {  // inclusive scan (Hillis-Steele)
    const long long v = sh.scan[cur][tid] + (tid >= o ? sh.scan[cur][tid - o] : 0);
    sh.scan[cur ^ 1][tid] = v;
    cur ^= 1;
    __syncthreads();
  }
  const long long total = sh.scan[cur][kBalanceThreads - 1];
  long long run = sh.scan[cur][tid] - sum;
  for (int L = a; L < b; ++L) {
    const int cst = L < kCostCache ? sh.cost[L] : tile_cost(m, c, tm, L);
    const int e = (int)min(7LL, (8 * (2 * run + cst)) / (2 * total));
    atomicMin(&sh.first[e], L);
    run += cst;
  }
  __syncthreads();
  if (tid == 0) {
    int* start = ctr + kBandStart;
    start[8] = ntiles;
    for (int e = 7; e >= 1; --e) start[e] = min(sh.first[e], start[e + 1]);
    start[0] = 0;
  }
}

// The balance alone, when the march reads prebuilt bricks (otherwise it runs
// in an extra workgroup of the relayout launch).
__global__ __launch_bounds__(256) void march_balance(MarchDev m, CamDev c, TileMap tm, int* __restrict__ ctr) {
  __shared__ BalanceLds sh;
  balance_tiles(m, c, tm, ctr, sh);
}

// The march's relayout: the same blocks behind one z slice whose first
// block cuts the screen tiles into the balanced band ranges (the others
// exit); that slice is dispatched first, so the balance runs beside the
// copy instead of after it.
__global__ __launch_bounds__(256) void relayout_balance(MarchDev m, CamDev c, TileMap tm, int* __restrict__ ctr,
                                                        float* __restrict__ brick) {
  __shared__ union {
    float rows[kRelayRows][kRelayRow];
    BalanceLds bal;
  } sh;
  if (blockIdx.z == 0) {
    if (blockIdx.x == 0 && blockIdx.y == 0) balance_tiles(m, c, tm, ctr, sh.bal);
    return;
  }
  relayout_block(m.rho, m.nx, m.ny, m.nz, m.nbx, m.nby, brick, sh.rows, blockIdx.x, blockIdx.y, blockIdx.z - 1);
}

// Entry r of the band lists concatenated in band order.
__device__ __forceinline__ int2 band_entry(const MarchBuf& buf, const int (&count)[8], int r) {
  int band = 0, off = r;
#pragma unroll
  for (int e = 0; e < 7; ++e) {
    if (band == e && off >= count[e]) {
      off -= count[e];
      band = e + 1;
    }
  }
  return buf.rec[(size_t)buf.ctr[kBandStart + band] * (kTile * kTile) * (size_t)buf.K + off];
}

// Scatter the records of the band lists into z-bucket order (srt).  Bucket
// b's records take entries [B_b, B_b + n_b), B the exclusive prefix sum of
// the counts n the primary march took.  Each block takes one contiguous
// share of the band-order records: it counts them per bucket in LDS,
// reserves each bucket's share with one global atomic, and writes its
// entries there on a second pass, so within a bucket the entries come in
// runs of neighbouring pixels.  Every write is bounded by its bucket's
// range.
__global__ __launch_bounds__(256) void zsort_records(MarchBuf buf) {
  __shared__ int scan[2][kZBuckets];
  __shared__ int bstart[kZBuckets], bend[kZBuckets], lcount[kZBuckets], lbase[kZBuckets];
  static_assert(kZBuckets == 256, "one lane per bucket");
  const int tid = threadIdx.x;
  const int n = buf.ctr[kZHist + tid];
  scan[0][tid] = n;
  lcount[tid] = 0;
  __syncthreads();
  int cur = 0;
  for (int o = 1; o < kZBuckets; o <<= 1) {  // inclusive scan (Hillis-Steele)
    scan[cur ^ 1][tid] = scan[cur][tid] + (tid >= o ? scan[cur][tid - o] : 0);
    cur ^= 1;
    __syncthreads();
  }
  bstart[tid] = scan[cur][tid] - n;
  bend[tid] = scan[cur][tid];
  int count[8], total = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    count[e] = buf.ctr[e];
    total += count[e];
  }
  const long per = ((long)total + gridDim.x - 1) / gridDim.x;
  const int r0 = (int)min((long)total, (long)blockIdx.x * per), r1 = (int)min((long)total, (long)r0 + per);
  // U entries per lane at a time, their loads and LDS atomics issued together
  constexpr int U = 4;
  for (int r = r0 + tid; r < r1; r += U * 256) {
    int zk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ru = r + u * 256;
      zk[u] = -1;
      if (ru < r1) {
        const int2 en = band_entry(buf, count, ru);
        zk[u] = buf.zb[(size_t)en.y * buf.P + en.x];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (zk[u] >= 0) atomicAdd(&lcount[zk[u]], 1);
  }
  __syncthreads();
  const int mine = lcount[tid];
  if (mine) lbase[tid] = atomicAdd(buf.ctr + kZCursor + tid, mine);
  lcount[tid] = 0;  // now the block's cursor per bucket
  __syncthreads();
  for (int r = r0 + tid; r < r1; r += U * 256) {
    int2 en[U];
    int zk[U], at[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ru = r + u * 256;
      zk[u] = -1;
      en[u] = make_int2(0, 0);
      if (ru < r1) {
        en[u] = band_entry(buf, count, ru);
        zk[u] = buf.zb[(size_t)en[u].y * buf.P + en[u].x];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) at[u] = zk[u] >= 0 ? atomicAdd(&lcount[zk[u]], 1) : 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (zk[u] < 0) continue;
      const long pos = (long)bstart[zk[u]] + lbase[zk[u]] + at[u];
      if (pos < bend[zk[u]]) buf.srt[pos] = en[u];
    }
  }
}

// Cell order: the records scattered into z-cell order (srt).  A block takes
// 64 pixels; wavefront w of the block takes the records k = w, w + 4, ... of
// each (one lane per pixel; whose cells the primary march wrote to zb), so a
// CU holds several blocks' loads in flight.  Cell b's records take entries
// [B_b, B_b + n_b), B the exclusive prefix sum of the counts n; each block
// counts its records per cell in LDS, reserves each cell's share with one
// global atomic and writes its entries there on a second pass.  Every write
// is bounded by its cell's range.
constexpr int kSortPixels = 64;
__global__ __launch_bounds__(256) void zsort_cells(MarchBuf buf) {
  __shared__ int wsum[kZBuckets / 64];
  __shared__ int bstart[kZBuckets], bend[kZBuckets], lcount[kZBuckets], lbase[kZBuckets];
  static_assert(kZBuckets == 256, "one lane per bucket");
  const int tid = threadIdx.x, lane = tid & 63;
  // the cells' ranges in the list: an inclusive scan of the histogram
  // within each wavefront, then across the four
  const int n = buf.ctr[kZHist + tid];
  int inc = n;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(inc, o);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[tid >> 6] = inc;
  lcount[tid] = 0;
  __syncthreads();
  for (int w = 0; w < (tid >> 6); ++w) inc += wsum[w];
  bstart[tid] = inc - n;
  bend[tid] = inc;
  // S lanes per pixel: lane tid takes records tid / kSortPixels + S j of
  // pixel tid % kSortPixels
  constexpr int S = 256 / kSortPixels;
  const int p = blockIdx.x * kSortPixels + tid % kSortPixels, k1 = tid / kSortPixels;
  const int cnt = p < buf.P ? min(buf.cnt[p], buf.K) : 0;
  // U of the lane's records at a time, their loads and LDS atomics issued
  // together (one record after the other leaves the lane waiting on each load)
  constexpr int U = 4;
  for (int k0 = k1; k0 < cnt; k0 += U * S) {
    int zk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) zk[u] = k0 + u * S < cnt ? buf.zb[(size_t)(k0 + u * S) * buf.P + p] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (zk[u] >= 0) atomicAdd(&lcount[zk[u]], 1);
  }
  __syncthreads();
  const int mine = lcount[tid];
  if (mine) lbase[tid] = atomicAdd(buf.ctr + kZCursor + tid, mine);
  lcount[tid] = 0;  // now the block's cursor per cell
  __syncthreads();
  for (int k0 = k1; k0 < cnt; k0 += U * S) {
    int zk[U], at[U];
#pragma unroll
    for (int u = 0; u < U; ++u) zk[u] = k0 + u * S < cnt ? buf.zb[(size_t)(k0 + u * S) * buf.P + p] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) at[u] = zk[u] >= 0 ? atomicAdd(&lcount[zk[u]], 1) : 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (zk[u] < 0) continue;
      const int b = zk[u];
      const long pos = (long)bstart[b] + lbase[b] + at[u];
      if (pos < bend[b]) buf.srt[pos] = make_int2(p, k0 + u * S);
    }
  }
}

// One lane per (record, light).  The records, in band order (the band
// lists concatenated: a spatially ordered sequence) or in z order (srt),
// are cut into 8 equal contiguous ranges, one per XCD (block b serves range
// b % 8, the XCD that runs it under round-robin placement), so every XCD
// and its L2 take an eighth of the light marches even when the smoke covers
// only a few screen bands.  A range is cut into 256-entry chunks and each
// chunk into two units, one per light, so a workgroup marches one light
// direction.  Band order: block b takes units b / 8, b / 8 + slots, ...  Z
// order: the grid is the blocks resident at once; block b takes unit b / 8,
// then units R, R + 1, ... in turn from its XCD's counter (R blocks per
// XCD), so the units in flight stay adjacent and sweep the XCD's slab of
// brick layers once, layer by layer (a side light keeps its sample's z, so
// the bricks in use at a time are about one layer).  Result: T toward the
// top (or first side) light in tl[0][k][pixel], toward the bottom (second
// side) light in tl[1][k][pixel].
template <bool Z>
__global__ __launch_bounds__(256) void march_lights(MarchDev m, CamDev c, MarchBuf buf, int slots) {
  int count[8], total = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    count[e] = buf.ctr[e];
    total += count[e];
  }
  const int part = blockIdx.x & 7;
  const int lo = (int)((long)total * part / 8), hi = (int)((long)total * (part + 1) / 8);
  const int units = 2 * ((hi - lo + 255) / 256);
  const int R = gridDim.x >> 3;
  __shared__ int s_unit;
  for (int unit = blockIdx.x >> 3; unit < units;) {
    do {  // one unit; `continue` leaves it
      const int light = unit & 1;
      if ((light ? m.wb : m.wt) == 0.0f) continue;
      const int r = lo + (unit >> 1) * 256 + threadIdx.x;
      if (r >= hi) continue;
      const int2 en = Z ? buf.srt[r] : band_entry(buf, count, r);
      // every entry of [0, total) is written by the primary march (and the
      // scatter); the check keeps a lane that would see anything else in bounds
      if ((unsigned)en.x >= (unsigned)buf.P || (unsigned)en.y >= (unsigned)buf.K) continue;
      const int pix = en.x, k = en.y;
      const size_t q = (size_t)k * buf.P + pix;
      V3 o, d;
      camera_ray(c, pix % c.W, pix / c.W, &o, &d);
      const float t = buf.t[q];
      V3 l = side_light(d, m.light_set);
      if (light) l = v3(-l.x, -l.y, -l.z);
      const V3 x = v3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
      buf.tl[(size_t)light * buf.K * buf.P + q] =
          l.z == 0.0f ? light_transmittance_batched<true>(m, x, l) : light_transmittance_batched<false>(m, x, l);
    } while (0);
    if constexpr (Z) {
      if (R >= units) break;
      __syncthreads();
      if (threadIdx.x == 0) s_unit = R + atomicAdd(buf.ctr + kUnitNext + part, 1);
      __syncthreads();
      unit = s_unit;
    } else {
      unit += slots;
    }
  }
}

// Cell order: one lane per record and light, the records sorted by their
// sample's z cell (srt), each workgroup staging the two grid planes of its
// cell in LDS.  The records of cell b form ceil(n_b / kCellRecs) units of
// kCellRecs records; wavefront w of the workgroup takes records 64 (w / 2)
// .. 64 (w / 2) + 63 of the unit toward light w % 2, so a wavefront's lanes
// march neighbouring samples in one direction (similar lengths, nearby
// taps; with the two lights of a sample in one wavefront, every step waited
// for the longer of two opposite marches).  Block g of the grid takes
// the contiguous run [g U / G, (g + 1) U / G) of the U units (g numbered so
// that the blocks of one XCD, b % 8, take adjacent runs: a slab of cells),
// and stages planes again only when its cell changes.  Flat lights (every
// light of the top/bottom set except the fallback of a ray along z) read
// LDS; others read the bricks.
constexpr int kCellThreads = 1024, kCellRecs = kCellThreads / 2;
constexpr int kCellEntries = (int)((kCellLdsBytes / sizeof(float2) + kCellThreads - 1) / kCellThreads);
constexpr int kCellQuads = (int)((kCellLdsBytes / sizeof(float2) / 4 + kCellThreads - 1) / kCellThreads);

// Grid planes b - 1 and b of cell b into the LDS table, zero outside the
// grid, as (below, above - below): lane tid takes entries tid + kCellThreads e
// of the (ny + 3) x pitch table, border included, in two batches of loads in
// flight together (clamped addresses, masked values).
// The lane index is passed through an empty asm statement so that the
// compiler recomputes the lane's entries at each staging instead of keeping
// them in registers across the whole march loop.
__device__ __forceinline__ int lane_index_here() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
__device__ __forceinline__ void stage_planes(const MarchDev& m, int b, float2* planes, int pitch) {
  const int tid = lane_index_here();
  const int n_ent = (m.ny + 3) * pitch, dy = kCellThreads / pitch, dx = kCellThreads % pitch;
  const int ps = m.nx * m.ny;
  const int p0 = min(max(b - 1, 0), m.nz - 1) * ps, p1 = min(b, m.nz - 1) * ps;
  const bool z0 = b - 1 >= 0 && b - 1 < m.nz, z1 = b < m.nz;
  constexpr int E = (kCellEntries + 1) / 2;  // entries per batch (two batches)
  int y = tid / pitch, x = tid - y * pitch;
  for (int e0 = 0; e0 < 2 * E; e0 += E) {
    float v0[E], v1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = y - 1, i = x - 1;
      const bool in = tid + (e0 + e) * kCellThreads < n_ent && j >= 0 && j < m.ny && i >= 0 && i < m.nx;
      const int col = in ? j * m.nx + i : 0;
      v0[e] = m.rho[(unsigned)(p0 + col)];
      v1[e] = m.rho[(unsigned)(p1 + col)];
      v0[e] = in && z0 ? v0[e] : 0.0f;
      v1[e] = in && z1 ? v1[e] : 0.0f;
      x += dx;
      y += dy;
      if (x >= pitch) {
        x -= pitch;
        ++y;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = tid + (e0 + e) * kCellThreads;
      if (q < n_ent) planes[q] = make_float2(v0[e], v1[e] - v0[e]);
    }
  }
}
// The same for rows of a multiple of four values (16-byte aligned): lane tid
// takes the four-value groups tid + kCellThreads e of the ny x nx / 4 grid
// part, one 16-byte load per plane each; the border is not written.
__device__ __forceinline__ void stage_planes_vec(const MarchDev& m, int b, float2* planes, int pitch) {
  const int tid = lane_index_here();
  const int q4 = m.nx >> 2, n4 = m.ny * q4, dj = kCellThreads / q4, dg = kCellThreads % q4;
  const int ps = m.nx * m.ny;
  const float4* r0 = reinterpret_cast<const float4*>(m.rho + (size_t)min(max(b - 1, 0), m.nz - 1) * ps);
  const float4* r1 = reinterpret_cast<const float4*>(m.rho + (size_t)min(b, m.nz - 1) * ps);
  const bool z0 = b - 1 >= 0 && b - 1 < m.nz, z1 = b < m.nz;
  float4 v0[kCellQuads], v1[kCellQuads];
  int j = tid / q4, g = tid - j * q4;
  int at[kCellQuads];
#pragma unroll
  for (int e = 0; e < kCellQuads; ++e) {
    const bool in = tid + e * kCellThreads < n4;
    const int q = in ? tid + e * kCellThreads : 0;
    v0[e] = r0[q];
    v1[e] = r1[q];
    if (!(in && z0)) v0[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (!(in && z1)) v1[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    at[e] = in ? (j + 1) * pitch + 4 * g + 1 : -1;
    g += dg;
    j += dj;
    if (g >= q4) {
      g -= q4;
      ++j;
    }
  }
#pragma unroll
  for (int e = 0; e < kCellQuads; ++e) {
    if (at[e] < 0) continue;
    float2* d = planes + at[e];
    d[0] = make_float2(v0[e].x, v1[e].x - v0[e].x);
    d[1] = make_float2(v0[e].y, v1[e].y - v0[e].y);
    d[2] = make_float2(v0[e].z, v1[e].z - v0[e].z);
    d[3] = make_float2(v0[e].w, v1[e].w - v0[e].w);
  }
}
__global__ __launch_bounds__(kCellThreads) void march_lights_cells(MarchDev m, CamDev c, MarchBuf buf) {
  extern __shared__ float2 planes[];  // [ny + 3][nx + 3] pairs (plane below, above - below)
  __shared__ int cnt[kZBuckets], ustart[kZBuckets + 1], rstart[kZBuckets], wsum[2][kZBuckets / 64];
  const int tid = threadIdx.x, lane = tid & 63;
  // units and record offsets of the cells: exclusive prefix sums over the
  // buckets, one lane each (scans within the wavefronts, then across them)
  int nc = 0, nu = 0, ic = 0, iu = 0;
  if (tid < kZBuckets) {
    nc = buf.ctr[kZHist + tid];
    nu = (nc + kCellRecs - 1) / kCellRecs;
    cnt[tid] = nc;
    ic = nc;
    iu = nu;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int tc = __shfl_up(ic, o), tu = __shfl_up(iu, o);
      if (lane >= o) {
        ic += tc;
        iu += tu;
      }
    }
    if (lane == 63) {
      wsum[0][tid >> 6] = ic;
      wsum[1][tid >> 6] = iu;
    }
  }
  __syncthreads();
  if (tid < kZBuckets) {
    for (int w = 0; w < (tid >> 6); ++w) {
      ic += wsum[0][w];
      iu += wsum[1][w];
    }
    rstart[tid] = ic - nc;
    ustart[tid] = iu - nu;
    if (tid == kZBuckets - 1) ustart[kZBuckets] = iu;
  }
  __syncthreads();
  const long units = ustart[kZBuckets];
  const int G = gridDim.x, g = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int u0 = (int)(units * g / G), u1 = (int)(units * (g + 1) / G);
  const int pitch = m.nx + 3;
  const int light = (tid >> 6) & 1, slot = ((tid >> 7) << 6) | (tid & 63);
  const float w = light ? m.wb : m.wt;
  int staged = -1;  // the cell whose planes are in LDS (the same in every lane)
  // rows of four grid values as one 16-byte load when the rows allow it; the
  // zero border is then written once here (the stagings write the interior)
  const bool vec = (m.nx & 3) == 0 && ((uintptr_t)m.rho & 15) == 0;
  if (vec) {
    const int nb = 3 * pitch + 3 * m.ny;  // rows 0, ny + 1, ny + 2; columns 0, nx + 1, nx + 2
    for (int t = tid; t < nb; t += kCellThreads) {
      int e;
      if (t < 3 * pitch) {
        const int r = t / pitch, x = t - r * pitch;
        e = (r == 0 ? 0 : m.ny + r) * pitch + x;
      } else {
        const int t2 = t - 3 * pitch, r = t2 / 3, cc = t2 - 3 * r;
        e = (r + 1) * pitch + (cc == 0 ? 0 : m.nx + cc);
      }
      planes[e] = make_float2(0.0f, 0.0f);
    }
  }
  for (int u = u0; u < u1; ++u) {
    int b = 0;  // the cell of unit u: the last b with ustart[b] <= u
    for (int step = 128; step > 0; step >>= 1)
      if (b + step < kZBuckets && ustart[b + step] <= u) b += step;
    if (b != staged) {
      __syncthreads();  // every lane is done with the previous cell's planes
      if (vec)
        stage_planes_vec(m, b, planes, pitch);
      else
        stage_planes(m, b, planes, pitch);
      __syncthreads();
      staged = b;
    }
    const int r = (u - ustart[b]) * kCellRecs + slot;
    if (r >= cnt[b] || w == 0.0f) continue;
    const int2 en = buf.srt[rstart[b] + r];
    // every entry of the list is written by the scatter; the check keeps a
    // lane that would see anything else in bounds
    if ((unsigned)en.x >= (unsigned)buf.P || (unsigned)en.y >= (unsigned)buf.K) continue;
    const int pix = en.x, k = en.y;
    const size_t q = (size_t)k * buf.P + pix;
    V3 o, d;
    camera_ray(c, pix % c.W, pix / c.W, &o, &d);
    const float t = buf.t[q];
    V3 l = side_light(d, m.light_set);
    if (light) l = v3(-l.x, -l.y, -l.z);
    const V3 x = v3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
    // the staged planes serve a flat light whose sample lies in cell b
    const float gz = fmaf(x.z, (float)m.nz, -0.5f);
    const bool in_cell = gz > -1.0f && gz < (float)m.nz && (int)floorf(gz) + 1 == b;
    float T;
    if (l.z == 0.0f && in_cell)
      T = light_transmittance_lds(m, x, l, planes, pitch);
    else if (l.z == 0.0f)
      T = light_transmittance_batched<true>(m, x, l);
    else
      T = light_transmittance_batched<false>(m, x, l);
    buf.tl[(size_t)light * buf.K * buf.P + q] = T;
  }
}

__global__ __launch_bounds__(256) void march_accumulate(MarchDev m, MarchBuf buf, float* __restrict__ guide) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= buf.P) return;
  const int cnt = buf.cnt[p];
  const size_t P = (size_t)buf.P, KP = (size_t)buf.K * P;
  const float wf = m.wf, wt = m.wt, wb = m.wb;
  float Ls = 0.0f;
  // eight records' loads issued together, then summed in sample order; the
  // front light's transmittance is T_{n-1} (marching toward w retraces the
  // earlier primary samples)
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    float a[8], tp[8], t0[8], t1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const size_t r = (size_t)min(k0 + q, cnt - 1) * P + p;
      a[q] = buf.a[r];
      tp[q] = buf.tp[r];
      t0[q] = wt != 0.0f ? buf.tl[r] : 0.0f;
      t1[q] = wb != 0.0f ? buf.tl[KP + r] : 0.0f;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (k0 + q >= cnt) break;
      float L = wf * tp[q];
      if (wt != 0.0f) L += wt * t0[q];
      if (wb != 0.0f) L += wb * t1[q];
      Ls += a[q] * L;
    }
  }
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

constexpr size_t kLightSlots = 512;  // workgroups per band in march_lights (band order)

hipError_t launch_relayout(const MarchDev& m, float* bricks, hipStream_t s) {
  const int nbx = bricks_along(m.nx), nby = bricks_along(m.ny), nbz = bricks_along(m.nz);
  hipLaunchKernelGGL(relayout_bricks,
                     dim3((nbx + kRelayBricks - 1) / kRelayBricks, (nby + kRelayY - 1) / kRelayY, nbz), dim3(256), 0, s,
                     m.rho, m.nx, m.ny, m.nz, nbx, nby, bricks);
  return hipGetLastError();
}

// Band screen rows instead of columns when the top light of the central ray
// runs more horizontally than vertically on screen.
static TileMap tile_map(const CamDev& c) {
  TileMap tm;
  tm.tiles_x = (c.W + kTile - 1) / kTile;
  tm.tiles_y = (c.H + kTile - 1) / kTile;
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

// Light-march blocks per XCD in z order: as many as are resident at once
// (the occupancy of march_lights on one XCD's CUs), at least one.
static int light_blocks_per_xcd() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, march_lights<true>, 256, 0) == hipSuccess)
      n = std::max(1, per_cu * cus / 8);
    else
      n = (int)kLightSlots;
  }
  return n;
}

// Cell-order light-march blocks per XCD: the CUs of one XCD (one block per CU).
static int cell_blocks_per_xcd() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, cus = 0;
    n = hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus >= 8
            ? cus / 8
            : 32;
  }
  return n;
}

hipError_t launch_march(const MarchDev& m0, const CamDev& cam, const MarchBuf& buf, float* guide, hipStream_t s) {
  MarchDev m = m0;
  m.nbx = buf.nbx;
  m.nby = buf.nby;
  m.nbz = buf.nbz;
  const TileMap tm = tile_map(cam);
  if (!m.brick) {  // build the bricks in the scratch; one extra block balances the bands
    m.brick = buf.brick;
    hipLaunchKernelGGL(relayout_balance,
                       dim3((m.nbx + kRelayBricks - 1) / kRelayBricks, (m.nby + kRelayY - 1) / kRelayY, m.nbz + 1),
                       dim3(256), 0, s, m, cam, tm, buf.ctr, buf.brick);
  } else {
    hipLaunchKernelGGL(march_balance, dim3(1), dim3(kBalanceThreads), 0, s, m, cam, tm, buf.ctr);
  }
  hipLaunchKernelGGL(march_primary, dim3(8 * tm.per_xcd), dim3(256), 0, s, m, cam, tm, buf, guide);
  if (m.zorder == kOrderCells) {
    // the scatter with one lane per pixel; the light marches with one
    // workgroup per CU (the planes take most of its LDS)
    hipLaunchKernelGGL(zsort_cells, dim3((buf.P + kSortPixels - 1) / kSortPixels), dim3(256), 0, s, buf);
    hipLaunchKernelGGL(march_lights_cells, dim3(8 * cell_blocks_per_xcd()), dim3(kCellThreads),
                       cell_planes_bytes(m.nx, m.ny), s, m, cam, buf);
  } else if (m.zorder) {
    // the blocks resident at once; each loops over units of its XCD's range
    const int slots = (int)std::min<size_t>((buf.cap + 255) / 256, (size_t)light_blocks_per_xcd());
    hipLaunchKernelGGL(zsort_records, dim3(8 * slots), dim3(256), 0, s, buf);
    hipLaunchKernelGGL(march_lights<true>, dim3(8 * slots), dim3(256), 0, s, m, cam, buf, slots);
  } else {
    // enough workgroups to fill the chip a few times over; each loops over
    // its eighth of the records
    const int slots = (int)std::min<size_t>((buf.cap + 255) / 256, kLightSlots);
    hipLaunchKernelGGL(march_lights<false>, dim3(8 * slots), dim3(256), 0, s, m, cam, buf, slots);
  }
  hipLaunchKernelGGL(march_accumulate, dim3((buf.P + 255) / 256), dim3(256), 0, s, m, buf, guide);
  return hipGetLastError();
}

hipError_t launch_reference(const MarchDev& m, const CamDev& cam, int srgb, float* lm, hipStream_t s) {
  dim3 grid((cam.W + 15) / 16, (cam.H + 15) / 16);
  hipLaunchKernelGGL(reference_kernel, grid, dim3(256), 0, s, m, cam, srgb, lm);
  return hipGetLastError();
}

}  // namespace lnm
