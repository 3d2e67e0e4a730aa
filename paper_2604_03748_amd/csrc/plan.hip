// Host-side planning of the kernels' work: the march's workspace layout,
// sample capacity and light-march order; the conv layers' tile heights and
// split-K factors; the channel adapters' supported widths.  Host code only
// (no kernels), shared by the entry points and the kernels' launchers.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace lnm {

// ---------------------------------------------------------------- march
int march_capacity(const MarchDev& m) {
  double d2 = 0.0;
  const int n[3] = {m.nx, m.ny, m.nz};
  for (int a = 0; a < 3; ++a) d2 += (1.0 + 1.0 / n[a]) * (1.0 + 1.0 / n[a]);
  return (int)std::ceil(std::sqrt(d2) / (double)m.h) + 2;
}

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }
int bricks_along(int n) { return (n >> 2) + 1; }
size_t bricks_bytes(int nx, int ny, int nz) {
  return sizeof(float) * kBrickSlot * (size_t)bricks_along(nx) * bricks_along(ny) * bricks_along(nz);
}

// Bricked grids above this size (the eight XCDs' L2s together) take the z
// order: measured at 256^3 / 1024^2, march 4.30 -> 2.73 ms; at 128^3 /
// 256^2 the scatter's launch costs more than the order saves.
constexpr size_t kZOrderBytes = (size_t)32 << 20;
static int tiles_per_band(int W, int H) { return (((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile) + 7) / 8; }

// Scratch: [K][P] planes t, A, T_{n-1}, T_top, T_bottom; per-pixel counts; the
// counter block; 8 band work lists of (pixel, k) with room for every sample
// of the band's pixels (not in cell order); in the z orders the [K][P]
// z-bucket plane and the z-ordered list (room for every sample); the bricked
// grid unless the caller supplies it.
size_t march_scratch_bytes(const MarchDev& m, int K, int W, int H) {
  const size_t P = (size_t)W * H, plane = a256(sizeof(float) * (size_t)K * P);
  const size_t cap = (size_t)tiles_per_band(W, H) * kTile * kTile * K;
  return 5 * plane + a256(sizeof(int) * P) + a256(kCounterBytes) +
         (m.zorder != kOrderCells ? a256(8 * cap * sizeof(int2)) : 0) +
         (m.zorder ? a256((size_t)K * P) + a256(sizeof(int2) * (size_t)K * P) : 0) +
         (m.brick ? 0 : a256(bricks_bytes(m.nx, m.ny, m.nz)));
}

// Cell order: the two planes of a cell in LDS, beside the kernel's own
// arrays, within the 160 KB a gfx950 workgroup may allocate; at most 255
// cells (z buckets).
size_t cell_planes_bytes(int nx, int ny) { return 2 * sizeof(float) * (size_t)(nx + 3) * (ny + 3); }
static bool cells_fit(int nx, int ny, int nz) { return cell_planes_bytes(nx, ny) <= kCellLdsBytes && nz < kZBuckets; }

int march_order(int work_order, int light_set, int nx, int ny, int nz) {
  if (work_order == LNM_ORDER_BANDS) return kOrderBands;
  if (work_order == LNM_ORDER_Z) return kOrderLayers;
  if (work_order == LNM_ORDER_CELLS) return cells_fit(nx, ny, nz) ? kOrderCells : -1;
  if (bricks_bytes(nx, ny, nz) > kZOrderBytes) return kOrderLayers;
  return light_set == LNM_LIGHTS_TOP_BOTTOM && cells_fit(nx, ny, nz) ? kOrderCells : kOrderBands;
}

MarchBuf march_buffers(void* ws, const MarchDev& m, int K, int W, int H) {
  char* p = static_cast<char*>(ws);
  const size_t P = (size_t)W * H, plane = a256(sizeof(float) * (size_t)K * P);
  MarchBuf b;
  b.t = reinterpret_cast<float*>(p);
  b.a = reinterpret_cast<float*>(p + plane);
  b.tp = reinterpret_cast<float*>(p + 2 * plane);
  b.tl = reinterpret_cast<float*>(p + 3 * plane);  // two planes
  p += 5 * plane;
  b.cnt = reinterpret_cast<int*>(p);
  p += a256(sizeof(int) * P);
  b.ctr = reinterpret_cast<int*>(p);
  p += a256(kCounterBytes);
  b.cap = (size_t)tiles_per_band(W, H) * kTile * kTile * K;
  b.rec = nullptr;  // cell order reads the records through the per-pixel counts
  if (m.zorder != kOrderCells) {
    b.rec = reinterpret_cast<int2*>(p);
    p += a256(8 * b.cap * sizeof(int2));
  }
  b.zb = nullptr;
  b.srt = nullptr;
  if (m.zorder) {
    b.zb = reinterpret_cast<uint8_t*>(p);
    p += a256((size_t)K * P);
    b.srt = reinterpret_cast<int2*>(p);
    p += a256(sizeof(int2) * (size_t)K * P);
  }
  b.brick = m.brick ? nullptr : reinterpret_cast<float*>(p);
  b.nbx = bricks_along(m.nx);
  b.nby = bricks_along(m.ny);
  b.nbz = bricks_along(m.nz);
  b.K = K;
  b.P = (int)P;
  return b;
}

// ---------------------------------------------------------------- conv layers
int conv_splits(long wgs, int nchunks, int target) {
  // grow the split until the layer has `target` workgroups; keep at least
  // two chunks per split
  int s = 1;
  while (wgs * s < target && 2 * (s * 2) <= nchunks && s < 16) s *= 2;
  return s;
}

// Tile height and split-K factor of conv layer i at level size h x w (tiles
// of th x 16 pixels x 32 output channels); the 3-channel input layer is
// never split.  The split grows until the layer has 256 workgroups (fp32) or
// 512 (bf16, fp8), the targets measured fastest per precision with the
// split-K reductions counted.  fp32 and bf16 layers take 4-row tiles where
// that needs a smaller split than 8-row tiles (the deep levels: twice the
// workgroups without partial sums to write, read and reduce) or where 8-row
// tiles leave one workgroup per CU (nothing else on the CU hides a
// workgroup's chunk-boundary stalls): 5 us per fp32 frame, 9 us per bf16
// frame.  fp8 layers, whose LDS footprint lets five 4-row workgroups share
// a CU, take 4-row tiles throughout: 19 us per frame.  Large bf16 layers
// take the 8-row x 64-channel form when it still gives two workgroups per
// CU.
//
// The split and the tile height follow the workgroup count of one image, so
// an image's sums (whose order the split sets) are the same alone and in any
// batch; only the bf16 large form, which sums in the same order as the
// default form, looks at the batch.
LayerTiling conv_layer_tiling(const lnm_net_s* net, int i, int B, int h, int w) {
  const LayerDesc& d = net->layers[i];
  if (d.ci == 3) return {8, 1};
  const int target = d.prec == LNM_FP32 ? 256 : 512, nch = d.ci_pad / d.ck;
  auto wgs = [&](int th) { return (long)((w + 15) / 16) * ((h + th - 1) / th) * (d.co_pad / kBN); };
  const int s8 = conv_splits(wgs(8), nch, target);
  if (d.prec == LNM_BF16 && s8 == 1) {
    // large bf16 layers: the 64-channel tile, when it still gives two
    // workgroups per CU
    const int nt = d.co_pad / kBN;
    const long large =
        (long)((w + 15) / 16) * ((h + kBf16LargeRows - 1) / kBf16LargeRows) * B * ((nt + 1) / 2);
    if (nt >= 2 && large >= 512) return {kBf16Large, 1};
  }
  const bool fp8 = d.prec == LNM_FP8_E4M3;
  if (s8 > 1 || wgs(8) <= 256 || fp8) {
    // the longest fp32 layers (16+ chunks) split on to two workgroups per CU
    const int s4 = conv_splits(wgs(4), nch, d.prec == LNM_FP32 && nch >= 16 ? 512 : target);
    if (s4 < s8 || wgs(8) <= 256 || fp8) return {4, s4};
  }
  return {8, s8};
}

// ---------------------------------------------------------------- channel adapters
bool adapter_width_supported(int c) { return c == 16 || c == 32 || c == 48 || c == 64; }

int adapter_tail_blocks_per_image(int H, int W) { return (H * W + 255) / 256; }

size_t adapter_wgrad_partial_bytes(size_t P, int c) {
  return sizeof(float) * ((P + kAdaptWgradChunk - 1) / kAdaptWgradChunk) * 2 * (size_t)c * c;
}

int adapter_tiles(int H, int W) {
  return ((H + kAdaptTileY - 1) / kAdaptTileY) * ((W + kAdaptTileX - 1) / kAdaptTileX);
}

}  // namespace lnm
