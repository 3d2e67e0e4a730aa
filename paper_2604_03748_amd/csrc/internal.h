// Internal declarations shared by the liblnm translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lnm.h"

namespace lnm {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
lnm_status fail(lnm_status st, const std::string& msg);
#define LNM_HIP_CHECK(expr)                                                              \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return ::lnm::fail(LNM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------- camera
// Camera basis prepared on the host in fp64 and rounded once to fp32.
struct CamDev {
  float eye[3], f[3], r[3], u[3];
  float tan_half, half_extent, aspect;
  int proj, W, H;
};
bool make_cam(const lnm_camera& c, CamDev* out, std::string* why);

// ---------------------------------------------------------------- march
struct MarchDev {
  const float* rho;  // caller's linear grid, x fastest
  int nx, ny, nz;
  float sigma_scale;
  float h;        // world step
  float depth_tau;
  float tau_max;  // -ln(eps), +inf when disabled
  int jitter_on;
  uint64_t seed;
  uint32_t frame;
  int quadrature;
  float wf, wt, wb;  // front and side light intensities
  int light_set;     // lnm_light_set
  int zorder;        // order of the light marches (march_order): bands, z layers or z cells
  const float* brick;  // bricked copy of rho (4^3 cells + apron per 128-float slot); caller's or scratch
  int nbx, nby, nbz;   // bricks per axis
};

struct MarchBuf {
  float* t;    // [K][P] sample parameter t_n
  float* a;    // [K][P] weight A_n
  float* tp;   // [K][P] transmittance before the sample, T_{n-1}
  float* tl;   // [2][K][P] transmittance toward the top / bottom (first / second side) light
  int* cnt;    // [P] recorded samples per pixel
  int* ctr;    // counter block: entries in each band's work list, the z-order unit counters, start[0..9)
               // of the bands' tile ranges, the records per z bucket and the z-order scatter cursors
  int2* rec;   // work lists of the primary march, (pixel, k); band e's from entry start[e] * 64 * K
               // (NULL in cell order)
  size_t cap;  // entries per band at equal bands (the lists hold 8 * cap)
  uint8_t* zb;  // z order: [K][P] z bucket (brick layer) of each record's sample, else NULL
  int2* srt;    // z order: [P * K] the records of all bands in z-bucket order, else NULL
  float* brick;
  int nbx, nby, nbz;
  int K, P;  // capacity per pixel, pixels
};

// Band order of the 8x8 pixel tiles; per_xcd = tiles / 8 rounded up, the
// primary march's workgroups per band.
struct TileMap {
  int tiles_x, tiles_y, per_xcd, band_rows;
};
// The march's layout constants.  kBrickSlot: floats per brick (5^3 values
// of a 4^3-cell brick and the next layer, padded).  kTile: side of the
// primary march's screen tiles.  The counter block (ints): the 8 band
// counters, the light marches' per-XCD next-unit counters from kUnitNext (z
// order), start[0..8] of the band tile ranges from kBandStart, the record
// count of each z bucket from kZHist and the z-order scatter cursors from
// kZCursor.
constexpr int kBrickSlot = 128;
constexpr int kTile = 8;
constexpr int kUnitNext = 8, kBandStart = 16;
constexpr int kZBuckets = 256;
constexpr int kZHist = 32, kZCursor = kZHist + kZBuckets;
constexpr size_t kCounterBytes = 4 * (kZCursor + kZBuckets);
// Bricks along an axis of n cells; bytes of a z cell's two grid planes in LDS.
int bricks_along(int n);
size_t cell_planes_bytes(int nx, int ny);
// LDS the cell order's plane pairs may take (the rest of the CU's 160 KB
// holds the kernel's own bookkeeping)
constexpr size_t kCellLdsBytes = 160 * 1024 - 4 * 1024;
// Capacity per pixel: the most primary samples a ray can take in the support box.
int march_capacity(const MarchDev& m);
// Order of a march's light marches (MarchDev::zorder) for lnm_work_order
// work_order; AUTO: z layers for grids whose bricks exceed the XCDs' L2s
// together, z cells for the top/bottom lights when a cell's two grid planes
// fit in LDS, else bands; -1 when LNM_ORDER_CELLS does not fit.
constexpr int kOrderBands = 0, kOrderLayers = 1, kOrderCells = 2;
int march_order(int work_order, int light_set, int nx, int ny, int nz);
// Scratch of one march; the bricked grid is part of it unless m.brick is set.
size_t march_scratch_bytes(const MarchDev& m, int K, int W, int H);
MarchBuf march_buffers(void* ws, const MarchDev& m, int K, int W, int H);
size_t bricks_bytes(int nx, int ny, int nz);
hipError_t launch_relayout(const MarchDev& m, float* bricks, hipStream_t s);
hipError_t launch_march(const MarchDev& m, const CamDev& cam, const MarchBuf& buf, float* guide, hipStream_t s);
hipError_t launch_reference(const MarchDev& m, const CamDev& cam, int srgb, float* lm, hipStream_t s);

// ---------------------------------------------------------------- network
constexpr int kBN = 32;  // output-channel tile of the conv kernels

enum Gather : int { G_GUIDE = 0, G_PLAIN = 1, G_POOL = 2, G_CONCAT_UP = 3, G_FIRST = 4 };

struct LayerDesc {
  int ci, co, k;
  int ck;        // input-channel chunk of the packed layout
  int ci_pad;    // ci rounded up to ck
  int co_pad;    // co rounded up to kBN
  size_t w_off;  // byte offset of the packed weights in the device buffer
  size_t b_off;  // byte offset of the fp32 biases (co_pad of them)
  size_t s_off;  // byte offset of fp32 per-output-channel weight scales (fp8)
  int prec;      // the layer's weights and matrix arithmetic (lnm_precision)
  int out_es;    // bytes per stored output element: 4 fp32, 2 bf16, 1 e4m3
};

// Activation element types: fp32 (4 bytes), bf16 (2), fp8 e4m3 (1).
struct ConvArgs {
  const void* src0;   // input (guide / plain / pooled source / skip)
  const void* src1;   // low-resolution tensor for concat-upsample
  int c0, c1;         // channels of src0 and src1
  int B, H, W;        // output spatial size
  int ci_pad, co;     // padded input channels, real output channels
  const void* w;      // packed weights
  const float* bias;  // [co_pad]
  void* out;          // [B][H][W][co]
  int relu;
  // fp8 form: y = in_scale * w_scale[o] * acc + bias; stored as y * out_inv_scale
  const float* w_scale;
  float in_scale, out_inv_scale;
  // split-K: blockIdx.z = n_tile + n_tiles * split; with splits > 1 each split
  // writes its raw fp32 sums to partial[split][pixel][co] and
  // launch_splitk_reduce finishes the layer
  int n_tiles, splits;
  float* partial;
  int th;  // tile height in rows: 4 or 8 (0 means 8; the input layer always 8); kBf16Large: the
           // bf16 large-layer form (kBf16LargeRows rows x 64 channels per workgroup; n_tiles >= 2,
           // no head)
  int out_bf16;  // fp8 layers: store max(y, 0) as bf16 (unscaled) instead of e4m3
  // G_FIRST: src0 is the guide and the layer's input is the network's first
  // layer, recomputed per tile from its packed weights and bias (fp8: stored
  // as e4m3 of y * w0_out_inv, the first layer's output scale)
  const void* w0;
  const float* b0;
  float w0_out_inv;
};
// Sum the split partials in split order, then bias, (scale,) ReLU and the
// output conversion of out_type (0 fp32, 1 bf16, 2 fp8; 3: fp8 partials,
// scaled like 2, stored as bf16).
hipError_t launch_splitk_reduce(const ConvArgs& a, int out_type, hipStream_t s);
// Splits for a layer launched with `wgs` workgroups over `nchunks` input chunks.
int conv_splits(long wgs, int nchunks, int target);
// Tile height (4 or 8 rows) and split-K factor of conv layer i of `net` at
// level size h x w and batch B.
struct LayerTiling {
  int th, splits;
};
// The bf16 large-layer tile (ConvArgs::th code and its height in rows).
constexpr int kBf16Large = 16, kBf16LargeRows = 8;
LayerTiling conv_layer_tiling(const lnm_net_s* net, int i, int B, int h, int w);
struct HeadFuse;
// head: the layer's epilogue also applies the 1x1 head (plain-input layers
// of at most 32 output channels, unsplit), instead of storing the layer
hipError_t launch_conv3x3_f32(int mode, int ck, const ConvArgs& a, hipStream_t s, const HeadFuse* head = nullptr);
hipError_t launch_conv3x3_bf16(int mode, const ConvArgs& a, hipStream_t s, const HeadFuse* head = nullptr);
hipError_t launch_conv3x3_fp8(int mode, const ConvArgs& a, hipStream_t s, const HeadFuse* head = nullptr);
constexpr int kAmaxBlocks = 256;
// max |x| over n floats into *out (partial: kAmaxBlocks floats of scratch)
hipError_t launch_amax(const float* x, long n, float* partial, float* out, hipStream_t s);

struct HeadArgs {
  const void* in;   // [P][C] activations of the last decoder layer
  int in_type;      // 0 fp32, 1 bf16, 2 fp8
  float in_scale;   // fp8 dequantisation scale
  int P, C;
  const float* w;   // [6][C]
  const float* b;   // [6]
  float* lm;        // [P][6] sigmoid output
  float* logits;    // optional [P][6]
};
struct CompositeArgs;
// comp: also shade each pixel (the frame's head and composite in one launch)
hipError_t launch_head(const HeadArgs& a, hipStream_t s, const CompositeArgs* comp = nullptr);

struct CompositeArgs {
  const float* lm;     // [P][6]
  const float* guide;  // [P][3]
  float* rgba;         // [P][4]
  int P;
  int n_lights;
  float l[16][3];      // light direction in the camera frame
  float rgb[16][3];
};
hipError_t launch_composite(const CompositeArgs& a, hipStream_t s);

// Shading of a batch of equally sized images, each with its own camera
// frame and lights: image b takes lights [light_lo[b], light_lo[b + 1]).
constexpr int kBatchShadeImages = 64, kBatchShadeLights = 64;
struct CompositeBatchArgs {
  const float* lm;     // [B][P][6]
  const float* guide;  // [B][P][3]
  float* rgba;         // [B][P][4]
  int P, B;            // pixels per image, images
  int light_lo[kBatchShadeImages + 1];
  float l[kBatchShadeLights][3];  // light direction in its image's camera frame
  float rgb[kBatchShadeLights][3];
};
hipError_t launch_composite_batch(const CompositeBatchArgs& a, hipStream_t s);

// The 1x1 head (+ sigmoid, + optional shading) applied in the last fp32 conv
// layer's epilogue: that layer's workgroup holds all its channels.
struct HeadFuse {
  const float* w;      // [6][C] head weights (C = the layer's output channels)
  const float* b;      // [6]
  float* lm;           // [P][6] lightmaps
  CompositeArgs comp;  // comp.rgba == nullptr: no shading
  float in_scale;      // e4m3 layers: the scale of the layer's stored activations
};

// ---------------------------------------------------------------- channel adapters
struct AdapterArgs {
  const void* feat;   // decoder output [P][c] in the network's precision
  float feat_scale;   // e4m3 features: their scale
  const float* prm;   // four adapters' parameters (parameter-file order)
  int B, H, W;
  size_t P;           // B H W
  float* v;           // [4][P][c] gated depthwise outputs
  float* part;        // [B][4][n_blk][c] per-tile sums of v
  int n_blk;          // adapter tiles per image (adapter_tiles)
  float* sca;         // [B][4][c] attention scales
  float* lm;          // [P][6]
  float* extra;       // [P][2] or NULL
  float* dsave;       // training: [4][P][2c] depthwise outputs, else NULL
  float* msave;       // training: [B][4][c] image means of v, else NULL
};
// the adapters' first kernel works on tiles of 8 x 32 pixels
constexpr int kAdaptTileY = 8, kAdaptTileX = 32;
int adapter_tiles(int H, int W);
bool adapter_width_supported(int c);
// Training of the adapters with the network (adapters_train.hip): the three
// groups with a lightmap target; per-pixel tensors [3][P][..]
struct AdapterTrainArgs {
  AdapterArgs f;           // forward (feat: the fp32 decoder output), dsave and msave set
  const float* target;     // [P][6] sRGB
  float* grad;             // adapter parameter gradient (parameter-file order), written
  float *dgt, *dyf, *dxf;  // [3][P][c] gate gradient (tail side), features' gradient (tail, front side)
  float *d5, *x5, *d3, *x3, *x4, *x1;  // [3][P][c] deltas and inputs of the 1x1 convolutions
  float *d4, *d1;          // [3][P][2c]
  float* tpart;            // [3][B * tpi][11c + 4] tail workgroup sums
  float* fpart;            // [3][B][n_blk][24c] front workgroup sums
  float* dmh;              // [B][4][c] image-mean term of the gate gradient
  float* lossg;            // [3] squared-error sums per group
  float* loss;             // the loss (1 float)
  int tpi;                 // tail workgroups per image (adapter_tail_blocks_per_image)
  float inv_n;             // 1 / (P * 6)
};
constexpr int kAdaptWgradChunk = 1024;  // pixels per partial sum of a 1x1 weight gradient
int adapter_tail_blocks_per_image(int H, int W);
size_t adapter_wgrad_partial_bytes(size_t P, int c);
// adapters' forward (keeping d, m), backward, weight gradients, and the
// features' gradient through the decoder's ReLU into g_last
hipError_t launch_adapters_train(int c, const AdapterTrainArgs& t, const float* y_last, float* g_last, float* wpart,
                                 hipStream_t s);
hipError_t launch_fill_zero(float* p, long n, hipStream_t s);
hipError_t launch_adapters(int c, const AdapterArgs& a, int in_type, hipStream_t s);
// the first two kernels only (v, the tile sums, the attention scales; with
// dsave and msave set, also d and m)
hipError_t launch_adapters_front(int c, const AdapterArgs& a, int in_type, hipStream_t s);

// ---------------------------------------------------------------- shadows
struct ShadowArgs {
  CompositeArgs c;
  CamDev cam;
  float origin[3];
  float E;  // half extent of the shadow maps
  int S;    // texels per side
  float bias;
  float e1[16][3], e2[16][3], lw[16][3];  // light space of each light (world)
  const float* depth[16];                 // [S][S] per light, NULL = unshadowed
  float* vis;                             // optional [n_lights][P]
};
hipError_t launch_shadow_map_sphere(int S, float E, float cu, float cv, float cz, float r2, float* depth,
                                    hipStream_t s);
hipError_t launch_composite_shadowed(const ShadowArgs& a, hipStream_t s);

}  // namespace lnm

struct lnm_ctx_s {
  int device;
  int cu_count;
  std::string arch;
  // per-launch timing (lnm_profile_enable)
  bool prof = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  // device address of the static frame workspace (LNM_STATIC_SCRATCH_BYTES)
  // on this context's device, looked up once at creation
  void* static_scratch = nullptr;
};

namespace lnm {
// Brackets one kernel launch with events when the context is profiling.
class ProfScope {
 public:
  ProfScope(lnm_ctx_s* ctx, int kind, hipStream_t s);
  ~ProfScope();

 private:
  lnm_ctx_s* ctx_;
  hipStream_t s_;
  int idx_ = -1;
};
}  // namespace lnm

struct lnm_adapters_s {
  const lnm_net_s* net;
  int c;
  float* dev;  // caller-owned parameter buffer
};

struct lnm_net_s {
  int levels, base, precision;
  std::vector<lnm::LayerDesc> layers;
  char* dev;  // caller-owned buffer
  size_t dev_bytes;
  std::vector<float> act_scale;  // fp8: per stored activation tensor (one per conv layer + the guide)
};

namespace lnm {
// ---------------------------------------------------------------- network helpers (api.hip)
int elem_bytes(int precision);
size_t align256(size_t x);
bool net_shape(int levels, int base, int precision, std::vector<LayerDesc>* out, size_t* dev_bytes, std::string* why);
size_t param_count(int levels, int base);
constexpr size_t kScratchBytes = 64 * 1024;  // small reductions (calibration)
struct Plan {
  std::vector<size_t> out_off;  // byte offset of each conv layer's output
  size_t partial_off;           // split-K partial sums (largest split layer)
  size_t scratch_off;           // kScratchBytes of scratch after the activations
  size_t bytes;
};
Plan plan_workspace(const lnm_net_s* net, int B, int H, int W);
// comp (batch 1): shade each pixel in the head launch as well.  fuse_head:
// an fp32 network may apply the head in its last conv layer's epilogue (that
// layer's output is then not stored; callers that read it pass false)
lnm_status run_unet(lnm_ctx_s* ctx, const lnm_net_s* net, int B, int H, int W, const float* guide, float* lm,
                    float* logits, char* ws, hipStream_t s, const CompositeArgs* comp = nullptr,
                    bool fuse_head = false, bool fuse_first = false);
lnm_status check_infer(const lnm_net_s* net, int B, int H, int W, size_t ws_bytes, const void* ws);
// lnm_frame on a caller's (or the library's static) workspace, and its size
lnm_status frame_impl(lnm_ctx_s* ctx, const lnm_net_s* net, const lnm_volume* vol, const lnm_camera* cam,
                      const lnm_march_params* prm, const lnm_light* lights, int n_lights, float* guide,
                      float* lightmaps, float* rgba, void* workspace, size_t ws_bytes, void* stream);
size_t frame_workspace_bytes(const lnm_net_s* net, const lnm_volume* vol, const lnm_camera* cam,
                             const lnm_march_params* prm);
// Device address of the library's static frame workspace on the current
// device (frame_static.hip); call with that device current.
hipError_t static_scratch_address(void** out);

// ---------------------------------------------------------------- training kernels (train.hip)
// Layer geometry shared by the backward kernels.
struct WgradArgs {
  ConvArgs x;       // the layer's (virtual) input, as the forward gather sees it
  const float* e;   // [B][H][W][co] gradient at the pre-activation
  int co, ci;       // real channels
  int ci_pad16;     // ci rounded up to 16
  int tiles_per_group;
  float* partial;   // [groups * 4][co_pad][ci_pad16][9]
};
hipError_t launch_wgrad3x3(int mode, const WgradArgs& a, int* n_partials, hipStream_t s);
hipError_t launch_wgrad_reduce(const float* partial, int n_partials, int co, int ci, int co_pad, int ci_pad16,
                               float* grad_w, hipStream_t s);
hipError_t launch_loss(const float* y, const float* t, float* dz, float* partial, long n, float* loss,
                       hipStream_t s);
hipError_t launch_colsum(const float* e, long P, int C, float* partial, float* out, hipStream_t s);
hipError_t launch_relu_mask(float* g, const float* y, long n, hipStream_t s);
hipError_t launch_head_bwd(const float* dz, const float* w, const float* x, long P, int C, float* e_out,
                           float* grad_w, float* grad_b, float* partial, hipStream_t s);
hipError_t launch_route_concat(const float* dx, int B, int H, int W, int c0, int c1, float* g_skip, float* g_low,
                               hipStream_t s);
hipError_t launch_route_pool(const float* dx, const float* y, int B, int h, int w, int c, float* g, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t s);
// Repack flat parameters into the fp32 forward layout (dgrad = 0) or the
// transposed, tap-flipped layout used to propagate gradients (dgrad = 1).
hipError_t launch_pack_f32(const float* flat_w, const float* flat_b, const LayerDesc& d, int dgrad, char* dst,
                           size_t w_off, size_t b_off, hipStream_t s);
constexpr int kLossBlocks = 256;
constexpr int kColsumBlocks = 128;
}  // namespace lnm

struct lnm_trainer_s {
  lnm_ctx_s* ctx;
  lnm_net_s net;         // fp32 forward weights inside the state buffer
  char* state;
  size_t n_params;
  float *p, *g, *m, *v;  // flat, parameter-file order
  std::vector<size_t> flat_w, flat_b;  // per layer offsets (floats) in the flat vector
  std::vector<lnm::LayerDesc> dgrad;   // transposed layout per layer (layer 0 unused)
  std::vector<size_t> dgrad_off;       // byte offset of each transposed weight block in the state
  float* zeros;          // zero bias for the data-gradient convolutions
  int step;
  // channel adapters trained with the network (attached before the first
  // step): width, parameter count, flat parameters, gradient, Adam moments
  int ad_c = 0;
  size_t ad_n = 0;
  float *ad_p = nullptr, *ad_g = nullptr, *ad_m = nullptr, *ad_v = nullptr;
};
