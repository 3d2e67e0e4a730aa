/*
 * lnm.h -- C ABI of liblnm, the MI355X (gfx950) library for the hot path of
 * "Real-time Neural Six-way Lightmaps": a coarse-step ray march of a smoke
 * density grid that produces a per-pixel guiding map, and a U-Net that maps
 * the guiding map to six directional lightmaps, followed by six-way shading.
 *
 * Conventions for every call:
 *  - Tensor pointers are DEVICE pointers owned by the caller, contiguous, and
 *    16-byte aligned (torch allocations are).  The library never keeps a
 *    pointer past the call except the weight buffer handed to lnm_net_create,
 *    which must outlive the net.
 *  - Calls enqueue work on `stream` (a hipStream_t passed as void*; NULL is the
 *    default stream) and return without synchronising, except where stated.
 *  - Every call validates its arguments before enqueuing anything; on error
 *    nothing is enqueued, a status is returned and lnm_last_error() describes
 *    it.  Nothing aborts and no exception crosses the ABI.
 *  - Floating-point inputs and outputs are fp32.  Layouts are row-major with
 *    the last index fastest.  Images are [batch][row][column][channel], row 0
 *    at the top.
 *  - World space is the unit cube [0,1]^3 holding the grid; voxel (i,j,k)
 *    of an [nz][ny][nx] grid has centre ((i+1/2)/nx, (j+1/2)/ny, (k+1/2)/nz).
 */
#ifndef LNM_H
#define LNM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LNM_API __attribute__((visibility("default")))

typedef enum {
  LNM_OK = 0,
  LNM_ERR_ARG = 1,         /* NULL pointer, non-finite or out-of-range value */
  LNM_ERR_SHAPE = 2,       /* inconsistent or unsupported sizes; workspace too small */
  LNM_ERR_OOM = 3,         /* a host allocation failed */
  LNM_ERR_DEVICE = 4,      /* a HIP runtime call failed */
  LNM_ERR_UNSUPPORTED = 5  /* valid request the library does not implement */
} lnm_status;

typedef enum { LNM_FP32 = 0, LNM_BF16 = 1, LNM_FP8_E4M3 = 2 } lnm_precision;
typedef enum { LNM_ORTHOGRAPHIC = 0, LNM_PERSPECTIVE = 1 } lnm_projection;
/* Weight of sample n in Algorithm 1: ALPHA = T_{n-1} (1 - exp(-sigma_n h)),
 * RIEMANN = T_{n-1} sigma_n h (the algorithm's term with the step length). */
typedef enum { LNM_QUAD_ALPHA = 0, LNM_QUAD_RIEMANN = 1 } lnm_quadrature;
/* Side lights of the guiding map (see lnm_march_params). */
typedef enum { LNM_LIGHTS_TOP_BOTTOM = 0, LNM_LIGHTS_LEFT_RIGHT = 1 } lnm_light_set;
/* Order in which the march hands its light marches to the GPU's XCDs (see
 * lnm_march_params); the guiding map is the same, bit for bit, in every
 * order.  LNM_ORDER_BANDS: screen bands (best when the bricked grid fits the
 * XCDs' L2 caches); LNM_ORDER_Z: the samples sorted by brick layer first
 * (best for large grids, one more kernel and a larger workspace);
 * LNM_ORDER_CELLS: the samples sorted by the grid cell of their z, each
 * workgroup reading the two grid planes of its cell from LDS (grids with
 * (nx + 2)(ny + 2) <= 19968 and nz < 256; LNM_ERR_UNSUPPORTED otherwise);
 * LNM_ORDER_AUTO: z order when the bricked grid exceeds 32 MiB, else cells
 * for the top/bottom lights when they fit, else bands. */
typedef enum { LNM_ORDER_AUTO = 0, LNM_ORDER_BANDS = 1, LNM_ORDER_Z = 2, LNM_ORDER_CELLS = 3 } lnm_work_order;

typedef struct lnm_ctx_s* lnm_ctx; /* per-device state: properties, error text */
typedef struct lnm_net_s* lnm_net; /* host descriptor of a packed network */

/* Density grid: the scattering coefficient sigma_s(x) = sigma_scale * rho~(x)
 * where rho~ is the zero-border, cell-centred trilinear interpolation of
 * `density` (Section 4.2 keeps sigma_s in a 3D texture).  sigma_t = sigma_s.
 * The march reads the grid as 4^3-cell bricks: by default each march call
 * builds them in its workspace; a caller that marches the same grid many
 * times may build them once with lnm_make_bricks and pass them in `bricks`
 * (the march then trusts that they were made from `density` and these
 * dimensions, and needs a smaller workspace). */
typedef struct {
  const float* density; /* device, [nz][ny][nx], x fastest */
  int32_t nx, ny, nz;   /* each >= 1 */
  float sigma_scale;    /* >= 0 */
  const float* bricks;  /* device, from lnm_make_bricks, or NULL */
} lnm_volume;           /* 32 bytes */

/* Pinhole or orthographic camera.  forward f = normalize(target - eye),
 * right r = normalize(f x up), up' = r x f.  Pixel (i, j) has screen
 * coordinates sx = 2(i+1/2)/W - 1, sy = 1 - 2(j+1/2)/H; a perspective ray is
 * d = normalize(f + tan(fov_y/2)(sx (W/H) r + sy up')) from the eye; an
 * orthographic ray starts at eye + e (sx (W/H) r + sy up') with d = f. */
typedef struct {
  int32_t projection;      /* lnm_projection */
  float eye[3], target[3], up[3];
  float fov_y_deg;         /* perspective: (0, 180) */
  float ortho_half_extent; /* orthographic: e > 0 */
  int32_t width, height;   /* W, H >= 1 */
} lnm_camera;              /* 56 bytes */

/* Parameters of the guiding-map march (Algorithm 1, Section 4.2).
 * h = step_voxels / max(nx, ny, nz) (the paper uses 10 voxels).
 * Samples sit at t_n = (n + u) h, n >= 1, u the per-ray jitter.
 * D = n h at the first sample with sigma_n > depth_tau (0 = no surface).
 * Early termination: the march stops after a sample whose transmittance is
 * below ert_eps and then reports T = 0; a light march stops when its optical
 * depth exceeds -ln(ert_eps) and reports 0.  ert_eps = 0 disables both.
 * Jitter u = (SplitMix64(jitter_seed ^ (frame << 32) ^ pixel) >> 40) / 2^24,
 * pixel = row * W + column, where SplitMix64(s) is the generator's output for
 * state s (finaliser of s + 0x9E3779B97F4A7C15); u = 0 when jitter_on = 0.
 * light_w = intensities of the front light and the two side lights
 * (front = w = -d).  light_set picks the side lights: LNM_LIGHTS_TOP_BOTTOM
 * (the method's set, Section 4.2) top = normalize(w x z), bottom = -top, with
 * the limit normalize(w x x) when w is parallel to z; LNM_LIGHTS_LEFT_RIGHT
 * (the alternative of the guiding-light ablation, Section 5) left =
 * normalize(w x top), right = -left.  The front-only configuration is
 * light_w = (1, 0, 0).  The phase function is isotropic. */
typedef struct {
  float step_voxels;  /* > 0 */
  float depth_tau;    /* >= 0 */
  float ert_eps;      /* in [0, 1) */
  int32_t jitter_on;
  uint64_t jitter_seed;
  uint32_t frame;
  int32_t quadrature; /* lnm_quadrature */
  float light_w[3];   /* front, first side, second side */
  int32_t light_set;  /* lnm_light_set */
  int32_t work_order; /* lnm_work_order; 0 (auto) for a zeroed struct */
} lnm_march_params;   /* 56 bytes */

/* A directional light for six-way shading: dir points toward the light (need
 * not be unit length; its camera-frame components weight the lightmaps). */
typedef struct {
  float dir[3];
  float rgb[3];
} lnm_light; /* 24 bytes */

/* Light space shared by the obstacle shadow maps (Section 4.5).  A light
 * with unit direction l (toward the light) gets the orthographic frame
 * e1 = normalize(a x l), a = +y (+x when |l_y| > 0.99), e2 = l x e1, and
 * coordinates (u, v, z) = ((p - origin).e1, (p - origin).e2, (p - origin).l).
 * Its shadow map is size x size texels over u, v in [-half_extent,
 * half_extent] (texel (i, j) covers u in [-E + 2E i/S, -E + 2E (i+1)/S),
 * row j likewise in v), each holding the largest z of the obstacle along the
 * texel centre's light ray (the occluder surface nearest the light), -inf
 * where there is none.  A smoke point at z is shadowed when its texel holds
 * a depth greater than z + bias. */
typedef struct {
  float origin[3];
  float half_extent;
  int32_t size;
  float bias;
} lnm_shadow_frame; /* 24 bytes */

/* sizeof of the structs above as compiled into the library, for bindings:
 * which = 0 volume, 1 camera, 2 march params, 3 light, 4 shadow frame; 0 for
 * other values. */
LNM_API size_t lnm_abi_struct_size(int32_t which);
/* Library version string (static storage). */
LNM_API const char* lnm_version(void);

/* Create a context bound to HIP device `hip_device` (made current on the
 * calling thread).  Reads device properties; allocates only host memory. */
LNM_API lnm_status lnm_ctx_create(int32_t hip_device, lnm_ctx* out);
LNM_API void lnm_ctx_destroy(lnm_ctx ctx);
/* Text of the last error reported on the calling thread ("" if none); valid
 * until the next library call on this thread. */
LNM_API const char* lnm_last_error(void);

/* ------------------------------------------------------------------ march */
/* Bytes of the bricked copy of an nx x ny x nz grid: ((n >> 2) + 1) bricks
 * per axis, 512 bytes each; 0 on invalid sizes. */
LNM_API size_t lnm_bricks_bytes(int32_t nx, int32_t ny, int32_t nz);
/* Build the bricked copy of vol->density into `bricks` (device, at least
 * lnm_bricks_bytes): grid index i + 1 (a zero layer on each side) cut into
 * bricks of 4 cells per axis, each storing its 5 x 5 x 5 values (the next
 * layer included) x fastest in a 128-float slot, bricks x fastest.
 * vol->bricks is ignored.  Stream ordered. */
LNM_API lnm_status lnm_make_bricks(lnm_ctx ctx, const lnm_volume* vol, float* bricks, size_t bytes, void* stream);

/* Device workspace (bytes) the march needs for this volume, camera and step:
 * per pixel, records of up to K primary samples (K bounded by the support
 * box diagonal over h) and their light terms, in z order (prm->work_order)
 * also a z-bucket byte and a sorted-list entry per record, plus the bricked
 * grid unless vol->bricks is given; 0 on invalid arguments. */
LNM_API size_t lnm_march_workspace_bytes(const lnm_volume* vol, const lnm_camera* cam,
                                         const lnm_march_params* prm);

/* Guiding map G[H][W][3] = (L~_scattering, T, D) per pixel: Algorithm 1 with
 * the three surrogate lights of Eq. approx (Section 4.2).  L~ = sum_n A_n L_n
 * with L_n = w_f T_{n-1} + w_t T^top_n + w_b T^bot_n, where T^top_n, T^bot_n
 * march from sample n to the grid's support box at step h.  Optical depth is
 * accumulated in fp32.  `guide` is device memory of 3 W H floats. */
LNM_API lnm_status lnm_march(lnm_ctx ctx, const lnm_volume* vol, const lnm_camera* cam, const lnm_march_params* prm,
                     float* guide, void* workspace, size_t ws_bytes, void* stream);

/* n guiding maps in one call (ragged: each march i has its own grid, camera,
 * parameters and guides[i], of 3 W_i H_i floats), e.g. one per request of a
 * serving batch (Algorithm 1 per map, as lnm_march).  The marches run in
 * order on `stream` and share the one workspace, which must hold the largest
 * of them: at least lnm_march_batch_workspace_bytes.  Every argument is
 * checked before anything is enqueued; n in [1, 4096]. */
LNM_API size_t lnm_march_batch_workspace_bytes(int32_t n, const lnm_volume* vols, const lnm_camera* cams,
                                               const lnm_march_params* prms);
LNM_API lnm_status lnm_march_batch(lnm_ctx ctx, int32_t n, const lnm_volume* vols, const lnm_camera* cams,
                                   const lnm_march_params* prms, float* const* guides, void* workspace,
                                   size_t ws_bytes, void* stream);

/* Fine-step six-way reference lightmaps lm[H][W][6] used as training targets
 * (they replace the offline path-traced references of Section 5): order
 * (+X, -X, +Y, -Y, +Z, -Z) of the camera frame (X = right, Y = up, Z = toward
 * the camera); L_a = sum_n A_n T^a_n with alpha weights, no jitter, step
 * step_voxels, T^a_n the transmittance from sample n toward axis a.  With
 * srgb != 0 the values are sRGB-encoded (IEC 61966-2-1), else linear. */
LNM_API lnm_status lnm_reference_lightmaps(lnm_ctx ctx, const lnm_volume* vol, const lnm_camera* cam, float step_voxels,
                                   float ert_eps, int32_t srgb, float* lm, void* stream);

/* ------------------------------------------------------------------ network */
/* The U-Net of Section 4.3 with L levels of widths C_l = base 2^l: two 3x3
 * convolutions (zero padding 1) + bias + ReLU per encoder level, then 2x2
 * max-pooling; two at the bottleneck; per decoder level nearest 2x upsampling,
 * concat(skip, up) and two 3x3 convolutions + ReLU; a 1x1 head to 6 channels
 * and a sigmoid.  Parameters are a flat fp32 vector: per layer (enc0a, enc0b,
 * ..., bottleneck a/b, dec(L-2)a ... dec0b, head) W[C_out][C_in][k][k] then
 * b[C_out]. */
LNM_API size_t lnm_net_param_count(int32_t levels, int32_t base);
/* Bytes of device memory the packed weights need at this precision. */
LNM_API size_t lnm_net_device_bytes(int32_t levels, int32_t base, int32_t precision);
/* Pack host parameters into `device_buf` (caller-owned, >= device_bytes,
 * must outlive the net, 256-byte aligned).  Synchronises `stream` before
 * returning.
 * precision: LNM_FP32 (fp32 weights and activations), LNM_BF16 (bf16 weights
 * and activations rounded to nearest even, fp32 accumulation, bias and ReLU
 * on the fp32 accumulator, fp32 head), LNM_FP8_E4M3 (OCP e4m3 weights with
 * one scale per output channel, max|W[o]|/448; activations stored as e4m3
 * with one scale per tensor, 4 amax/448 (headroom for inputs beyond the
 * calibrated maxima), the two inputs of each decoder
 * concatenation sharing the larger; fp32 accumulation; the 3-channel input
 * layer and the last 3x3 layer, whose features the head reads, in bf16, the
 * layer before that storing bf16 for it).  Other values:
 * LNM_ERR_UNSUPPORTED.
 * act_scales: LNM_FP8_E4M3 only (else NULL): the calibrated maximum |output|
 * of each convolution layer (4 levels - 2 floats, see lnm_calibrate_amax).
 * levels in [2, 6]; base in [1, 256] with base multiple of 16 for levels
 * whose skip must align to 16-channel chunks (base % 16 == 0 required). */
LNM_API lnm_status lnm_net_create(lnm_ctx ctx, int32_t levels, int32_t base, int32_t precision, const float* host_params,
                          size_t n_params, const float* act_scales, void* device_buf, size_t device_buf_bytes,
                          void* stream, lnm_net* out);
LNM_API void lnm_net_destroy(lnm_net net);

/* Calibration for the FP8 form: run an LNM_FP32 net on guide[B][H][W][3] and
 * write, per convolution layer in parameter-file order, the maximum |output|
 * to host_amax (n = 4 levels - 2 floats).  The maxima of a calibration set
 * (element-wise maximum over calls) are the act_scales of lnm_net_create for
 * LNM_FP8_E4M3.  Synchronises `stream`. */
LNM_API lnm_status lnm_calibrate_amax(lnm_ctx ctx, lnm_net net, int32_t batch, int32_t H, int32_t W,
                                      const float* guide, float* host_amax, int32_t n, void* workspace,
                                      size_t ws_bytes, void* stream);

/* Device workspace for lnm_infer / lnm_frame at this batch and image size. */
LNM_API size_t lnm_workspace_bytes(lnm_net net, int32_t batch, int32_t H, int32_t W);

/* Lightmaps L[B][H][W][6] = sigmoid(U-Net(G)) from guide G[B][H][W][3]
 * (Section 4.3).  logits (optional, may be NULL): the pre-sigmoid head output,
 * same layout.  H and W must be divisible by 2^(levels-1).  The workspace is
 * scratch: its contents after the call are unspecified (without logits the
 * head runs in the last conv layer's epilogue and that layer's activations
 * are never stored). */
LNM_API lnm_status lnm_infer(lnm_ctx ctx, lnm_net net, int32_t batch, int32_t H, int32_t W, const float* guide,
                     float* lightmaps, float* logits, void* workspace, size_t ws_bytes, void* stream);

/* One frame of the whole path: march -> guide, U-Net -> lightmaps, and the
 * six-way shading of Section 3: rgba[H][W][4] with
 * rgb = sum_lights rgb_l sum_{p in x,y,z} |l_p| lin(L_p^{sign l_p}), l the
 * light direction in the camera frame (right, up, toward camera), lin the
 * sRGB decode of the network output, alpha = 1 - T.  guide and lightmaps
 * receive the intermediates (device, [H][W][3] and [H][W][6]).  rgba may be
 * NULL (no shading); n_lights in [0, 16].  workspace: at least
 * lnm_frame_workspace_bytes. */
LNM_API lnm_status lnm_frame(lnm_ctx ctx, lnm_net net, const lnm_volume* vol, const lnm_camera* cam,
                     const lnm_march_params* prm, const lnm_light* lights, int32_t n_lights, float* guide,
                     float* lightmaps, float* rgba, void* workspace, size_t ws_bytes, void* stream);

/* Workspace (bytes) of lnm_frame: the larger of the march's and the U-Net's
 * (the two use the same bytes one after the other); 0 on invalid arguments. */
LNM_API size_t lnm_frame_workspace_bytes(lnm_net net, const lnm_volume* vol, const lnm_camera* cam,
                                         const lnm_march_params* prm);

/* Size of the library's static frame workspace: 128 MiB, held on every
 * device the library runs on until the process ends. */
#define LNM_STATIC_SCRATCH_BYTES 134217728u
/* lnm_frame for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same frame, bit for bit, computed in the library's static workspace
 * instead of a caller-provided one.  It allocates no device memory and
 * calls no allocating routine.  The caller still provides guide, lightmaps
 * and rgba (rgba may be NULL) as for lnm_frame.  A frame whose
 * lnm_frame_workspace_bytes exceeds LNM_STATIC_SCRATCH_BYTES (the 128^3 grid
 * at 256 x 256 takes about 123 MiB) returns LNM_ERR_SHAPE with nothing
 * enqueued.  All calls on one device share its one workspace: calls that
 * may overlap on a device (other streams, other threads, other contexts)
 * race and must be serialised by the caller.  Nothing needs clearing between
 * calls: every byte the frame reads is written earlier in the same call. */
LNM_API lnm_status lnm_frame_static(lnm_ctx ctx, lnm_net net, const lnm_volume* vol, const lnm_camera* cam,
                                    const lnm_march_params* prm, const lnm_light* lights, int32_t n_lights,
                                    float* guide, float* lightmaps, float* rgba, void* stream);

/* Six-way shading alone (the shading step of lnm_frame) for B images that share
 * one camera and light set. */
LNM_API lnm_status lnm_composite(lnm_ctx ctx, const lnm_camera* cam, const lnm_light* lights, int32_t n_lights,
                         int32_t batch, int32_t H, int32_t W, const float* lightmaps, const float* guide, float* rgba,
                         void* stream);

/* Six-way shading (Section 3, as lnm_composite) of B images of one size in
 * one launch, each with its own camera and lights, e.g. the frames of a
 * serving batch: image b is shaded with cams[b] (width W, height H) and the
 * host lights[light_start[b] .. light_start[b + 1]), exactly as lnm_composite
 * shades it alone.  lightmaps [B][H][W][6], guides [B][H][W][3], rgba
 * [B][H][W][4] (device).  batch in [1, 64], light_start[0] = 0, at most 16
 * lights per image and 64 in all. */
LNM_API lnm_status lnm_composite_batch(lnm_ctx ctx, int32_t batch, const lnm_camera* cams, const lnm_light* lights,
                                       const int32_t* light_start, int32_t H, int32_t W, const float* lightmaps,
                                       const float* guides, float* rgba, void* stream);

/* ----------------------------------------------------------- channel adapters */
/* Channel adapters (Section 4.3): four NAFBlocks on the decoder output of a
 * network (width c = its base), one per output group, each followed by a 1x1
 * head to the group's two channels and a sigmoid; they replace the plain
 * 6-channel head.  The NAFBlock (Chen et al. 2022) with both expansions 2:
 *   x = LN1(in); x = conv1x1(c -> 2c); x = depthwise conv3x3 (zero pad);
 *   x = x[:c] * x[c:]; x = x * (W_sca mean_image(x) + b_sca); x = conv1x1(c -> c);
 *   y = in + beta * x; x = LN2(y); x = conv1x1(c -> 2c); x = x[:c] * x[c:];
 *   x = conv1x1(c -> c); out = y + gamma * x.
 * LN normalises the channels of each pixel (biased variance, eps 1e-6) with
 * per-channel weight and bias; the mean is over each image of a batch.
 * Parameters per adapter, fp32, in order: ln1 w[c] b[c]; conv1 W[2c][c]
 * b[2c]; depthwise W[2c][3][3] b[2c]; sca W[c][c] b[c]; conv3 W[c][c] b[c];
 * beta[c]; ln2 w[c] b[c]; conv4 W[2c][c] b[2c]; conv5 W[c][c] b[c]; gamma[c];
 * head W[2][c] b[2]; the four adapters in group order front/back,
 * left/right, up/down, alpha/emissive.  Outputs: lightmaps channels
 * (+Z, -Z), (+X, -X), (+Y, -Y) from groups 0-2, extra[..][2] = (alpha,
 * emissive) from group 3.  Widths 16, 32, 48 and 64 are supported. */
typedef struct lnm_adapters_s* lnm_adapters;
LNM_API size_t lnm_adapters_param_count(int32_t c);
LNM_API size_t lnm_adapters_device_bytes(int32_t c);
/* Bind adapters to `net` (which must outlive them) and upload the host
 * parameters into dev_buf (caller-owned device memory, at least
 * lnm_adapters_device_bytes(net base)).  Synchronises `stream`. */
LNM_API lnm_status lnm_adapters_create(lnm_ctx ctx, lnm_net net, const float* host_params, size_t n_params,
                                       void* dev_buf, size_t dev_bytes, void* stream, lnm_adapters* out);
LNM_API void lnm_adapters_destroy(lnm_adapters ad);
/* Workspace of lnm_infer_adapters: the network's plus the adapters'
 * intermediates (about 12 c floats per pixel); 0 on invalid arguments. */
LNM_API size_t lnm_adapters_workspace_bytes(lnm_adapters ad, int32_t batch, int32_t H, int32_t W);
/* The network's trunk on guide[B][H][W][3] and the four adapters:
 * lightmaps[B][H][W][6] and, when extra is not NULL, extra[B][H][W][2]
 * (device). */
LNM_API lnm_status lnm_infer_adapters(lnm_ctx ctx, lnm_adapters ad, int32_t batch, int32_t H, int32_t W,
                                      const float* guide, float* lightmaps, float* extra, void* workspace,
                                      size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ obstacle shadows */
/* Shadow map (see lnm_shadow_frame) of a sphere obstacle (centre, radius in
 * world units) for the light direction light_dir[3] (host, need not be unit):
 * depth[size][size] (device, row v, column u) = c_z + sqrt(r^2 - (u - c_u)^2
 * - (v - c_v)^2) at texel centres inside the sphere's disc, -inf outside. */
LNM_API lnm_status lnm_shadow_map_sphere(lnm_ctx ctx, const lnm_shadow_frame* sf, const float* light_dir,
                                         const float* centre, float radius, float* depth, void* stream);

/* Six-way shading with obstacle shadows (Section 4.5): lnm_composite with
 * light k's term multiplied by the visibility of each pixel's smoke surface
 * P = o + D d (the guide's depth channel, ray of the pixel centre) in the
 * shadow map depth_maps[k] (device [size][size] in the frame sf).
 * depth_maps is a host array of n_lights device pointers; a NULL array or
 * entry leaves that light unshadowed, and pixels with D = 0 (no smoke
 * surface) or outside the map are lit.  vis (device [n_lights][batch][H][W],
 * optional) receives the visibilities (0 or 1). */
LNM_API lnm_status lnm_composite_shadowed(lnm_ctx ctx, const lnm_camera* cam, const lnm_light* lights,
                                          int32_t n_lights, const lnm_shadow_frame* sf, const float* const* depth_maps,
                                          int32_t batch, int32_t H, int32_t W, const float* lightmaps,
                                          const float* guide, float* rgba, float* vis, void* stream);

/* ------------------------------------------------------------------ training */
/* Training of the fp32 network on the GPU (Section 4.4 pixel loss, Section 5
 * optimiser).  Loss = mean over B H W 6 of (y - t)^2 where y is the network's
 * sigmoid output and t the target lightmaps in sRGB; the paper's perceptual
 * and temporal terms need pretrained networks and are not part of it.
 * Backward: sigmoid' = y(1-y), ReLU'(0) = 0, a 2x2 max-pool routes its
 * gradient to the first maximum of the window in raster order, nearest
 * upsampling sums its 2x2 block, the concatenation splits.  Every reduction
 * runs in a fixed order, so results do not depend on scheduling.
 * Optimiser: Adam with bias correction, step t = 1, 2, ...
 *
 * A trainer owns no device memory: its state (master parameters in the
 * parameter-file order, gradients, Adam moments, packed forward and
 * transposed weights) lives in a caller-provided buffer. */
typedef struct lnm_trainer_s* lnm_trainer;
LNM_API size_t lnm_trainer_state_bytes(int32_t levels, int32_t base);
LNM_API size_t lnm_train_workspace_bytes(int32_t levels, int32_t base, int32_t batch, int32_t H, int32_t W);
/* Upload host parameters (flat fp32, n_params) and zero the moments.
 * Synchronises `stream`. */
LNM_API lnm_status lnm_trainer_create(lnm_ctx ctx, int32_t levels, int32_t base, const float* host_params,
                                      size_t n_params, void* state_buf, size_t state_bytes, void* stream,
                                      lnm_trainer* out);
LNM_API void lnm_trainer_destroy(lnm_trainer tr);
/* Loss and gradient for one batch: guide[B][H][W][3], target[B][H][W][6]
 * (device).  loss (device, 1 float) and grad (device, n_params floats in the
 * parameter-file order) receive the results; either may be NULL. */
LNM_API lnm_status lnm_train_grad(lnm_ctx ctx, lnm_trainer tr, int32_t batch, int32_t H, int32_t W, const float* guide,
                                  const float* target, float* loss, float* grad, void* workspace, size_t ws_bytes,
                                  void* stream);
/* One optimisation step: gradient as above, then Adam(lr, beta1, beta2, eps)
 * on the master parameters and repacking of the network weights. */
LNM_API lnm_status lnm_train_step(lnm_ctx ctx, lnm_trainer tr, int32_t batch, int32_t H, int32_t W, const float* guide,
                                  const float* target, float lr, float beta1, float beta2, float eps, float* loss,
                                  void* workspace, size_t ws_bytes, void* stream);
/* Copy the current master parameters to host memory (synchronises `stream`). */
LNM_API lnm_status lnm_trainer_read_params(lnm_trainer tr, float* host_params, size_t n_params, void* stream);
/* Current Adam moments m, v (device-to-host) and step count, for
 * checkpointing; and the inverse, to resume bit-identically. */
LNM_API lnm_status lnm_trainer_save(lnm_trainer tr, float* host_m, float* host_v, int32_t* step, size_t n_params,
                                    void* stream);
LNM_API lnm_status lnm_trainer_load(lnm_trainer tr, const float* host_params, const float* host_m,
                                    const float* host_v, int32_t step, size_t n_params, void* stream);
/* Channel adapters (Section 4.3) trained with the network: once attached
 * (before the first step), lnm_train_grad and lnm_train_step compute the
 * loss on the adapters' lightmaps in place of the plain head's (same loss as
 * above; the alpha/emissive group has no target, so its gradient is zero,
 * and so is the unused head's), back-propagate through the four NAFBlocks
 * into the trunk, and lnm_train_step applies Adam to both parameter sets
 * with the same step count.  Backward of the blocks: layer norm dx = r (dxh
 * - mean(dxh) - xh mean(dxh xh)) with xh the normalised input and r = 1 /
 * sqrt(var + 1e-6); the channel attention's mean over each image passes its
 * gradient back divided by H W; the depthwise conv's input gradient uses
 * the mirrored taps; every sum runs in a fixed order.  The adapters' state
 * (parameters, gradient, Adam moments, each 256-byte aligned) lives in
 * state_buf (device, lnm_trainer_adapters_state_bytes, 256-byte aligned);
 * parameters: lnm_adapters_param_count(base) floats in the order of
 * lnm_adapters_create.  Checkpoints (lnm_trainer_save/load) cover the trunk
 * only.  LNM_ERR_UNSUPPORTED for a base width other than 16, 32, 48, 64;
 * LNM_ERR_ARG if adapters are attached twice or after a step. */
LNM_API size_t lnm_trainer_adapters_state_bytes(int32_t c);
LNM_API lnm_status lnm_trainer_attach_adapters(lnm_trainer tr, const float* host_params, size_t n_params,
                                               void* state_buf, size_t state_bytes, void* stream);
/* Workspace of lnm_train_grad / lnm_train_step for this trainer (with its
 * adapters, if attached); 0 for invalid sizes. */
LNM_API size_t lnm_trainer_workspace_bytes(lnm_trainer tr, int32_t batch, int32_t H, int32_t W);
/* The adapters' current parameters to host memory (synchronises), and the
 * last computed adapter gradient to device memory (n_params floats). */
LNM_API lnm_status lnm_trainer_read_adapters(lnm_trainer tr, float* host_params, size_t n_params, void* stream);
LNM_API lnm_status lnm_trainer_adapter_grad(lnm_trainer tr, float* grad, size_t n_params, void* stream);
/* Forward pass with the trainer's current weights (same as lnm_infer on an
 * fp32 net holding those weights).  LNM_ERR_UNSUPPORTED once adapters are
 * attached: their network is inferred with lnm_infer_adapters on a net and
 * adapters created from lnm_trainer_read_params / lnm_trainer_read_adapters. */
LNM_API lnm_status lnm_trainer_infer(lnm_ctx ctx, lnm_trainer tr, int32_t batch, int32_t H, int32_t W,
                                     const float* guide, float* lightmaps, void* workspace, size_t ws_bytes,
                                     void* stream);

/* ------------------------------------------------------------------ profiling */
/* Kernel kinds for per-launch timing. */
typedef enum {
  LNM_K_MARCH = 0,      /* guiding-map march */
  LNM_K_CONV = 1,       /* 3x3 convolution layers */
  LNM_K_HEAD = 2,       /* 1x1 head + sigmoid (in lnm_frame with rgba: + six-way shading, one launch) */
  LNM_K_COMPOSITE = 3,  /* six-way shading (lnm_composite, lnm_composite_shadowed) */
  LNM_K_REFERENCE = 4,  /* reference lightmaps */
  LNM_K_ADAPTERS = 5,   /* channel adapters */
  LNM_K_COUNT = 6
} lnm_kernel_kind;

/* on != 0: discard earlier records and, from now on, bracket every kernel
 * this context launches with a pair of HIP events on the launch stream (the
 * kernels themselves are unchanged; the events add a small gap between
 * launches).  on == 0 stops recording.  At most 65536 launches are kept. */
LNM_API lnm_status lnm_profile_enable(lnm_ctx ctx, int32_t on);
/* Number of recorded launches of `kind` and their summed durations in ms.
 * Blocks until the recorded events have completed. */
LNM_API lnm_status lnm_profile_read(lnm_ctx ctx, int32_t kind, int32_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* LNM_H */
