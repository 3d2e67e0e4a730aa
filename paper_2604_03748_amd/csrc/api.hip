// C ABI of liblnm: argument validation, weight packing, the layer schedule of
// the U-Net and the entry points declared in lnm.h.
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace lnm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

lnm_status fail(lnm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

ProfScope::ProfScope(lnm_ctx_s* ctx, int kind, hipStream_t s) : ctx_(ctx), s_(s) {
  if (!ctx || !ctx->prof || ctx->recs.size() >= 65536) return;
  while (ctx->pool.size() < ctx->pool_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    ctx->pool.push_back(e);
  }
  lnm_ctx_s::Rec r{kind, ctx->pool[ctx->pool_used], ctx->pool[ctx->pool_used + 1]};
  if (hipEventRecord(r.a, s) != hipSuccess) return;
  ctx->pool_used += 2;
  idx_ = (int)ctx->recs.size();
  ctx->recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (idx_ >= 0) (void)hipEventRecord(ctx_->recs[idx_].b, s_);
}

static bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

bool make_cam(const lnm_camera& c, CamDev* out, std::string* why) {
  if (c.projection != LNM_ORTHOGRAPHIC && c.projection != LNM_PERSPECTIVE) return *why = "camera.projection", false;
  if (c.width < 1 || c.height < 1) return *why = "camera width/height must be >= 1", false;
  if (!finite3(c.eye) || !finite3(c.target) || !finite3(c.up)) return *why = "camera vectors must be finite", false;
  double f[3], r[3], u[3];
  for (int a = 0; a < 3; ++a) f[a] = (double)c.target[a] - c.eye[a];
  double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(nf > 0.0)) return *why = "camera target equals eye", false;
  for (double& v : f) v /= nf;
  r[0] = f[1] * c.up[2] - f[2] * c.up[1];
  r[1] = f[2] * c.up[0] - f[0] * c.up[2];
  r[2] = f[0] * c.up[1] - f[1] * c.up[0];
  double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(nr > 1e-12)) return *why = "camera up is parallel to the view direction", false;
  for (double& v : r) v /= nr;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  if (c.projection == LNM_PERSPECTIVE && !(c.fov_y_deg > 0.0f && c.fov_y_deg < 180.0f))
    return *why = "camera.fov_y_deg must be in (0, 180)", false;
  if (c.projection == LNM_ORTHOGRAPHIC && !(c.ortho_half_extent > 0.0f && std::isfinite(c.ortho_half_extent)))
    return *why = "camera.ortho_half_extent must be > 0", false;
  for (int a = 0; a < 3; ++a) {
    out->eye[a] = c.eye[a];
    out->f[a] = (float)f[a];
    out->r[a] = (float)r[a];
    out->u[a] = (float)u[a];
  }
  out->tan_half = (float)std::tan(0.5 * (double)c.fov_y_deg * M_PI / 180.0);
  out->half_extent = c.ortho_half_extent;
  out->aspect = (float)((double)c.width / (double)c.height);
  out->proj = c.projection;
  out->W = c.width;
  out->H = c.height;
  return true;
}

static lnm_status check_volume(const lnm_volume* v) {
  if (!v) return fail(LNM_ERR_ARG, "volume is NULL");
  if (!v->density) return fail(LNM_ERR_ARG, "volume.density is NULL");
  if (v->nx < 1 || v->ny < 1 || v->nz < 1) return fail(LNM_ERR_SHAPE, "volume dimensions must be >= 1");
  if ((double)v->nx * v->ny * v->nz > 4.0e9) return fail(LNM_ERR_SHAPE, "volume larger than 2^32 voxels");
  if (bricks_bytes(v->nx, v->ny, v->nz) > 0xFFFFFFFFull)
    return fail(LNM_ERR_SHAPE, "volume too large for the march's bricked grid (4 GiB, about 1000^3 voxels)");
  if (!(v->sigma_scale >= 0.0f) || !std::isfinite(v->sigma_scale))
    return fail(LNM_ERR_ARG, "volume.sigma_scale must be finite and >= 0");
  return LNM_OK;
}

static lnm_status march_setup(const lnm_volume* vol, const lnm_camera* cam, const lnm_march_params* prm,
                              MarchDev* m, CamDev* c) {
  lnm_status st = check_volume(vol);
  if (st) return st;
  if (!cam || !prm) return fail(LNM_ERR_ARG, "camera or params is NULL");
  std::string why;
  if (!make_cam(*cam, c, &why)) return fail(LNM_ERR_ARG, why);
  if (!(prm->step_voxels > 0.0f) || !std::isfinite(prm->step_voxels))
    return fail(LNM_ERR_ARG, "params.step_voxels must be > 0");
  if (!(prm->depth_tau >= 0.0f) || !std::isfinite(prm->depth_tau)) return fail(LNM_ERR_ARG, "params.depth_tau");
  if (!(prm->ert_eps >= 0.0f && prm->ert_eps < 1.0f)) return fail(LNM_ERR_ARG, "params.ert_eps must be in [0, 1)");
  if (prm->quadrature != LNM_QUAD_ALPHA && prm->quadrature != LNM_QUAD_RIEMANN)
    return fail(LNM_ERR_ARG, "params.quadrature");
  if (!finite3(prm->light_w)) return fail(LNM_ERR_ARG, "params.light_w must be finite");
  if (prm->light_set != LNM_LIGHTS_TOP_BOTTOM && prm->light_set != LNM_LIGHTS_LEFT_RIGHT)
    return fail(LNM_ERR_ARG, "params.light_set");
  if (prm->work_order != LNM_ORDER_AUTO && prm->work_order != LNM_ORDER_BANDS && prm->work_order != LNM_ORDER_Z &&
      prm->work_order != LNM_ORDER_CELLS)
    return fail(LNM_ERR_ARG, "params.work_order");
  const int nmax = std::max(vol->nx, std::max(vol->ny, vol->nz));
  m->rho = vol->density;
  m->nx = vol->nx;
  m->ny = vol->ny;
  m->nz = vol->nz;
  m->sigma_scale = vol->sigma_scale;
  m->h = (float)((double)prm->step_voxels / nmax);
  m->depth_tau = prm->depth_tau;
  m->tau_max = prm->ert_eps > 0.0f ? (float)-std::log((double)prm->ert_eps) : INFINITY;
  m->jitter_on = prm->jitter_on != 0;
  m->seed = prm->jitter_seed;
  m->frame = prm->frame;
  m->quadrature = prm->quadrature;
  m->wf = prm->light_w[0];
  m->wt = prm->light_w[1];
  m->wb = prm->light_w[2];
  m->light_set = prm->light_set;
  m->zorder = march_order(prm->work_order, prm->light_set, vol->nx, vol->ny, vol->nz);
  if (m->zorder < 0)
    return fail(LNM_ERR_UNSUPPORTED, "params.work_order: a z cell's two grid planes do not fit in LDS");
  m->brick = vol->bricks;  // NULL: launch_march builds them in its scratch
  m->nbx = m->nby = m->nbz = 0;
  return LNM_OK;
}

// ---------------------------------------------------------------- network
int elem_bytes(int precision) { return precision == LNM_FP32 ? 4 : precision == LNM_BF16 ? 2 : 1; }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Layer table and packed-weight layout of a network at one precision.
// fp32: chunks of 16 input channels (4 for the 3-channel input);
// bf16: chunks of 32 (the 3-channel input packs its 27 taps x channels into
// one 32-wide K step).  The fp8 network keeps its last 3x3 layer, the one
// the head reads, in bf16: the layer before it stores bf16 activations for
// it, and the head reads bf16 instead of e4m3 features (e4m3's 3-bit
// mantissa on the features the head sums is the largest single term of the
// fp8 form's error).
bool net_shape(int levels, int base, int precision, std::vector<LayerDesc>* out, size_t* dev_bytes,
                      std::string* why) {
  if (levels < 2 || levels > 6) return *why = "levels must be in [2, 6]", false;
  if (base < 16 || base > 256 || base % 16) return *why = "base must be a multiple of 16 in [16, 256]", false;
  if ((base << (levels - 1)) > 4096) return *why = "deepest width exceeds 4096", false;
  if (precision != LNM_FP32 && precision != LNM_BF16 && precision != LNM_FP8_E4M3)
    return *why = "unknown precision", false;
  std::vector<LayerDesc> L;
  auto add = [&](int ci, int co, int k) {
    LayerDesc d{};
    d.ci = ci;
    d.co = co;
    d.k = k;
    d.prec = precision;
    d.out_es = elem_bytes(precision);
    if (precision == LNM_FP32) {
      d.ck = ci == 3 ? 4 : 16;
      d.ci_pad = (ci + d.ck - 1) / d.ck * d.ck;
    } else {
      d.ck = 32;
      d.ci_pad = ci == 3 ? 32 : (ci + 31) / 32 * 32;
    }
    d.co_pad = (co + kBN - 1) / kBN * kBN;
    L.push_back(d);
  };
  int cin = 3;
  for (int l = 0; l < levels - 1; ++l) {
    add(cin, base << l, 3);
    add(base << l, base << l, 3);
    cin = base << l;
  }
  add(cin, base << (levels - 1), 3);
  add(base << (levels - 1), base << (levels - 1), 3);
  for (int l = levels - 2; l >= 0; --l) {
    add((base << l) + (base << (l + 1)), base << l, 3);
    add(base << l, base << l, 3);
  }
  add(base, 6, 1);
  if (precision == LNM_FP8_E4M3) {
    const size_t last = L.size() - 2;  // the last 3x3 layer
    L[last].prec = LNM_BF16;
    L[last].out_es = 2;
    L[last - 1].out_es = 2;
  }
  L.back().out_es = 4;
  size_t off = 0;
  for (auto& d : L) {
    off = align256(off);
    d.w_off = off;
    if (d.k == 1)
      off += sizeof(float) * 6 * d.ci;  // the head stays fp32
    else if (precision != LNM_FP32 && d.ci == 3)
      off += sizeof(uint16_t) * d.co_pad * 32;  // the 3-channel input layer is bf16 in both reduced forms
    else
      off += (size_t)elem_bytes(d.prec) * d.co_pad * d.ci_pad * 9;
    off = align256(off);
    d.b_off = off;
    off += sizeof(float) * (d.k == 3 ? d.co_pad : 6);
    if (d.prec == LNM_FP8_E4M3 && d.k == 3 && d.ci != 3) {
      off = align256(off);
      d.s_off = off;
      off += sizeof(float) * d.co_pad;
    }
  }
  *out = std::move(L);
  *dev_bytes = align256(off);
  return true;
}

size_t param_count(int levels, int base) {
  std::vector<LayerDesc> L;
  size_t f;
  std::string why;
  if (!net_shape(levels, base, LNM_FP32, &L, &f, &why)) return 0;
  size_t n = 0;
  for (auto& d : L) n += (size_t)d.co * d.ci * d.k * d.k + d.co;
  return n;
}

// fp32 -> bf16 bits, round to nearest even (finite inputs).
static uint16_t host_f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// fp32 -> OCP e4m3 (bias 7, 3 mantissa bits, max 448), round to nearest
// even, saturating; subnormals are multiples of 2^-9.
static uint8_t host_f2e4m3(float f) {
  const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
  float a = std::fabs(f);
  if (!(a == a)) return 0x7f;
  if (a >= 448.0f) return sign | 0x7e;
  int e;
  std::frexp(a, &e);  // a = m 2^e, m in [0.5, 1)
  e -= 1;             // a = (1 + f) 2^e
  if (e < -6) {       // subnormal (or zero): q * 2^-9, q in [0, 8]
    const float q = std::nearbyint(std::ldexp(a, 9));
    return sign | (uint8_t)q;  // q = 8 is the smallest normal, encoded alike
  }
  float mq = std::nearbyint((std::ldexp(a, -e) - 1.0f) * 8.0f);
  if (mq == 8.0f) {
    mq = 0.0f;
    e += 1;
  }
  const int ef = e + 7;
  if (ef > 15 || (ef == 15 && mq == 7.0f)) return sign | 0x7e;
  return sign | (uint8_t)((ef << 3) | (int)mq);
}

// Packed 3x3 layout: [n_tile][chunk][tap][n (32)][c (ck)], zero padded; the
// bf16 3-channel input layer: [n_tile][n (32)][k = 3 tap + c (32)].
static void pack_layer(const LayerDesc& d, int precision, const float* w, const float* b, char* dst) {
  float* bias = reinterpret_cast<float*>(dst + d.b_off);
  if (d.k == 1) {
    std::memcpy(dst + d.w_off, w, sizeof(float) * 6 * d.ci);
    std::memcpy(bias, b, sizeof(float) * 6);
    return;
  }
  for (int n = 0; n < d.co_pad; ++n) bias[n] = n < d.co ? b[n] : 0.0f;
  const int nt = d.co_pad / kBN, nch = d.ci_pad / d.ck;
  auto W = [&](int oc, int ic, int tap) -> float {
    return (oc < d.co && ic < d.ci) ? w[((size_t)oc * d.ci + ic) * 9 + tap] : 0.0f;
  };
  if (precision == LNM_FP32) {
    float* o = reinterpret_cast<float*>(dst + d.w_off);
    for (int t = 0; t < nt; ++t)
      for (int ch = 0; ch < nch; ++ch)
        for (int tap = 0; tap < 9; ++tap)
          for (int n = 0; n < kBN; ++n)
            for (int cc = 0; cc < d.ck; ++cc) *o++ = W(t * kBN + n, ch * d.ck + cc, tap);
    return;
  }
  if (precision == LNM_FP8_E4M3 && d.ci != 3) {
    // per-output-channel scale s = max|W[o]| / 448
    float* sc = reinterpret_cast<float*>(dst + d.s_off);
    for (int n = 0; n < d.co_pad; ++n) {
      float m = 0.0f;
      if (n < d.co)
        for (int ic = 0; ic < d.ci; ++ic)
          for (int tap = 0; tap < 9; ++tap) m = std::max(m, std::fabs(W(n, ic, tap)));
      sc[n] = m > 0.0f ? m / 448.0f : 1.0f;
    }
    uint8_t* q = reinterpret_cast<uint8_t*>(dst + d.w_off);
    for (int t = 0; t < nt; ++t)
      for (int ch = 0; ch < nch; ++ch)
        for (int tap = 0; tap < 9; ++tap)
          for (int n = 0; n < kBN; ++n)
            for (int cc = 0; cc < d.ck; ++cc) {
              const int oc = t * kBN + n;
              *q++ = host_f2e4m3(W(oc, ch * d.ck + cc, tap) / sc[oc]);
            }
    return;
  }
  uint16_t* o = reinterpret_cast<uint16_t*>(dst + d.w_off);
  if (d.ci == 3) {
    for (int t = 0; t < nt; ++t)
      for (int n = 0; n < kBN; ++n)
        for (int k = 0; k < 32; ++k) *o++ = host_f2bf(k < 27 ? W(t * kBN + n, k % 3, k / 3) : 0.0f);
    return;
  }
  for (int t = 0; t < nt; ++t)
    for (int ch = 0; ch < nch; ++ch)
      for (int tap = 0; tap < 9; ++tap)
        for (int n = 0; n < kBN; ++n)
          for (int cc = 0; cc < d.ck; ++cc) *o++ = host_f2bf(W(t * kBN + n, ch * d.ck + cc, tap));
}

static int layer_splits(const lnm_net_s* net, int i, int B, int h, int w) {
  return conv_layer_tiling(net, i, B, h, w).splits;
}

static int layer_level(int L, int i) { return i < 2 * L ? i / 2 : L - 2 - (i - 2 * L) / 2; }

Plan plan_workspace(const lnm_net_s* net, int B, int H, int W) {
  Plan p;
  size_t off = 0;
  const int L = net->levels;
  int li = 0;
  auto add = [&](int lvl) {
    const LayerDesc& d = net->layers[li++];
    off = align256(off);
    p.out_off.push_back(off);
    off += (size_t)d.out_es * B * (H >> lvl) * (W >> lvl) * d.co;
  };
  for (int l = 0; l < L; ++l) {
    add(l);
    add(l);
  }
  for (int l = L - 2; l >= 0; --l) {
    add(l);
    add(l);
  }
  size_t part = 0;
  for (int i = 0; i + 1 < (int)net->layers.size(); ++i) {
    const int lvl = layer_level(L, i), h = H >> lvl, w = W >> lvl;
    const int s = layer_splits(net, i, B, h, w);
    if (s > 1) part = std::max(part, sizeof(float) * (size_t)s * B * h * w * net->layers[i].co);
  }
  p.partial_off = align256(off);
  off = p.partial_off + part;
  p.scratch_off = align256(off);
  p.bytes = p.scratch_off + kScratchBytes;
  return p;
}

lnm_status run_unet(lnm_ctx_s* ctx, const lnm_net_s* net, int B, int H, int W, const float* guide, float* lm,
                    float* logits, char* ws, hipStream_t s, const CompositeArgs* comp, bool fuse_head,
                    bool fuse_first) {
  const Plan p = plan_workspace(net, B, H, W);
  const int L = net->levels;
  auto buf = [&](int i) { return static_cast<void*>(ws + p.out_off[i]); };
  std::vector<int> skip(L);
  int li = 0;
  // src: conv layer that produced the input (-1: the guide), for fp8 scales
  auto conv = [&](int lvl, int mode, int src, const void* s0, int c0, const void* s1, int c1,
                  const HeadFuse* head = nullptr) -> hipError_t {
    const LayerDesc& d = net->layers[li];
    ConvArgs a{};
    a.src0 = s0;
    a.src1 = s1;
    a.c0 = c0;
    a.c1 = c1;
    a.B = B;
    a.H = H >> lvl;
    a.W = W >> lvl;
    a.ci_pad = d.ci_pad;
    a.co = d.co;
    a.w = net->dev + d.w_off;
    a.bias = reinterpret_cast<const float*>(net->dev + d.b_off);
    a.out = buf(li);
    a.relu = 1;
    if (d.prec == LNM_FP8_E4M3) {
      a.in_scale = src >= 0 ? net->act_scale[src] : 1.0f;
      a.w_scale = d.s_off ? reinterpret_cast<const float*>(net->dev + d.s_off) : nullptr;
      a.out_inv_scale = 1.0f / net->act_scale[li];
      a.out_bf16 = d.out_es == 2;
    }
    if (mode == G_FIRST) {
      const LayerDesc& d0 = net->layers[0];
      a.w0 = net->dev + d0.w_off;
      a.b0 = reinterpret_cast<const float*>(net->dev + d0.b_off);
      if (d0.prec == LNM_FP8_E4M3) a.w0_out_inv = 1.0f / net->act_scale[0];
    }
    a.n_tiles = d.co_pad / kBN;
    const LayerTiling tl = conv_layer_tiling(net, li, B, a.H, a.W);
    a.th = tl.th;
    a.splits = tl.splits;
    a.partial = reinterpret_cast<float*>(ws + p.partial_off);
    ++li;
    ProfScope ps(ctx, LNM_K_CONV, s);
    hipError_t err;
    int out_type = 0;
    if (d.prec == LNM_FP8_E4M3) {
      err = launch_conv3x3_fp8(mode, a, s, head);
      out_type = a.out_bf16 ? 3 : 2;
    } else if (d.prec == LNM_BF16) {
      err = launch_conv3x3_bf16(mode, a, s, head);
      out_type = 1;
    } else {
      err = launch_conv3x3_f32(mode, d.ck, a, s, head);
    }
    if (err == hipSuccess && a.splits > 1) err = launch_splitk_reduce(a, out_type, s);
    return err;
  };
  // inference: the last layer's epilogue applies the head (and the frame's
  // shading) when its one 32-channel tile is unsplit, so the layer's output
  // is never stored and the head needs no launch of its own; the head reads
  // the activations in the precision they would have been stored in, so the
  // result equals the separate head kernel's
  const int n_conv = (int)net->layers.size() - 1;
  const LayerDesc& hd = net->layers[n_conv];
  HeadFuse hf{};
  hf.w = reinterpret_cast<const float*>(net->dev + hd.w_off);
  hf.b = reinterpret_cast<const float*>(net->dev + hd.b_off);
  hf.lm = lm;
  if (comp) hf.comp = *comp;
  const bool last_e4m3 = net->layers[n_conv - 1].out_es == 1;  // features the head reads
  hf.in_scale = last_e4m3 ? net->act_scale[n_conv - 1] : 1.0f;
  const bool fused = fuse_head && lm && !logits && net->layers[n_conv - 1].co <= kBN &&
                     layer_splits(net, n_conv - 1, B, H, W) == 1;
  // the first two layers in one launch (fp32, fp8, or bf16 in the default
  // tile form): the second recomputes the first's outputs on its tiles
  // (their halo included) from the guide, so the first layer's output is
  // neither stored nor read
  const LayerDesc &d0 = net->layers[0], &d1 = net->layers[1];
  const bool first =
      fuse_first && ((d0.prec == LNM_FP32 && d1.prec == LNM_FP32 && d0.ck == 4 && d1.ck == 16) ||
                     (d0.prec == LNM_BF16 && d1.prec == LNM_BF16 &&
                      conv_layer_tiling(net, 1, B, H, W).th != kBf16Large) ||
                     (d0.prec == LNM_FP8_E4M3 && d1.prec == LNM_FP8_E4M3 && d0.out_es == 1));
  hipError_t e;
  const void* x = guide;
  int cx = 3;
  for (int l = 0; l < L; ++l) {
    const int mode = l == 0 ? G_GUIDE : G_POOL;
    if (l == 0 && first) {
      ++li;
      cx = net->layers[0].co;
      if ((e = conv(0, G_FIRST, 0, guide, cx, nullptr, 0)) != hipSuccess)
        return fail(LNM_ERR_DEVICE, hipGetErrorString(e));
      x = buf(li - 1);
      cx = net->layers[li - 1].co;
      skip[0] = li - 1;
      continue;
    }
    if ((e = conv(l, mode, l == 0 ? -1 : skip[l - 1], x, cx, nullptr, 0)) != hipSuccess)
      return fail(LNM_ERR_DEVICE, hipGetErrorString(e));
    x = buf(li - 1);
    cx = net->layers[li - 1].co;
    if ((e = conv(l, G_PLAIN, li - 1, x, cx, nullptr, 0)) != hipSuccess)
      return fail(LNM_ERR_DEVICE, hipGetErrorString(e));
    x = buf(li - 1);
    cx = net->layers[li - 1].co;
    skip[l] = li - 1;
  }
  for (int l = L - 2; l >= 0; --l) {
    const int cs = net->layers[skip[l]].co;
    if ((e = conv(l, G_CONCAT_UP, skip[l], buf(skip[l]), cs, x, cx)) != hipSuccess)
      return fail(LNM_ERR_DEVICE, hipGetErrorString(e));
    x = buf(li - 1);
    cx = net->layers[li - 1].co;
    if ((e = conv(l, G_PLAIN, li - 1, x, cx, nullptr, 0, fused && l == 0 ? &hf : nullptr)) != hipSuccess)
      return fail(LNM_ERR_DEVICE, hipGetErrorString(e));
    x = buf(li - 1);
    cx = net->layers[li - 1].co;
  }
  if (!lm || fused) return LNM_OK;  // convolutions only (calibration), or the head ran in the last layer
  HeadArgs h{};
  h.in = x;
  h.in_type = net->layers[li - 1].out_es == 4 ? 0 : net->layers[li - 1].out_es == 2 ? 1 : 2;
  h.in_scale = last_e4m3 ? net->act_scale[li - 1] : 1.0f;
  h.P = B * H * W;
  h.C = cx;
  h.w = reinterpret_cast<const float*>(net->dev + hd.w_off);
  h.b = reinterpret_cast<const float*>(net->dev + hd.b_off);
  h.lm = lm;
  h.logits = logits;
  {
    ProfScope ps(ctx, LNM_K_HEAD, s);
    e = launch_head(h, s, comp);
  }
  if (e != hipSuccess) return fail(LNM_ERR_DEVICE, hipGetErrorString(e));
  return LNM_OK;
}

lnm_status check_infer(const lnm_net_s* net, int B, int H, int W, size_t ws_bytes, const void* ws) {
  if (!net) return fail(LNM_ERR_ARG, "net is NULL");
  if (B < 1 || H < 1 || W < 1) return fail(LNM_ERR_SHAPE, "batch, H and W must be >= 1");
  const int div = 1 << (net->levels - 1);
  if (H % div || W % div) return fail(LNM_ERR_SHAPE, "H and W must be divisible by 2^(levels-1)");
  if ((double)B * H * W > 2.0e9 / 8) return fail(LNM_ERR_SHAPE, "batch x H x W too large");
  const size_t need = plan_workspace(net, B, H, W).bytes;
  if (ws_bytes < need || (need && !ws))
    return fail(LNM_ERR_SHAPE, "workspace too small: need " + std::to_string(need) + " bytes");
  return LNM_OK;
}

static lnm_status light_setup(const CamDev& c, const lnm_light* lights, int n, CompositeArgs* a) {
  if (n < 0 || n > 16) return fail(LNM_ERR_ARG, "n_lights must be in [0, 16]");
  if (n && !lights) return fail(LNM_ERR_ARG, "lights is NULL");
  a->n_lights = n;
  for (int k = 0; k < n; ++k) {
    if (!finite3(lights[k].dir) || !finite3(lights[k].rgb)) return fail(LNM_ERR_ARG, "light values must be finite");
    double d[3] = {lights[k].dir[0], lights[k].dir[1], lights[k].dir[2]};
    a->l[k][0] = (float)(d[0] * c.r[0] + d[1] * c.r[1] + d[2] * c.r[2]);
    a->l[k][1] = (float)(d[0] * c.u[0] + d[1] * c.u[1] + d[2] * c.u[2]);
    a->l[k][2] = (float)-(d[0] * c.f[0] + d[1] * c.f[1] + d[2] * c.f[2]);
    for (int q = 0; q < 3; ++q) a->rgb[k][q] = lights[k].rgb[q];
  }
  return LNM_OK;
}

lnm_status frame_impl(lnm_ctx_s* ctx, const lnm_net_s* net, const lnm_volume* vol, const lnm_camera* cam,
                      const lnm_march_params* prm, const lnm_light* lights, int n_lights, float* guide,
                      float* lightmaps, float* rgba, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (!guide || !lightmaps) return fail(LNM_ERR_ARG, "guide or lightmaps is NULL");
  MarchDev m;
  CamDev c;
  lnm_status st = march_setup(vol, cam, prm, &m, &c);
  if (st) return st;
  st = check_infer(net, 1, c.H, c.W, ws_bytes, workspace);
  if (st) return st;
  const int K = march_capacity(m);
  const size_t need = march_scratch_bytes(m, K, c.W, c.H);
  if (ws_bytes < need) return fail(LNM_ERR_SHAPE, "workspace too small for the march: need " + std::to_string(need));
  CompositeArgs a{};
  if (rgba) {
    st = light_setup(c, lights, n_lights, &a);
    if (st) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  {
    ProfScope ps(ctx, LNM_K_MARCH, s);
    LNM_HIP_CHECK(launch_march(m, c, march_buffers(workspace, m, K, c.W, c.H), guide, s));
  }
  // the head launch also shades the frame when rgba is requested
  a.lm = lightmaps;
  a.guide = guide;
  a.rgba = rgba;
  a.P = c.H * c.W;
  return run_unet(ctx, net, 1, c.H, c.W, guide, lightmaps, nullptr, static_cast<char*>(workspace), s,
                  rgba ? &a : nullptr, true, true);
}

size_t frame_workspace_bytes(const lnm_net_s* net, const lnm_volume* vol, const lnm_camera* cam,
                             const lnm_march_params* prm) {
  MarchDev m;
  CamDev c;
  if (!net || march_setup(vol, cam, prm, &m, &c)) return 0;
  const int div = 1 << (net->levels - 1);
  if (c.H % div || c.W % div) return 0;
  // the march's records are dead once the guide is written, so the U-Net
  // activations reuse the same bytes
  return std::max(march_scratch_bytes(m, march_capacity(m), c.W, c.H), plan_workspace(net, 1, c.H, c.W).bytes);
}

}  // namespace lnm

using namespace lnm;

extern "C" {

size_t lnm_abi_struct_size(int32_t which) {
  switch (which) {
    case 0: return sizeof(lnm_volume);
    case 1: return sizeof(lnm_camera);
    case 2: return sizeof(lnm_march_params);
    case 3: return sizeof(lnm_light);
    case 4: return sizeof(lnm_shadow_frame);
    default: return 0;
  }
}

const char* lnm_version(void) { return "liblnm 0.1 gfx950"; }

const char* lnm_last_error(void) { return g_err.c_str(); }

lnm_status lnm_ctx_create(int32_t hip_device, lnm_ctx* out) {
  if (!out) return fail(LNM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  LNM_HIP_CHECK(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) return fail(LNM_ERR_ARG, "no such HIP device");
  LNM_HIP_CHECK(hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  LNM_HIP_CHECK(hipGetDeviceProperties(&prop, hip_device));
  auto* c = new (std::nothrow) lnm_ctx_s;
  if (!c) return fail(LNM_ERR_OOM, "host allocation failed");
  c->device = hip_device;
  c->cu_count = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  // each device holds its own copy of the static workspace: look up this
  // device's address now, with the device current
  const hipError_t e = static_scratch_address(&c->static_scratch);
  if (e != hipSuccess || !c->static_scratch) {
    delete c;
    return fail(LNM_ERR_DEVICE, std::string("static workspace address: ") + hipGetErrorString(e));
  }
  *out = c;
  return LNM_OK;
}

void lnm_ctx_destroy(lnm_ctx ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
}

lnm_status lnm_profile_enable(lnm_ctx ctx, int32_t on) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (on) {
    ctx->recs.clear();
    ctx->pool_used = 0;
  }
  ctx->prof = on != 0;
  return LNM_OK;
}

lnm_status lnm_profile_read(lnm_ctx ctx, int32_t kind, int32_t* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms) return fail(LNM_ERR_ARG, "NULL argument");
  if (kind < 0 || kind >= LNM_K_COUNT) return fail(LNM_ERR_ARG, "unknown kernel kind");
  int n = 0;
  double ms = 0.0;
  for (const auto& r : ctx->recs) {
    if (r.kind != kind) continue;
    LNM_HIP_CHECK(hipEventSynchronize(r.b));
    float t = 0.0f;
    LNM_HIP_CHECK(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return LNM_OK;
}

size_t lnm_march_workspace_bytes(const lnm_volume* vol, const lnm_camera* cam, const lnm_march_params* prm) {
  MarchDev m;
  CamDev c;
  if (march_setup(vol, cam, prm, &m, &c)) return 0;
  return march_scratch_bytes(m, march_capacity(m), c.W, c.H);
}

lnm_status lnm_march(lnm_ctx ctx, const lnm_volume* vol, const lnm_camera* cam, const lnm_march_params* prm,
                     float* guide, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (!guide) return fail(LNM_ERR_ARG, "guide is NULL");
  MarchDev m;
  CamDev c;
  lnm_status st = march_setup(vol, cam, prm, &m, &c);
  if (st) return st;
  const int K = march_capacity(m);
  const size_t need = march_scratch_bytes(m, K, c.W, c.H);
  if (!workspace || ws_bytes < need)
    return fail(LNM_ERR_SHAPE, "march workspace too small: need " + std::to_string(need) + " bytes");
  ProfScope ps(ctx, LNM_K_MARCH, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_march(m, c, march_buffers(workspace, m, K, c.W, c.H), guide, (hipStream_t)stream));
  return LNM_OK;
}

size_t lnm_march_batch_workspace_bytes(int32_t n, const lnm_volume* vols, const lnm_camera* cams,
                                       const lnm_march_params* prms) {
  if (n < 1 || n > 4096 || !vols || !cams || !prms) return 0;
  size_t need = 0;
  for (int i = 0; i < n; ++i) {
    const size_t b = lnm_march_workspace_bytes(vols + i, cams + i, prms + i);
    if (!b) return 0;
    need = std::max(need, b);
  }
  return need;
}

lnm_status lnm_march_batch(lnm_ctx ctx, int32_t n, const lnm_volume* vols, const lnm_camera* cams,
                           const lnm_march_params* prms, float* const* guides, void* workspace, size_t ws_bytes,
                           void* stream) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (n < 1 || n > 4096) return fail(LNM_ERR_ARG, "n must be in [1, 4096]");
  if (!vols || !cams || !prms || !guides) return fail(LNM_ERR_ARG, "vols, cams, prms or guides is NULL");
  std::vector<MarchDev> ms(n);
  std::vector<CamDev> cs(n);
  size_t need = 0;
  for (int i = 0; i < n; ++i) {  // everything is checked before the first launch
    if (!guides[i]) return fail(LNM_ERR_ARG, "guides[" + std::to_string(i) + "] is NULL");
    const lnm_status st = march_setup(vols + i, cams + i, prms + i, &ms[i], &cs[i]);
    if (st) return fail(st, "march " + std::to_string(i) + ": " + g_err);
    need = std::max(need, march_scratch_bytes(ms[i], march_capacity(ms[i]), cs[i].W, cs[i].H));
  }
  if (!workspace || ws_bytes < need)
    return fail(LNM_ERR_SHAPE, "march workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps(ctx, LNM_K_MARCH, s);
  for (int i = 0; i < n; ++i) {
    const int K = march_capacity(ms[i]);
    LNM_HIP_CHECK(launch_march(ms[i], cs[i], march_buffers(workspace, ms[i], K, cs[i].W, cs[i].H), guides[i], s));
  }
  return LNM_OK;
}

size_t lnm_frame_workspace_bytes(lnm_net net, const lnm_volume* vol, const lnm_camera* cam,
                                 const lnm_march_params* prm) {
  return frame_workspace_bytes(net, vol, cam, prm);
}

lnm_status lnm_reference_lightmaps(lnm_ctx ctx, const lnm_volume* vol, const lnm_camera* cam, float step_voxels,
                                   float ert_eps, int32_t srgb, float* lm, void* stream) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (!lm) return fail(LNM_ERR_ARG, "lm is NULL");
  lnm_march_params prm{};
  prm.step_voxels = step_voxels;
  prm.depth_tau = 0.0f;
  prm.ert_eps = ert_eps;
  prm.light_w[0] = prm.light_w[1] = prm.light_w[2] = 1.0f;
  MarchDev m;
  CamDev c;
  lnm_status st = march_setup(vol, cam, &prm, &m, &c);
  if (st) return st;
  ProfScope ps(ctx, LNM_K_REFERENCE, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_reference(m, c, srgb != 0, lm, (hipStream_t)stream));
  return LNM_OK;
}

size_t lnm_net_param_count(int32_t levels, int32_t base) { return param_count(levels, base); }

size_t lnm_net_device_bytes(int32_t levels, int32_t base, int32_t precision) {
  std::vector<LayerDesc> L;
  size_t bytes;
  std::string why;
  if (!net_shape(levels, base, precision, &L, &bytes, &why)) return 0;
  return bytes;
}

lnm_status lnm_net_create(lnm_ctx ctx, int32_t levels, int32_t base, int32_t precision, const float* host_params,
                          size_t n_params, const float* act_scales, void* device_buf, size_t device_buf_bytes,
                          void* stream, lnm_net* out) {
  if (!ctx || !out || !host_params || !device_buf) return fail(LNM_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (precision != LNM_FP32 && precision != LNM_BF16 && precision != LNM_FP8_E4M3)
    return fail(LNM_ERR_UNSUPPORTED, "precision " + std::to_string(precision) + " is not built");
  const bool fp8 = precision == LNM_FP8_E4M3;
  if (!fp8 && act_scales) return fail(LNM_ERR_ARG, "act_scales must be NULL for fp32 and bf16");
  if (fp8 && !act_scales) return fail(LNM_ERR_ARG, "the fp8 form needs calibrated activation maxima");
  std::vector<LayerDesc> L;
  size_t bytes;
  std::string why;
  if (!net_shape(levels, base, precision, &L, &bytes, &why)) return fail(LNM_ERR_SHAPE, why);
  // fp8: per stored activation tensor s = kFp8Headroom amax / 448, the two
  // inputs of each decoder concatenation sharing the larger one.  The
  // headroom keeps activations of inputs beyond the calibration set's maxima
  // from saturating at 448: on the trained network, frames unlike the
  // calibration frames reach 2.6 times the calibrated maxima in the deep
  // layers, and saturation then dominates the error (max abs 0.13 per
  // channel); e4m3's range below 448 is wide enough that the headroom costs
  // no measurable precision (max abs 0.055 with headroom 4, the same at 8
  // and 16; CPU emulation of the fp8 form).
  constexpr float kFp8Headroom = 4.0f;
  std::vector<float> scale;
  if (fp8) {
    const int n_conv = (int)L.size() - 1;
    for (int i = 0; i < n_conv; ++i) {
      const float a = act_scales[i];
      if (!(a >= 0.0f) || !std::isfinite(a)) return fail(LNM_ERR_ARG, "activation maxima must be finite and >= 0");
      scale.push_back(a > 0.0f ? kFp8Headroom * a / 448.0f : 1.0f);
    }
    int li = 2 * levels;  // first decoder conv
    for (int l = levels - 2; l >= 0; --l) {
      const int skip = 2 * l + 1, low = li - 1;
      const float s = std::max(scale[skip], scale[low]);
      scale[skip] = scale[low] = s;
      li += 2;
    }
  }
  if (n_params != param_count(levels, base))
    return fail(LNM_ERR_SHAPE, "n_params is " + std::to_string(n_params) + ", expected " +
                                   std::to_string(param_count(levels, base)));
  if (device_buf_bytes < bytes) return fail(LNM_ERR_SHAPE, "device_buf too small");
  if (reinterpret_cast<uintptr_t>(device_buf) % 256) return fail(LNM_ERR_ARG, "device_buf must be 256-byte aligned");
  for (size_t i = 0; i < n_params; ++i)
    if (!std::isfinite(host_params[i])) return fail(LNM_ERR_ARG, "parameters must be finite");
  std::vector<char> packed;
  try {
    packed.assign(bytes, 0);
  } catch (...) {
    return fail(LNM_ERR_OOM, "host allocation failed");
  }
  size_t off = 0;
  for (auto& d : L) {
    const size_t nw = (size_t)d.co * d.ci * d.k * d.k;
    pack_layer(d, d.prec, host_params + off, host_params + off + nw, packed.data());
    off += nw + d.co;
  }
  auto* net = new (std::nothrow) lnm_net_s;
  if (!net) return fail(LNM_ERR_OOM, "host allocation failed");
  net->levels = levels;
  net->base = base;
  net->precision = precision;
  net->layers = std::move(L);
  net->dev = static_cast<char*>(device_buf);
  net->dev_bytes = bytes;
  net->act_scale = std::move(scale);
  hipError_t e = hipMemcpyAsync(device_buf, packed.data(), bytes, hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    delete net;
    return fail(LNM_ERR_DEVICE, std::string("weight upload: ") + hipGetErrorString(e));
  }
  *out = net;
  return LNM_OK;
}

void lnm_net_destroy(lnm_net net) { delete net; }

lnm_status lnm_calibrate_amax(lnm_ctx ctx, lnm_net net, int32_t batch, int32_t H, int32_t W, const float* guide,
                              float* host_amax, int32_t n, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx || !net || !guide || !host_amax) return fail(LNM_ERR_ARG, "NULL argument");
  if (net->precision != LNM_FP32) return fail(LNM_ERR_ARG, "calibration runs the fp32 network");
  const int n_conv = (int)net->layers.size() - 1;
  if (n != n_conv) return fail(LNM_ERR_SHAPE, "n must be the number of convolution layers");
  lnm_status st = check_infer(net, batch, H, W, ws_bytes, workspace);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = static_cast<char*>(workspace);
  const Plan p = plan_workspace(net, batch, H, W);
  float* amax = reinterpret_cast<float*>(ws + p.scratch_off);
  float* part = amax + 1024;  // kAmaxBlocks floats
  st = run_unet(ctx, net, batch, H, W, guide, nullptr, nullptr, ws, s);  // convolutions only
  if (st) return st;
  const int L = net->levels;
  for (int i = 0; i < n_conv; ++i) {
    const int lvl = i < 2 * L ? i / 2 : L - 2 - (i - 2 * L) / 2;
    const long count = (long)batch * (H >> lvl) * (W >> lvl) * net->layers[i].co;
    LNM_HIP_CHECK(launch_amax(reinterpret_cast<const float*>(ws + p.out_off[i]), count, part, amax + i, s));
  }
  LNM_HIP_CHECK(hipMemcpyAsync(host_amax, amax, sizeof(float) * n_conv, hipMemcpyDeviceToHost, s));
  LNM_HIP_CHECK(hipStreamSynchronize(s));
  return LNM_OK;
}

size_t lnm_workspace_bytes(lnm_net net, int32_t batch, int32_t H, int32_t W) {
  if (!net || batch < 1 || H < 1 || W < 1) return 0;
  return plan_workspace(net, batch, H, W).bytes;
}

lnm_status lnm_infer(lnm_ctx ctx, lnm_net net, int32_t batch, int32_t H, int32_t W, const float* guide,
                     float* lightmaps, float* logits, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return fail(LNM_ERR_ARG, "ctx is NULL");
  if (!guide || !lightmaps) return fail(LNM_ERR_ARG, "guide or lightmaps is NULL");
  lnm_status st = check_infer(net, batch, H, W, ws_bytes, workspace);
  if (st) return st;
  return run_unet(ctx, net, batch, H, W, guide, lightmaps, logits, static_cast<char*>(workspace),
                  (hipStream_t)stream, nullptr, true, true);
}

lnm_status lnm_composite(lnm_ctx ctx, const lnm_camera* cam, const lnm_light* lights, int32_t n_lights,
                         int32_t batch, int32_t H, int32_t W, const float* lightmaps, const float* guide, float* rgba,
                         void* stream) {
  if (!ctx || !cam || !lightmaps || !guide || !rgba) return fail(LNM_ERR_ARG, "NULL argument");
  if (batch < 1 || H < 1 || W < 1) return fail(LNM_ERR_SHAPE, "batch, H and W must be >= 1");
  CamDev c;
  std::string why;
  if (!make_cam(*cam, &c, &why)) return fail(LNM_ERR_ARG, why);
  CompositeArgs a{};
  lnm_status st = light_setup(c, lights, n_lights, &a);
  if (st) return st;
  a.lm = lightmaps;
  a.guide = guide;
  a.rgba = rgba;
  a.P = batch * H * W;
  ProfScope ps(ctx, LNM_K_COMPOSITE, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_composite(a, (hipStream_t)stream));
  return LNM_OK;
}

lnm_status lnm_composite_batch(lnm_ctx ctx, int32_t batch, const lnm_camera* cams, const lnm_light* lights,
                               const int32_t* light_start, int32_t H, int32_t W, const float* lightmaps,
                               const float* guides, float* rgba, void* stream) {
  if (!ctx || !cams || !light_start || !lightmaps || !guides || !rgba) return fail(LNM_ERR_ARG, "NULL argument");
  if (batch < 1 || batch > kBatchShadeImages) return fail(LNM_ERR_ARG, "batch must be in [1, 64]");
  if (H < 1 || W < 1 || (double)batch * H * W > 2.0e9) return fail(LNM_ERR_SHAPE, "H and W must be >= 1");
  if (light_start[0] != 0) return fail(LNM_ERR_ARG, "light_start[0] must be 0");
  const int n_lights = light_start[batch];
  if (n_lights < 0 || n_lights > kBatchShadeLights) return fail(LNM_ERR_ARG, "at most 64 lights in all");
  if (n_lights && !lights) return fail(LNM_ERR_ARG, "lights is NULL");
  CompositeBatchArgs a{};
  for (int b = 0; b < batch; ++b) {
    if (light_start[b + 1] < light_start[b]) return fail(LNM_ERR_ARG, "light_start must not decrease");
    if (cams[b].width != W || cams[b].height != H)
      return fail(LNM_ERR_SHAPE, "camera " + std::to_string(b) + " is not W x H");
    CamDev c;
    std::string why;
    if (!make_cam(cams[b], &c, &why)) return fail(LNM_ERR_ARG, "camera " + std::to_string(b) + ": " + why);
    CompositeArgs one{};
    const int k0 = light_start[b], nk = light_start[b + 1] - k0;
    if (nk > 16) return fail(LNM_ERR_ARG, "at most 16 lights per image");
    lnm_status st = light_setup(c, lights + k0, nk, &one);
    if (st) return st;
    for (int k = 0; k < nk; ++k)
      for (int q = 0; q < 3; ++q) {
        a.l[k0 + k][q] = one.l[k][q];
        a.rgb[k0 + k][q] = one.rgb[k][q];
      }
    a.light_lo[b] = k0;
  }
  a.light_lo[batch] = n_lights;
  a.lm = lightmaps;
  a.guide = guides;
  a.rgba = rgba;
  a.P = H * W;
  a.B = batch;
  ProfScope ps(ctx, LNM_K_COMPOSITE, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_composite_batch(a, (hipStream_t)stream));
  return LNM_OK;
}

// ---------------------------------------------------------------- channel adapters
static size_t adapters_params(int c) { return c >= 1 ? 4 * (7 * (size_t)c * c + 35 * (size_t)c + 2) : 0; }

struct AdapterPlan {
  size_t net_bytes, v_off, part_off, sca_off, bytes;
  int n_blk;
};
static AdapterPlan adapter_plan(const lnm_adapters_s* ad, int B, int H, int W) {
  AdapterPlan p;
  const size_t P = (size_t)B * H * W, c = ad->c;
  p.n_blk = adapter_tiles(H, W);
  p.net_bytes = plan_workspace(ad->net, B, H, W).bytes;
  p.v_off = align256(p.net_bytes);
  p.part_off = align256(p.v_off + sizeof(float) * 4 * c * P);
  p.sca_off = align256(p.part_off + sizeof(float) * (size_t)B * 4 * c * p.n_blk);
  p.bytes = p.sca_off + sizeof(float) * (size_t)B * 4 * c;
  return p;
}

size_t lnm_adapters_param_count(int32_t c) { return adapter_width_supported(c) ? adapters_params(c) : 0; }

size_t lnm_adapters_device_bytes(int32_t c) {
  return adapter_width_supported(c) ? align256(sizeof(float) * adapters_params(c)) : 0;
}

lnm_status lnm_adapters_create(lnm_ctx ctx, lnm_net net, const float* host_params, size_t n_params, void* dev_buf,
                               size_t dev_bytes, void* stream, lnm_adapters* out) {
  if (!ctx || !net || !host_params || !dev_buf || !out) return fail(LNM_ERR_ARG, "NULL argument");
  *out = nullptr;
  const int c = net->base;
  if (!adapter_width_supported(c)) return fail(LNM_ERR_UNSUPPORTED, "adapters need a base width of 16, 32, 48 or 64");
  if (n_params != adapters_params(c))
    return fail(LNM_ERR_SHAPE, "adapter parameters: expected " + std::to_string(adapters_params(c)));
  if (dev_bytes < lnm_adapters_device_bytes(c)) return fail(LNM_ERR_SHAPE, "adapter device buffer too small");
  for (size_t i = 0; i < n_params; ++i)
    if (!std::isfinite(host_params[i])) return fail(LNM_ERR_ARG, "adapter parameters must be finite");
  hipStream_t s = (hipStream_t)stream;
  LNM_HIP_CHECK(hipMemcpyAsync(dev_buf, host_params, sizeof(float) * n_params, hipMemcpyHostToDevice, s));
  LNM_HIP_CHECK(hipStreamSynchronize(s));
  lnm_adapters_s* ad = new (std::nothrow) lnm_adapters_s;
  if (!ad) return fail(LNM_ERR_OOM, "out of host memory");
  ad->net = net;
  ad->c = c;
  ad->dev = static_cast<float*>(dev_buf);
  *out = ad;
  return LNM_OK;
}

void lnm_adapters_destroy(lnm_adapters ad) { delete ad; }

size_t lnm_adapters_workspace_bytes(lnm_adapters ad, int32_t batch, int32_t H, int32_t W) {
  if (!ad || check_infer(ad->net, batch, H, W, SIZE_MAX, reinterpret_cast<void*>(1))) return 0;
  return adapter_plan(ad, batch, H, W).bytes;
}

lnm_status lnm_infer_adapters(lnm_ctx ctx, lnm_adapters ad, int32_t batch, int32_t H, int32_t W, const float* guide,
                              float* lightmaps, float* extra, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx || !ad) return fail(LNM_ERR_ARG, "ctx or adapters is NULL");
  if (!guide || !lightmaps) return fail(LNM_ERR_ARG, "guide or lightmaps is NULL");
  lnm_status st = check_infer(ad->net, batch, H, W, ws_bytes, workspace);
  if (st) return st;
  const AdapterPlan ap = adapter_plan(ad, batch, H, W);
  if (ws_bytes < ap.bytes) return fail(LNM_ERR_SHAPE, "workspace too small: need " + std::to_string(ap.bytes));
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = (hipStream_t)stream;
  st = run_unet(ctx, ad->net, batch, H, W, guide, nullptr, nullptr, ws, s, nullptr, false, true);  // trunk only
  if (st) return st;
  const lnm_net_s* net = ad->net;
  const int n_conv = (int)net->layers.size() - 1;
  AdapterArgs a{};
  a.feat = ws + plan_workspace(net, batch, H, W).out_off[n_conv - 1];
  const int feat_es = net->layers[n_conv - 1].out_es;  // the decoder features as stored
  a.feat_scale = feat_es == 1 ? net->act_scale[n_conv - 1] : 1.0f;
  a.prm = ad->dev;
  a.B = batch;
  a.H = H;
  a.W = W;
  a.P = (size_t)batch * H * W;
  a.v = reinterpret_cast<float*>(ws + ap.v_off);
  a.part = reinterpret_cast<float*>(ws + ap.part_off);
  a.n_blk = ap.n_blk;
  a.sca = reinterpret_cast<float*>(ws + ap.sca_off);
  a.lm = lightmaps;
  a.extra = extra;
  const int in_type = feat_es == 4 ? 0 : feat_es == 2 ? 1 : 2;
  ProfScope ps(ctx, LNM_K_ADAPTERS, s);
  LNM_HIP_CHECK(launch_adapters(ad->c, a, in_type, s));
  return LNM_OK;
}

size_t lnm_bricks_bytes(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1 || (double)nx * ny * nz > 4.0e9) return 0;
  return bricks_bytes(nx, ny, nz);
}

lnm_status lnm_make_bricks(lnm_ctx ctx, const lnm_volume* vol, float* bricks, size_t bytes, void* stream) {
  if (!ctx || !bricks) return fail(LNM_ERR_ARG, "NULL argument");
  lnm_status st = check_volume(vol);
  if (st) return st;
  if (bytes < bricks_bytes(vol->nx, vol->ny, vol->nz))
    return fail(LNM_ERR_SHAPE, "bricks buffer too small: need " + std::to_string(bricks_bytes(vol->nx, vol->ny, vol->nz)));
  MarchDev m{};
  m.rho = vol->density;
  m.nx = vol->nx;
  m.ny = vol->ny;
  m.nz = vol->nz;
  ProfScope ps(ctx, LNM_K_MARCH, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_relayout(m, bricks, (hipStream_t)stream));
  return LNM_OK;
}

// Light space of the shadow maps, in fp64 then rounded once.
static void light_frame(const float* dir, float e1[3], float e2[3], float lw[3]) {
  double l[3] = {dir[0], dir[1], dir[2]};
  const double n = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
  for (double& x : l) x /= n;
  const double a[3] = {std::fabs(l[1]) > 0.99 ? 1.0 : 0.0, std::fabs(l[1]) > 0.99 ? 0.0 : 1.0, 0.0};
  double u[3] = {a[1] * l[2] - a[2] * l[1], a[2] * l[0] - a[0] * l[2], a[0] * l[1] - a[1] * l[0]};
  const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (double& x : u) x /= un;
  const double v[3] = {l[1] * u[2] - l[2] * u[1], l[2] * u[0] - l[0] * u[2], l[0] * u[1] - l[1] * u[0]};
  for (int q = 0; q < 3; ++q) {
    e1[q] = (float)u[q];
    e2[q] = (float)v[q];
    lw[q] = (float)l[q];
  }
}

static lnm_status check_shadow_frame(const lnm_shadow_frame* sf) {
  if (!sf) return fail(LNM_ERR_ARG, "shadow frame is NULL");
  if (!finite3(sf->origin)) return fail(LNM_ERR_ARG, "shadow frame origin must be finite");
  if (!(sf->half_extent > 0.0f) || !std::isfinite(sf->half_extent))
    return fail(LNM_ERR_ARG, "shadow frame half_extent must be > 0");
  if (sf->size < 1 || sf->size > 16384) return fail(LNM_ERR_SHAPE, "shadow frame size must be in [1, 16384]");
  if (!std::isfinite(sf->bias)) return fail(LNM_ERR_ARG, "shadow frame bias must be finite");
  return LNM_OK;
}

static bool nonzero3(const float* v) { return v[0] != 0.0f || v[1] != 0.0f || v[2] != 0.0f; }

lnm_status lnm_shadow_map_sphere(lnm_ctx ctx, const lnm_shadow_frame* sf, const float* light_dir, const float* centre,
                                 float radius, float* depth, void* stream) {
  if (!ctx || !light_dir || !centre || !depth) return fail(LNM_ERR_ARG, "NULL argument");
  lnm_status st = check_shadow_frame(sf);
  if (st) return st;
  if (!finite3(light_dir) || !nonzero3(light_dir)) return fail(LNM_ERR_ARG, "light_dir must be finite and nonzero");
  if (!finite3(centre) || !(radius >= 0.0f) || !std::isfinite(radius))
    return fail(LNM_ERR_ARG, "centre must be finite and radius >= 0");
  float e1[3], e2[3], lw[3];
  light_frame(light_dir, e1, e2, lw);
  double c[3];
  for (int q = 0; q < 3; ++q) c[q] = (double)centre[q] - sf->origin[q];
  auto dotd = [&](const float* e) { return c[0] * e[0] + c[1] * e[1] + c[2] * e[2]; };
  ProfScope ps(ctx, LNM_K_COMPOSITE, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_shadow_map_sphere(sf->size, sf->half_extent, (float)dotd(e1), (float)dotd(e2), (float)dotd(lw),
                                         radius * radius, depth, (hipStream_t)stream));
  return LNM_OK;
}

lnm_status lnm_composite_shadowed(lnm_ctx ctx, const lnm_camera* cam, const lnm_light* lights, int32_t n_lights,
                                  const lnm_shadow_frame* sf, const float* const* depth_maps, int32_t batch, int32_t H,
                                  int32_t W, const float* lightmaps, const float* guide, float* rgba, float* vis,
                                  void* stream) {
  if (!ctx || !cam || !lightmaps || !guide || !rgba) return fail(LNM_ERR_ARG, "NULL argument");
  if (batch < 1 || H < 1 || W < 1) return fail(LNM_ERR_SHAPE, "batch, H and W must be >= 1");
  if ((long)batch * H * W > INT32_MAX / 4) return fail(LNM_ERR_SHAPE, "too many pixels");
  lnm_status st = check_shadow_frame(sf);
  if (st) return st;
  ShadowArgs a{};
  std::string why;
  if (!make_cam(*cam, &a.cam, &why)) return fail(LNM_ERR_ARG, why);
  if (a.cam.W != W || a.cam.H != H) return fail(LNM_ERR_SHAPE, "H and W must match the camera's size");
  st = light_setup(a.cam, lights, n_lights, &a.c);
  if (st) return st;
  for (int k = 0; k < n_lights; ++k) {
    a.depth[k] = depth_maps ? depth_maps[k] : nullptr;
    if (a.depth[k] && !nonzero3(lights[k].dir)) return fail(LNM_ERR_ARG, "a shadowed light needs a nonzero direction");
    if (a.depth[k]) light_frame(lights[k].dir, a.e1[k], a.e2[k], a.lw[k]);
  }
  for (int q = 0; q < 3; ++q) a.origin[q] = sf->origin[q];
  a.E = sf->half_extent;
  a.S = sf->size;
  a.bias = sf->bias;
  a.c.lm = lightmaps;
  a.c.guide = guide;
  a.c.rgba = rgba;
  a.c.P = batch * H * W;
  a.vis = vis;
  ProfScope ps(ctx, LNM_K_COMPOSITE, (hipStream_t)stream);
  LNM_HIP_CHECK(launch_composite_shadowed(a, (hipStream_t)stream));
  return LNM_OK;
}

lnm_status lnm_frame(lnm_ctx ctx, lnm_net net, const lnm_volume* vol, const lnm_camera* cam,
                     const lnm_march_params* prm, const lnm_light* lights, int32_t n_lights, float* guide,
                     float* lightmaps, float* rgba, void* workspace, size_t ws_bytes, void* stream) {
  return frame_impl(ctx, net, vol, cam, prm, lights, n_lights, guide, lightmaps, rgba, workspace, ws_bytes, stream);
}

}  // extern "C"
