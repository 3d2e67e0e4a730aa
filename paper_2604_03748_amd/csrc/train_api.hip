// Training entry points: forward with saved activations, backward through the
// U-Net in reverse layer order, Adam, and repacking of the weights.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace lnm {
namespace {

struct ConvStep {
  int level, mode;
  int src0, src1;  // producing conv layer of each input (-1: the guide / none)
};

// The forward schedule of run_unet, as a table.
std::vector<ConvStep> schedule(int L) {
  std::vector<ConvStep> s;
  std::vector<int> skip(L);
  int i = 0;
  for (int l = 0; l < L; ++l) {
    s.push_back({l, l == 0 ? G_GUIDE : G_POOL, l == 0 ? -1 : skip[l - 1], -1});
    ++i;
    s.push_back({l, G_PLAIN, i - 1, -1});
    ++i;
    skip[l] = i - 1;
  }
  for (int l = L - 2; l >= 0; --l) {
    s.push_back({l, G_CONCAT_UP, skip[l], i - 1});
    ++i;
    s.push_back({l, G_PLAIN, i - 1, -1});
    ++i;
  }
  return s;
}

struct StateLayout {
  size_t p, g, m, v, net, zeros, bytes;
  std::vector<size_t> dgrad_w;
  std::vector<LayerDesc> fwd, dg;
  size_t net_bytes;
  size_t n_params;
  int max_dg_co_pad;
};

bool state_layout(int levels, int base, StateLayout* s, std::string* why) {
  if (!net_shape(levels, base, LNM_FP32, &s->fwd, &s->net_bytes, why)) return false;
  s->n_params = param_count(levels, base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t nb = sizeof(float) * s->n_params;
  s->p = take(nb);
  s->g = take(nb);
  s->m = take(nb);
  s->v = take(nb);
  s->net = take(s->net_bytes);
  s->dg.assign(s->fwd.size(), LayerDesc{});
  s->dgrad_w.assign(s->fwd.size(), 0);
  s->max_dg_co_pad = 32;
  for (size_t i = 1; i + 1 < s->fwd.size(); ++i) {
    const LayerDesc& f = s->fwd[i];
    LayerDesc d{};
    d.ci = f.co;
    d.co = f.ci;
    d.k = 3;
    d.ck = 16;
    d.ci_pad = (f.co + 15) / 16 * 16;
    d.co_pad = (f.ci + kBN - 1) / kBN * kBN;
    d.prec = LNM_FP32;
    d.out_es = 4;
    s->dg[i] = d;
    s->dgrad_w[i] = take(sizeof(float) * d.co_pad * d.ci_pad * 9);
    s->max_dg_co_pad = std::max(s->max_dg_co_pad, d.co_pad);
  }
  s->zeros = take(sizeof(float) * s->max_dg_co_pad);
  s->bytes = align256(off);
  return true;
}

// workspace of the adapters' training (offsets; per-pixel tensors of the
// three groups with a lightmap target, forward tensors of all four)
struct AdapterTrainPlan {
  size_t v, dsave, part, sca, msave, dgt, dyf, dxf, d5, x5, d3, x3, x4, x1, d4, d1, tpart, fpart, dmh, lossg, wpart;
  int n_blk, tpi;
};

struct TrainPlan {
  Plan fwd;
  size_t g_base, lm, dz, dx, part, colpart, losspart, loss, bytes;
  std::vector<int> tiles_per_group;
  AdapterTrainPlan ad;
};

constexpr size_t kPartialBudget = 48u << 20;  // bytes of weight-gradient partial sums per layer

TrainPlan train_plan(const lnm_net_s* net, int B, int H, int W, int ad_c = 0) {
  TrainPlan t;
  t.fwd = plan_workspace(net, B, H, W);
  const auto sch = schedule(net->levels);
  size_t off = t.fwd.bytes;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += bytes;
    return o;
  };
  t.g_base = take(t.fwd.bytes);
  const size_t P = (size_t)B * H * W;
  t.lm = take(sizeof(float) * P * 6);
  t.dz = take(sizeof(float) * P * 6);
  size_t dx = 0, part = 0;
  int maxc = 6;
  for (size_t i = 0; i < sch.size(); ++i) {
    const LayerDesc& d = net->layers[i];
    const int h = H >> sch[i].level, w = W >> sch[i].level;
    if (sch[i].mode == G_POOL || sch[i].mode == G_CONCAT_UP) dx = std::max(dx, (size_t)B * h * w * d.ci);
    const int tiles = B * ((w + 15) / 16) * ((h + 7) / 8);
    const int co_pad = (d.co + kBN - 1) / kBN * kBN, ci16 = (d.ci + 15) / 16 * 16;
    const size_t per_group = sizeof(float) * 4 * (size_t)co_pad * ci16 * 9;
    int groups = (int)std::max<size_t>(1, std::min<size_t>({(size_t)tiles, kPartialBudget / per_group, 512}));
    const int tpg = (tiles + groups - 1) / groups;
    groups = (tiles + tpg - 1) / tpg;
    t.tiles_per_group.push_back(tpg);
    part = std::max(part, per_group * groups);
    maxc = std::max(maxc, d.co);
  }
  t.dx = take(sizeof(float) * std::max<size_t>(dx, 1));
  t.part = take(part);
  t.colpart = take(sizeof(float) * kColsumBlocks * maxc);
  t.losspart = take(sizeof(float) * kLossBlocks);
  t.loss = take(sizeof(float));
  t.ad = AdapterTrainPlan{};
  if (ad_c > 0) {
    AdapterTrainPlan& a = t.ad;
    const size_t c = ad_c, f = sizeof(float);
    a.n_blk = adapter_tiles(H, W);
    a.tpi = adapter_tail_blocks_per_image(H, W);
    a.v = take(f * 4 * P * c);
    a.dsave = take(f * 4 * P * 2 * c);
    a.part = take(f * (size_t)B * 4 * c * a.n_blk);
    a.sca = take(f * (size_t)B * 4 * c);
    a.msave = take(f * (size_t)B * 4 * c);
    for (size_t* o : {&a.dgt, &a.dyf, &a.dxf, &a.d5, &a.x5, &a.d3, &a.x3, &a.x4, &a.x1}) *o = take(f * 3 * P * c);
    a.d4 = take(f * 3 * P * 2 * c);
    a.d1 = take(f * 3 * P * 2 * c);
    a.tpart = take(f * 3 * (size_t)B * a.tpi * (11 * c + 4));
    a.fpart = take(f * 3 * (size_t)B * a.n_blk * 24 * c);
    a.dmh = take(f * (size_t)B * 4 * c);
    a.lossg = take(f * 4);
    a.wpart = take(adapter_wgrad_partial_bytes(P, ad_c));
  }
  t.bytes = align256(off);
  return t;
}

lnm_status repack(lnm_trainer_s* tr, hipStream_t s) {
  const auto& L = tr->net.layers;
  for (size_t i = 0; i < L.size(); ++i) {
    const float* w = tr->p + tr->flat_w[i];
    const float* b = tr->p + tr->flat_b[i];
    if (L[i].k == 1) {
      LNM_HIP_CHECK(hipMemcpyAsync(tr->net.dev + L[i].w_off, w, sizeof(float) * 6 * L[i].ci,
                                   hipMemcpyDeviceToDevice, s));
      LNM_HIP_CHECK(hipMemcpyAsync(tr->net.dev + L[i].b_off, b, sizeof(float) * 6, hipMemcpyDeviceToDevice, s));
      continue;
    }
    LNM_HIP_CHECK(launch_pack_f32(w, b, L[i], 0, tr->net.dev, L[i].w_off, L[i].b_off, s));
    if (i > 0) LNM_HIP_CHECK(launch_pack_f32(w, b, tr->dgrad[i], 1, tr->state, tr->dgrad_off[i], 0, s));
  }
  return LNM_OK;
}

lnm_status check_train(lnm_ctx ctx, lnm_trainer tr, int B, int H, int W, const float* guide, const float* target,
                       const void* ws, size_t ws_bytes) {
  if (!ctx || !tr || !guide || !target) return fail(LNM_ERR_ARG, "NULL argument");
  if (B < 1 || H < 1 || W < 1) return fail(LNM_ERR_SHAPE, "batch, H and W must be >= 1");
  const int div = 1 << (tr->net.levels - 1);
  if (H % div || W % div) return fail(LNM_ERR_SHAPE, "H and W must be divisible by 2^(levels-1)");
  if ((double)B * H * W > 2.0e9 / 64) return fail(LNM_ERR_SHAPE, "batch x H x W too large");
  const size_t need = train_plan(&tr->net, B, H, W, tr->ad_c).bytes;
  if (!ws || ws_bytes < need) return fail(LNM_ERR_SHAPE, "workspace too small: need " + std::to_string(need));
  return LNM_OK;
}

lnm_status grad_impl(lnm_ctx ctx, lnm_trainer tr, int B, int H, int W, const float* guide, const float* target,
                     char* ws, hipStream_t s) {
  const lnm_net_s* net = &tr->net;
  const TrainPlan tp = train_plan(net, B, H, W, tr->ad_c);
  const auto sch = schedule(net->levels);
  const size_t P = (size_t)B * H * W;
  float* lm = reinterpret_cast<float*>(ws + tp.lm);
  float* dz = reinterpret_cast<float*>(ws + tp.dz);
  auto Y = [&](int i) { return reinterpret_cast<float*>(ws + tp.fwd.out_off[i]); };
  auto G = [&](int i) { return reinterpret_cast<float*>(ws + tp.g_base + tp.fwd.out_off[i]); };
  float* dx = reinterpret_cast<float*>(ws + tp.dx);
  float* part = reinterpret_cast<float*>(ws + tp.part);
  float* colpart = reinterpret_cast<float*>(ws + tp.colpart);

  const int nl = (int)net->layers.size(), hi = nl - 1, last = nl - 2;
  const LayerDesc& hd = net->layers[hi];
  if (tr->ad_c) {
    // the adapters in place of the head: trunk forward, the adapters' forward
    // and backward (their gradient into ad_g), the features' gradient into
    // G(last); the unused head takes a zero gradient
    lnm_status st = run_unet(ctx, net, B, H, W, guide, nullptr, nullptr, ws, s);
    if (st) return st;
    const AdapterTrainPlan& ap = tp.ad;
    auto F = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    AdapterTrainArgs t{};
    AdapterArgs& a = t.f;
    a.feat = Y(last);
    a.feat_scale = 1.0f;
    a.prm = tr->ad_p;
    a.B = B;
    a.H = H;
    a.W = W;
    a.P = P;
    a.v = F(ap.v);
    a.part = F(ap.part);
    a.n_blk = ap.n_blk;
    a.sca = F(ap.sca);
    a.dsave = F(ap.dsave);
    a.msave = F(ap.msave);
    t.target = target;
    t.grad = tr->ad_g;
    t.dgt = F(ap.dgt);
    t.dyf = F(ap.dyf);
    t.dxf = F(ap.dxf);
    t.d5 = F(ap.d5);
    t.x5 = F(ap.x5);
    t.d3 = F(ap.d3);
    t.x3 = F(ap.x3);
    t.x4 = F(ap.x4);
    t.x1 = F(ap.x1);
    t.d4 = F(ap.d4);
    t.d1 = F(ap.d1);
    t.tpart = F(ap.tpart);
    t.fpart = F(ap.fpart);
    t.dmh = F(ap.dmh);
    t.lossg = F(ap.lossg);
    t.loss = F(tp.loss);
    t.tpi = ap.tpi;
    t.inv_n = (float)(1.0 / ((double)P * 6.0));
    {
      ProfScope ps(ctx, LNM_K_ADAPTERS, s);
      LNM_HIP_CHECK(launch_adapters_train(tr->ad_c, t, Y(last), G(last), F(ap.wpart), s));
    }
    LNM_HIP_CHECK(launch_fill_zero(tr->g + tr->flat_w[hi], (long)(6 * hd.ci + 6), s));
  } else {
    lnm_status st = run_unet(ctx, net, B, H, W, guide, lm, nullptr, ws, s);
    if (st) return st;
    LNM_HIP_CHECK(launch_loss(lm, target, dz, reinterpret_cast<float*>(ws + tp.losspart), (long)P * 6,
                              reinterpret_cast<float*>(ws + tp.loss), s));
    LNM_HIP_CHECK(launch_head_bwd(dz, reinterpret_cast<const float*>(net->dev + hd.w_off), Y(last), (long)P,
                                  hd.ci, G(last), tr->g + tr->flat_w[hi], tr->g + tr->flat_b[hi], nullptr, s));
  }
  for (int i = last; i >= 0; --i) {
    const LayerDesc& d = net->layers[i];
    const ConvStep& c = sch[i];
    const int h = H >> c.level, w = W >> c.level;
    const long n_out = (long)B * h * w * d.co;
    if (i != last) LNM_HIP_CHECK(launch_relu_mask(G(i), Y(i), n_out, s));  // dL/d(pre-activation)
    LNM_HIP_CHECK(launch_colsum(G(i), (long)B * h * w, d.co, colpart, tr->g + tr->flat_b[i], s));
    // the layer's input exactly as the forward gather read it
    ConvArgs x{};
    x.src0 = c.src0 < 0 ? static_cast<const void*>(guide) : Y(c.src0);
    x.src1 = c.src1 < 0 ? nullptr : Y(c.src1);
    x.c0 = c.src0 < 0 ? 3 : net->layers[c.src0].co;
    x.c1 = c.src1 < 0 ? 0 : net->layers[c.src1].co;
    x.B = B;
    x.H = h;
    x.W = w;
    WgradArgs wa{};
    wa.x = x;
    wa.e = G(i);
    wa.co = d.co;
    wa.ci = d.ci;
    wa.ci_pad16 = (d.ci + 15) / 16 * 16;
    wa.tiles_per_group = tp.tiles_per_group[i];
    wa.partial = part;
    int n_part = 0;
    {
      ProfScope ps(ctx, LNM_K_CONV, s);
      LNM_HIP_CHECK(launch_wgrad3x3(c.mode, wa, &n_part, s));
    }
    LNM_HIP_CHECK(launch_wgrad_reduce(part, n_part, d.co, d.ci, (d.co + kBN - 1) / kBN * kBN, wa.ci_pad16,
                                      tr->g + tr->flat_w[i], s));
    if (i == 0) break;
    // gradient with respect to the layer's input: the convolution with the
    // transposed, tap-mirrored weights
    const LayerDesc& dg = tr->dgrad[i];
    ConvArgs a{};
    a.src0 = G(i);
    a.c0 = d.co;
    a.B = B;
    a.H = h;
    a.W = w;
    a.ci_pad = dg.ci_pad;
    a.co = dg.co;
    a.w = tr->state + tr->dgrad_off[i];
    a.bias = tr->zeros;
    a.out = c.mode == G_PLAIN ? static_cast<void*>(G(c.src0)) : static_cast<void*>(dx);
    a.relu = 0;
    a.n_tiles = dg.co_pad / kBN;
    a.splits = 1;
    {
      ProfScope ps(ctx, LNM_K_CONV, s);
      LNM_HIP_CHECK(launch_conv3x3_f32(G_PLAIN, 16, a, s));
    }
    if (c.mode == G_POOL) {
      LNM_HIP_CHECK(launch_route_pool(dx, Y(c.src0), B, h, w, d.ci, G(c.src0), s));
    } else if (c.mode == G_CONCAT_UP) {
      LNM_HIP_CHECK(launch_route_concat(dx, B, h, w, net->layers[c.src0].co, net->layers[c.src1].co, G(c.src0),
                                        G(c.src1), s));
    }
  }
  return LNM_OK;
}

}  // namespace
}  // namespace lnm

using namespace lnm;

extern "C" {

size_t lnm_trainer_state_bytes(int32_t levels, int32_t base) {
  StateLayout s;
  std::string why;
  return state_layout(levels, base, &s, &why) ? s.bytes : 0;
}

size_t lnm_train_workspace_bytes(int32_t levels, int32_t base, int32_t batch, int32_t H, int32_t W) {
  if (batch < 1 || H < 1 || W < 1) return 0;
  lnm_net_s net;
  size_t bytes;
  std::string why;
  if (!net_shape(levels, base, LNM_FP32, &net.layers, &bytes, &why)) return 0;
  net.levels = levels;
  net.base = base;
  net.precision = LNM_FP32;
  return train_plan(&net, batch, H, W).bytes;
}

lnm_status lnm_trainer_create(lnm_ctx ctx, int32_t levels, int32_t base, const float* host_params, size_t n_params,
                              void* state_buf, size_t state_bytes, void* stream, lnm_trainer* out) {
  if (!ctx || !host_params || !state_buf || !out) return fail(LNM_ERR_ARG, "NULL argument");
  *out = nullptr;
  StateLayout sl;
  std::string why;
  if (!state_layout(levels, base, &sl, &why)) return fail(LNM_ERR_SHAPE, why);
  if (n_params != sl.n_params) return fail(LNM_ERR_SHAPE, "n_params does not match the network");
  if (state_bytes < sl.bytes) return fail(LNM_ERR_SHAPE, "state buffer too small: need " + std::to_string(sl.bytes));
  if (reinterpret_cast<uintptr_t>(state_buf) % 256) return fail(LNM_ERR_ARG, "state_buf must be 256-byte aligned");
  for (size_t i = 0; i < n_params; ++i)
    if (!std::isfinite(host_params[i])) return fail(LNM_ERR_ARG, "parameters must be finite");
  auto* tr = new (std::nothrow) lnm_trainer_s;
  if (!tr) return fail(LNM_ERR_OOM, "host allocation failed");
  char* st = static_cast<char*>(state_buf);
  tr->ctx = ctx;
  tr->state = st;
  tr->n_params = n_params;
  tr->p = reinterpret_cast<float*>(st + sl.p);
  tr->g = reinterpret_cast<float*>(st + sl.g);
  tr->m = reinterpret_cast<float*>(st + sl.m);
  tr->v = reinterpret_cast<float*>(st + sl.v);
  tr->net.levels = levels;
  tr->net.base = base;
  tr->net.precision = LNM_FP32;
  tr->net.layers = sl.fwd;
  tr->net.dev = st + sl.net;
  tr->net.dev_bytes = sl.net_bytes;
  tr->dgrad = sl.dg;
  tr->dgrad_off = sl.dgrad_w;
  tr->zeros = reinterpret_cast<float*>(st + sl.zeros);
  tr->step = 0;
  size_t off = 0;
  for (auto& d : sl.fwd) {
    tr->flat_w.push_back(off);
    off += (size_t)d.co * d.ci * d.k * d.k;
    tr->flat_b.push_back(off);
    off += d.co;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(tr->p, host_params, sizeof(float) * n_params, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(tr->g, 0, sizeof(float) * n_params, s);
  if (e == hipSuccess) e = hipMemsetAsync(tr->m, 0, sizeof(float) * n_params, s);
  if (e == hipSuccess) e = hipMemsetAsync(tr->v, 0, sizeof(float) * n_params, s);
  if (e == hipSuccess) e = hipMemsetAsync(tr->zeros, 0, sizeof(float) * sl.max_dg_co_pad, s);
  if (e != hipSuccess) {
    delete tr;
    return fail(LNM_ERR_DEVICE, std::string("trainer upload: ") + hipGetErrorString(e));
  }
  lnm_status rs = repack(tr, s);
  if (rs == LNM_OK && hipStreamSynchronize(s) != hipSuccess) rs = fail(LNM_ERR_DEVICE, "synchronise failed");
  if (rs) {
    delete tr;
    return rs;
  }
  *out = tr;
  return LNM_OK;
}

void lnm_trainer_destroy(lnm_trainer tr) { delete tr; }

lnm_status lnm_train_grad(lnm_ctx ctx, lnm_trainer tr, int32_t batch, int32_t H, int32_t W, const float* guide,
                          const float* target, float* loss, float* grad, void* workspace, size_t ws_bytes,
                          void* stream) {
  lnm_status st = check_train(ctx, tr, batch, H, W, guide, target, workspace, ws_bytes);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = static_cast<char*>(workspace);
  st = grad_impl(ctx, tr, batch, H, W, guide, target, ws, s);
  if (st) return st;
  const TrainPlan tp = train_plan(&tr->net, batch, H, W, tr->ad_c);
  if (loss) LNM_HIP_CHECK(hipMemcpyAsync(loss, ws + tp.loss, sizeof(float), hipMemcpyDeviceToDevice, s));
  if (grad)
    LNM_HIP_CHECK(hipMemcpyAsync(grad, tr->g, sizeof(float) * tr->n_params, hipMemcpyDeviceToDevice, s));
  return LNM_OK;
}

lnm_status lnm_train_step(lnm_ctx ctx, lnm_trainer tr, int32_t batch, int32_t H, int32_t W, const float* guide,
                          const float* target, float lr, float beta1, float beta2, float eps, float* loss,
                          void* workspace, size_t ws_bytes, void* stream) {
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(LNM_ERR_ARG, "Adam hyper-parameters out of range");
  lnm_status st = lnm_train_grad(ctx, tr, batch, H, W, guide, target, loss, nullptr, workspace, ws_bytes, stream);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  tr->step += 1;
  LNM_HIP_CHECK(launch_adam(tr->p, tr->g, tr->m, tr->v, (long)tr->n_params, lr, beta1, beta2, eps, tr->step, s));
  if (tr->ad_c)
    LNM_HIP_CHECK(launch_adam(tr->ad_p, tr->ad_g, tr->ad_m, tr->ad_v, (long)tr->ad_n, lr, beta1, beta2, eps,
                              tr->step, s));
  return repack(tr, s);
}

size_t lnm_trainer_adapters_state_bytes(int32_t c) {
  if (!adapter_width_supported(c)) return 0;
  return 4 * align256(sizeof(float) * 4 * (7 * (size_t)c * c + 35 * (size_t)c + 2));
}

lnm_status lnm_trainer_attach_adapters(lnm_trainer tr, const float* host_params, size_t n_params, void* state_buf,
                                       size_t state_bytes, void* stream) {
  if (!tr || !host_params || !state_buf) return fail(LNM_ERR_ARG, "NULL argument");
  const int c = tr->net.base;
  if (!adapter_width_supported(c)) return fail(LNM_ERR_UNSUPPORTED, "adapters need a base width of 16, 32, 48 or 64");
  if (tr->ad_c) return fail(LNM_ERR_ARG, "the trainer already has adapters");
  if (tr->step != 0) return fail(LNM_ERR_ARG, "adapters are attached before the first step");
  const size_t n = 4 * (7 * (size_t)c * c + 35 * (size_t)c + 2);
  if (n_params != n) return fail(LNM_ERR_SHAPE, "adapter parameters: expected " + std::to_string(n));
  if (state_bytes < lnm_trainer_adapters_state_bytes(c))
    return fail(LNM_ERR_SHAPE, "adapter state buffer too small: need " +
                                   std::to_string(lnm_trainer_adapters_state_bytes(c)));
  if (reinterpret_cast<uintptr_t>(state_buf) % 256) return fail(LNM_ERR_ARG, "state_buf must be 256-byte aligned");
  for (size_t i = 0; i < n_params; ++i)
    if (!std::isfinite(host_params[i])) return fail(LNM_ERR_ARG, "adapter parameters must be finite");
  char* st = static_cast<char*>(state_buf);
  const size_t one = align256(sizeof(float) * n);
  float* p = reinterpret_cast<float*>(st);
  float* g = reinterpret_cast<float*>(st + one);
  float* m = reinterpret_cast<float*>(st + 2 * one);
  float* v = reinterpret_cast<float*>(st + 3 * one);
  hipStream_t s = (hipStream_t)stream;
  LNM_HIP_CHECK(hipMemcpyAsync(p, host_params, sizeof(float) * n, hipMemcpyHostToDevice, s));
  LNM_HIP_CHECK(launch_fill_zero(g, (long)n, s));
  LNM_HIP_CHECK(launch_fill_zero(m, (long)n, s));
  LNM_HIP_CHECK(launch_fill_zero(v, (long)n, s));
  LNM_HIP_CHECK(hipStreamSynchronize(s));
  tr->ad_c = c;
  tr->ad_n = n;
  tr->ad_p = p;
  tr->ad_g = g;
  tr->ad_m = m;
  tr->ad_v = v;
  return LNM_OK;
}

size_t lnm_trainer_workspace_bytes(lnm_trainer tr, int32_t batch, int32_t H, int32_t W) {
  if (!tr || batch < 1 || H < 1 || W < 1) return 0;
  return train_plan(&tr->net, batch, H, W, tr->ad_c).bytes;
}

lnm_status lnm_trainer_read_adapters(lnm_trainer tr, float* host_params, size_t n_params, void* stream) {
  if (!tr || !host_params) return fail(LNM_ERR_ARG, "NULL argument");
  if (!tr->ad_c) return fail(LNM_ERR_ARG, "the trainer has no adapters");
  if (n_params != tr->ad_n) return fail(LNM_ERR_SHAPE, "n_params does not match the adapters");
  LNM_HIP_CHECK(hipMemcpyAsync(host_params, tr->ad_p, sizeof(float) * n_params, hipMemcpyDeviceToHost,
                               (hipStream_t)stream));
  LNM_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  return LNM_OK;
}

lnm_status lnm_trainer_adapter_grad(lnm_trainer tr, float* grad, size_t n_params, void* stream) {
  if (!tr || !grad) return fail(LNM_ERR_ARG, "NULL argument");
  if (!tr->ad_c) return fail(LNM_ERR_ARG, "the trainer has no adapters");
  if (n_params != tr->ad_n) return fail(LNM_ERR_SHAPE, "n_params does not match the adapters");
  LNM_HIP_CHECK(hipMemcpyAsync(grad, tr->ad_g, sizeof(float) * n_params, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
  return LNM_OK;
}

lnm_status lnm_trainer_read_params(lnm_trainer tr, float* host_params, size_t n_params, void* stream) {
  if (!tr || !host_params) return fail(LNM_ERR_ARG, "NULL argument");
  if (n_params != tr->n_params) return fail(LNM_ERR_SHAPE, "n_params does not match");
  LNM_HIP_CHECK(hipMemcpyAsync(host_params, tr->p, sizeof(float) * n_params, hipMemcpyDeviceToHost,
                               (hipStream_t)stream));
  LNM_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  return LNM_OK;
}

lnm_status lnm_trainer_save(lnm_trainer tr, float* host_m, float* host_v, int32_t* step, size_t n_params,
                            void* stream) {
  if (!tr || !host_m || !host_v || !step) return fail(LNM_ERR_ARG, "NULL argument");
  if (n_params != tr->n_params) return fail(LNM_ERR_SHAPE, "n_params does not match");
  hipStream_t s = (hipStream_t)stream;
  LNM_HIP_CHECK(hipMemcpyAsync(host_m, tr->m, sizeof(float) * n_params, hipMemcpyDeviceToHost, s));
  LNM_HIP_CHECK(hipMemcpyAsync(host_v, tr->v, sizeof(float) * n_params, hipMemcpyDeviceToHost, s));
  LNM_HIP_CHECK(hipStreamSynchronize(s));
  *step = tr->step;
  return LNM_OK;
}

lnm_status lnm_trainer_load(lnm_trainer tr, const float* host_params, const float* host_m, const float* host_v,
                            int32_t step, size_t n_params, void* stream) {
  if (!tr || !host_params || !host_m || !host_v) return fail(LNM_ERR_ARG, "NULL argument");
  if (n_params != tr->n_params || step < 0) return fail(LNM_ERR_SHAPE, "n_params or step does not match");
  hipStream_t s = (hipStream_t)stream;
  LNM_HIP_CHECK(hipMemcpyAsync(tr->p, host_params, sizeof(float) * n_params, hipMemcpyHostToDevice, s));
  LNM_HIP_CHECK(hipMemcpyAsync(tr->m, host_m, sizeof(float) * n_params, hipMemcpyHostToDevice, s));
  LNM_HIP_CHECK(hipMemcpyAsync(tr->v, host_v, sizeof(float) * n_params, hipMemcpyHostToDevice, s));
  tr->step = step;
  lnm_status st = repack(tr, s);
  if (st) return st;
  LNM_HIP_CHECK(hipStreamSynchronize(s));
  return LNM_OK;
}

lnm_status lnm_trainer_infer(lnm_ctx ctx, lnm_trainer tr, int32_t batch, int32_t H, int32_t W, const float* guide,
                             float* lightmaps, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx || !tr || !guide || !lightmaps) return fail(LNM_ERR_ARG, "NULL argument");
  if (tr->ad_c)
    return fail(LNM_ERR_UNSUPPORTED,
                "the trainer has adapters: infer with lnm_infer_adapters on its read-back parameters");
  lnm_status st = check_infer(&tr->net, batch, H, W, ws_bytes, workspace);
  if (st) return st;
  return run_unet(ctx, &tr->net, batch, H, W, guide, lightmaps, nullptr, static_cast<char*>(workspace),
                  (hipStream_t)stream, nullptr, false, true);
}

}  // extern "C"
