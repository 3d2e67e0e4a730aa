// Error paths of the C ABI, run against the library's host code built for the
// CPU with counting launch stubs (fake_device.cpp): every call with a bad
// argument returns its documented status, sets an error message and
// enqueues nothing; valid calls return LNM_OK and launch.  Built and run
// under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py.  Test infrastructure only.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lnm.h"

extern "C" long fake_launch_count();
extern "C" void fake_fail_after(long n);

static int g_failures = 0, g_checks = 0;

// status must equal `want`; an error must set a message and launch nothing
static void expect(const char* what, lnm_status got, lnm_status want, long launches_before) {
  ++g_checks;
  const long launched = fake_launch_count() - launches_before;
  bool ok = got == want;
  if (want != LNM_OK) ok = ok && launched == 0 && lnm_last_error()[0] != '\0';
  if (want == LNM_OK) ok = ok && launched > 0;
  if (!ok) {
    ++g_failures;
    std::printf("FAIL %s: status %d (want %d), %ld launches, error \"%s\"\n", what, (int)got, (int)want, launched,
                lnm_last_error());
  }
}
// a condition with no status (sizes), or a call that only copies memory
#define CHECK(cond)                                              \
  do {                                                           \
    ++g_checks;                                                  \
    if (!(cond)) {                                               \
      ++g_failures;                                              \
      std::printf("FAIL %s (error \"%s\")\n", #cond, lnm_last_error()); \
    }                                                            \
  } while (0)

#define EXPECT(call, want)                       \
  do {                                           \
    const long before_ = fake_launch_count();    \
    expect(#call, (call), (want), before_);      \
  } while (0)

static lnm_camera camera(int w, int h) {
  lnm_camera c{};
  c.projection = LNM_PERSPECTIVE;
  c.eye[0] = 3.0f;
  c.eye[1] = c.eye[2] = 0.5f;
  c.target[0] = c.target[1] = c.target[2] = 0.5f;
  c.up[1] = 1.0f;
  c.fov_y_deg = 60.0f;
  c.ortho_half_extent = 0.8f;
  c.width = w;
  c.height = h;
  return c;
}

static lnm_march_params params() {
  lnm_march_params p{};
  p.step_voxels = 4.0f;
  p.depth_tau = 0.1f;
  p.ert_eps = 1e-6f;
  p.jitter_on = 1;
  p.light_w[0] = p.light_w[1] = p.light_w[2] = 1.0f;
  return p;
}

int main() {
  lnm_ctx ctx = nullptr;
  EXPECT(lnm_ctx_create(0, nullptr), LNM_ERR_ARG);
  EXPECT(lnm_ctx_create(3, &ctx), LNM_ERR_ARG);
  if (lnm_ctx_create(0, &ctx) != LNM_OK || !ctx) {
    std::printf("FAIL lnm_ctx_create\n");
    return 1;
  }

  // ---------------------------------------------------------------- march
  std::vector<float> grid(32 * 32 * 32, 0.5f);
  lnm_volume vol{grid.data(), 32, 32, 32, 8.0f, nullptr};
  lnm_camera cam = camera(64, 48);
  lnm_march_params prm = params();
  const size_t ws_bytes = lnm_march_workspace_bytes(&vol, &cam, &prm);
  std::vector<char> ws(ws_bytes + 256);
  std::vector<float> guide(64 * 48 * 3);
  EXPECT(lnm_march(ctx, &vol, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_OK);
  EXPECT(lnm_march(nullptr, &vol, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
  EXPECT(lnm_march(ctx, &vol, &cam, &prm, nullptr, ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
  EXPECT(lnm_march(ctx, nullptr, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
  EXPECT(lnm_march(ctx, &vol, nullptr, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
  EXPECT(lnm_march(ctx, &vol, &cam, &prm, guide.data(), ws.data(), ws_bytes - 1, nullptr), LNM_ERR_SHAPE);
  EXPECT(lnm_march(ctx, &vol, &cam, &prm, guide.data(), nullptr, ws_bytes, nullptr), LNM_ERR_SHAPE);
  {
    lnm_volume v = vol;
    v.density = nullptr;
    EXPECT(lnm_march(ctx, &v, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    v = vol;
    v.ny = 0;
    EXPECT(lnm_march(ctx, &v, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_SHAPE);
    v = vol;
    v.nx = v.ny = v.nz = 2000;  // over the 4 GiB bricked-grid limit
    EXPECT(lnm_march(ctx, &v, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_SHAPE);
    v = vol;
    v.sigma_scale = -1.0f;
    EXPECT(lnm_march(ctx, &v, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    v.sigma_scale = NAN;
    EXPECT(lnm_march(ctx, &v, &cam, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
  }
  {
    lnm_camera c = cam;
    c.projection = 7;
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    c = cam;
    c.width = 0;
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    c = cam;
    c.eye[1] = INFINITY;
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    c = cam;
    c.eye[0] = c.eye[1] = c.eye[2] = 0.5f;  // target == eye
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    c = cam;
    c.up[0] = -1.0f;  // up parallel to the view direction
    c.up[1] = 0.0f;
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    c = cam;
    c.fov_y_deg = 180.0f;
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    c = cam;
    c.projection = LNM_ORTHOGRAPHIC;
    c.ortho_half_extent = 0.0f;
    EXPECT(lnm_march(ctx, &vol, &c, &prm, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
  }
  {
    lnm_march_params p = prm;
    p.step_voxels = 0.0f;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    p = prm;
    p.depth_tau = -0.5f;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    p = prm;
    p.ert_eps = 1.0f;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    p = prm;
    p.quadrature = 2;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    p = prm;
    p.light_w[2] = NAN;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    p = prm;
    p.light_set = 2;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    p = prm;
    p.work_order = 9;
    EXPECT(lnm_march(ctx, &vol, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_ARG);
    lnm_volume big = vol;
    big.nx = big.ny = 160;  // a z cell's planes do not fit in LDS
    p = prm;
    p.work_order = LNM_ORDER_CELLS;
    EXPECT(lnm_march(ctx, &big, &cam, &p, guide.data(), ws.data(), ws_bytes, nullptr), LNM_ERR_UNSUPPORTED);
  }
  // batch: every entry is checked before the first launch
  {
    lnm_volume vols[2] = {vol, vol};
    lnm_camera cams[2] = {cam, cam};
    lnm_march_params prms[2] = {prm, prm};
    float* outs[2] = {guide.data(), guide.data()};
    const size_t bw = lnm_march_batch_workspace_bytes(2, vols, cams, prms);
    std::vector<char> bws(bw);
    EXPECT(lnm_march_batch(ctx, 2, vols, cams, prms, outs, bws.data(), bw, nullptr), LNM_OK);
    EXPECT(lnm_march_batch(ctx, 0, vols, cams, prms, outs, bws.data(), bw, nullptr), LNM_ERR_ARG);
    cams[1].fov_y_deg = 0.0f;
    EXPECT(lnm_march_batch(ctx, 2, vols, cams, prms, outs, bws.data(), bw, nullptr), LNM_ERR_ARG);
    cams[1] = cam;
    outs[1] = nullptr;
    EXPECT(lnm_march_batch(ctx, 2, vols, cams, prms, outs, bws.data(), bw, nullptr), LNM_ERR_ARG);
  }
  // bricks and reference lightmaps
  {
    const size_t bb = lnm_bricks_bytes(32, 32, 32);
    std::vector<char> bricks(bb);
    EXPECT(lnm_make_bricks(ctx, &vol, reinterpret_cast<float*>(bricks.data()), bb, nullptr), LNM_OK);
    EXPECT(lnm_make_bricks(ctx, &vol, reinterpret_cast<float*>(bricks.data()), bb - 4, nullptr), LNM_ERR_SHAPE);
    std::vector<float> lm(64 * 48 * 6);
    EXPECT(lnm_reference_lightmaps(ctx, &vol, &cam, 0.25f, 1e-6f, 1, lm.data(), nullptr), LNM_OK);
    EXPECT(lnm_reference_lightmaps(ctx, &vol, &cam, -1.0f, 1e-6f, 1, lm.data(), nullptr), LNM_ERR_ARG);
    EXPECT(lnm_reference_lightmaps(ctx, &vol, &cam, 0.25f, 1e-6f, 1, nullptr, nullptr), LNM_ERR_ARG);
  }

  // ---------------------------------------------------------------- network
  const int L = 3, base = 16;
  const size_t np = lnm_net_param_count(L, base);
  std::vector<float> prm_host(np, 0.01f);
  const size_t nb32 = lnm_net_device_bytes(L, base, LNM_FP32);
  std::vector<char> dev_storage(nb32 + 512);
  char* dev = dev_storage.data() + (256 - reinterpret_cast<uintptr_t>(dev_storage.data()) % 256) % 256;
  lnm_net net = nullptr;
  EXPECT(lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np, nullptr, dev, nb32, nullptr, nullptr),
         LNM_ERR_ARG);
  EXPECT(lnm_net_create(ctx, L, base, 7, prm_host.data(), np, nullptr, dev, nb32, nullptr, &net),
         LNM_ERR_UNSUPPORTED);
  EXPECT(lnm_net_create(ctx, L, 24, LNM_FP32, prm_host.data(), np, nullptr, dev, nb32, nullptr, &net),
         LNM_ERR_SHAPE);
  EXPECT(lnm_net_create(ctx, 1, base, LNM_FP32, prm_host.data(), np, nullptr, dev, nb32, nullptr, &net),
         LNM_ERR_SHAPE);
  EXPECT(lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np - 1, nullptr, dev, nb32, nullptr, &net),
         LNM_ERR_SHAPE);
  EXPECT(lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np, nullptr, dev, nb32 - 1, nullptr, &net),
         LNM_ERR_SHAPE);
  EXPECT(lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np, nullptr, dev + 16, nb32, nullptr, &net),
         LNM_ERR_ARG);
  {
    std::vector<float> scales(4 * L - 2, 1.0f);
    EXPECT(lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np, scales.data(), dev, nb32, nullptr, &net),
           LNM_ERR_ARG);
    EXPECT(lnm_net_create(ctx, L, base, LNM_FP8_E4M3, prm_host.data(), np, nullptr, dev, nb32, nullptr, &net),
           LNM_ERR_ARG);
    scales[1] = -1.0f;
    EXPECT(lnm_net_create(ctx, L, base, LNM_FP8_E4M3, prm_host.data(), np, scales.data(), dev, nb32, nullptr, &net),
           LNM_ERR_ARG);
    std::vector<float> bad = prm_host;
    bad[5] = NAN;
    EXPECT(lnm_net_create(ctx, L, base, LNM_FP32, bad.data(), np, nullptr, dev, nb32, nullptr, &net), LNM_ERR_ARG);
  }
  // a failed weight upload: LNM_ERR_DEVICE and no net
  fake_fail_after(0);
  {
    const long before = fake_launch_count();
    lnm_net failed = nullptr;
    const lnm_status st = lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np, nullptr, dev, nb32, nullptr,
                                         &failed);
    ++g_checks;
    if (st != LNM_ERR_DEVICE || failed || fake_launch_count() != before) {
      ++g_failures;
      std::printf("FAIL upload failure: status %d\n", (int)st);
    }
  }
  fake_fail_after(-1);
  if (lnm_net_create(ctx, L, base, LNM_FP32, prm_host.data(), np, nullptr, dev, nb32, nullptr, &net) != LNM_OK) {
    std::printf("FAIL lnm_net_create: %s\n", lnm_last_error());
    return 1;
  }
  {
    const int B = 2, H = 32, W = 40;
    const size_t iw = lnm_workspace_bytes(net, B, H, W);
    std::vector<char> iws(iw);
    std::vector<float> g(B * H * W * 3), lm(B * H * W * 6);
    EXPECT(lnm_infer(ctx, net, B, H, W, g.data(), lm.data(), nullptr, iws.data(), iw, nullptr), LNM_OK);
    EXPECT(lnm_infer(ctx, nullptr, B, H, W, g.data(), lm.data(), nullptr, iws.data(), iw, nullptr), LNM_ERR_ARG);
    EXPECT(lnm_infer(ctx, net, 0, H, W, g.data(), lm.data(), nullptr, iws.data(), iw, nullptr), LNM_ERR_SHAPE);
    EXPECT(lnm_infer(ctx, net, B, 30, W, g.data(), lm.data(), nullptr, iws.data(), iw, nullptr), LNM_ERR_SHAPE);
    EXPECT(lnm_infer(ctx, net, B, H, W, g.data(), lm.data(), nullptr, iws.data(), iw - 1, nullptr), LNM_ERR_SHAPE);
    // a failed launch in the middle of the network: LNM_ERR_DEVICE
    fake_fail_after(3);
    ++g_checks;
    if (lnm_infer(ctx, net, B, H, W, g.data(), lm.data(), nullptr, iws.data(), iw, nullptr) != LNM_ERR_DEVICE) {
      ++g_failures;
      std::printf("FAIL launch failure in lnm_infer\n");
    }
    fake_fail_after(-1);
    std::vector<float> amax(4 * L - 2);
    EXPECT(lnm_calibrate_amax(ctx, net, 1, H, W, g.data(), amax.data(), 4 * L - 3, iws.data(), iw, nullptr),
           LNM_ERR_SHAPE);
    EXPECT(lnm_calibrate_amax(ctx, net, 1, H, W, g.data(), amax.data(), 4 * L - 2, iws.data(), iw, nullptr), LNM_OK);
  }
  // frame, static frame, shading
  {
    lnm_camera c = camera(64, 64);
    const size_t fw = lnm_frame_workspace_bytes(net, &vol, &c, &prm);
    std::vector<char> fws(fw);
    std::vector<float> g(64 * 64 * 3), lm(64 * 64 * 6), rgba(64 * 64 * 4);
    lnm_light light{{0.3f, 1.0f, -0.2f}, {1.0f, 1.0f, 1.0f}};
    EXPECT(lnm_frame(ctx, net, &vol, &c, &prm, &light, 1, g.data(), lm.data(), rgba.data(), fws.data(), fw, nullptr),
           LNM_OK);
    EXPECT(lnm_frame(ctx, net, &vol, &c, &prm, &light, 17, g.data(), lm.data(), rgba.data(), fws.data(), fw,
                     nullptr),
           LNM_ERR_ARG);
    EXPECT(lnm_frame(ctx, net, &vol, &c, &prm, &light, 1, g.data(), lm.data(), rgba.data(), fws.data(), fw / 2,
                     nullptr),
           LNM_ERR_SHAPE);
    EXPECT(lnm_frame_static(ctx, net, &vol, &c, &prm, &light, 1, g.data(), lm.data(), rgba.data(), nullptr), LNM_OK);
    lnm_camera huge = camera(1024, 1024);
    std::vector<float> hg(1024 * 1024 * 3), hlm(1024 * 1024 * 6);
    EXPECT(lnm_frame_static(ctx, net, &vol, &huge, &prm, &light, 1, hg.data(), hlm.data(), nullptr, nullptr),
           LNM_ERR_SHAPE);
    EXPECT(lnm_composite(ctx, &c, &light, 1, 1, 64, 64, lm.data(), g.data(), rgba.data(), nullptr), LNM_OK);
    lnm_light bad_light{{NAN, 1.0f, 0.0f}, {1.0f, 1.0f, 1.0f}};
    EXPECT(lnm_composite(ctx, &c, &bad_light, 1, 1, 64, 64, lm.data(), g.data(), rgba.data(), nullptr), LNM_ERR_ARG);
    lnm_camera cams[2] = {c, c};
    lnm_light lights[2] = {light, light};
    int32_t start[3] = {0, 1, 2};
    std::vector<float> g2(2 * 64 * 64 * 3), lm2(2 * 64 * 64 * 6), rgba2(2 * 64 * 64 * 4);
    EXPECT(lnm_composite_batch(ctx, 2, cams, lights, start, 64, 64, lm2.data(), g2.data(), rgba2.data(), nullptr),
           LNM_OK);
    start[0] = 1;
    EXPECT(lnm_composite_batch(ctx, 2, cams, lights, start, 64, 64, lm2.data(), g2.data(), rgba2.data(), nullptr),
           LNM_ERR_ARG);
    start[0] = 0;
    cams[1].width = 65;
    EXPECT(lnm_composite_batch(ctx, 2, cams, lights, start, 64, 64, lm2.data(), g2.data(), rgba2.data(), nullptr),
           LNM_ERR_SHAPE);
    EXPECT(lnm_composite_batch(ctx, 65, cams, lights, start, 64, 64, lm2.data(), g2.data(), rgba2.data(), nullptr),
           LNM_ERR_ARG);
    // shadows
    lnm_shadow_frame sf{{0.5f, 0.5f, 0.5f}, 0.9f, 64, 0.01f};
    std::vector<float> depth(64 * 64);
    const float centre[3] = {0.5f, 0.5f, 0.5f};
    EXPECT(lnm_shadow_map_sphere(ctx, &sf, light.dir, centre, 0.15f, depth.data(), nullptr), LNM_OK);
    lnm_shadow_frame bad_sf = sf;
    bad_sf.size = 0;
    EXPECT(lnm_shadow_map_sphere(ctx, &bad_sf, light.dir, centre, 0.15f, depth.data(), nullptr), LNM_ERR_SHAPE);
    bad_sf = sf;
    bad_sf.half_extent = -1.0f;
    EXPECT(lnm_shadow_map_sphere(ctx, &bad_sf, light.dir, centre, 0.15f, depth.data(), nullptr), LNM_ERR_ARG);
    const float* maps[1] = {depth.data()};
    EXPECT(lnm_composite_shadowed(ctx, &c, &light, 1, &sf, maps, 1, 64, 64, lm.data(), g.data(), rgba.data(),
                                  nullptr, nullptr),
           LNM_OK);
    EXPECT(lnm_composite_shadowed(ctx, &c, &light, 1, &bad_sf, maps, 1, 64, 64, lm.data(), g.data(), rgba.data(),
                                  nullptr, nullptr),
           LNM_ERR_ARG);
  }
  // channel adapters
  {
    const size_t na = lnm_adapters_param_count(base);
    std::vector<float> ap(na, 0.0f);
    std::vector<char> adev(lnm_adapters_device_bytes(base) + 256);
    lnm_adapters ad = nullptr;
    EXPECT(lnm_adapters_create(ctx, net, ap.data(), na - 1, adev.data(), adev.size(), nullptr, &ad), LNM_ERR_SHAPE);
    if (lnm_adapters_create(ctx, net, ap.data(), na, adev.data(), adev.size(), nullptr, &ad) == LNM_OK) {
      const size_t aw = lnm_adapters_workspace_bytes(ad, 1, 32, 32);
      std::vector<char> aws(aw);
      std::vector<float> g(32 * 32 * 3), lm(32 * 32 * 6);
      EXPECT(lnm_infer_adapters(ctx, ad, 1, 32, 32, g.data(), lm.data(), nullptr, aws.data(), aw, nullptr), LNM_OK);
      EXPECT(lnm_infer_adapters(ctx, ad, 1, 32, 32, g.data(), lm.data(), nullptr, aws.data(), aw - 1, nullptr),
             LNM_ERR_SHAPE);
      lnm_adapters_destroy(ad);
    } else {
      ++g_failures;
      std::printf("FAIL lnm_adapters_create: %s\n", lnm_last_error());
    }
  }
  // training
  {
    const size_t sb = lnm_trainer_state_bytes(L, base);
    std::vector<char> state(sb + 512);
    char* st = state.data() + (256 - reinterpret_cast<uintptr_t>(state.data()) % 256) % 256;
    lnm_trainer tr = nullptr;
    EXPECT(lnm_trainer_create(ctx, L, base, prm_host.data(), np - 1, st, sb, nullptr, &tr), LNM_ERR_SHAPE);
    if (lnm_trainer_create(ctx, L, base, prm_host.data(), np, st, sb, nullptr, &tr) == LNM_OK) {
      const int B = 2, H = 32, W = 32;
      const size_t tw = lnm_train_workspace_bytes(L, base, B, H, W);
      std::vector<char> tws(tw);
      std::vector<float> g(B * H * W * 3), t(B * H * W * 6);
      EXPECT(lnm_train_step(ctx, tr, B, H, W, g.data(), t.data(), 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, tws.data(), tw,
                            nullptr),
             LNM_OK);
      EXPECT(lnm_train_step(ctx, tr, B, H, W, g.data(), t.data(), 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, tws.data(),
                            tw - 1, nullptr),
             LNM_ERR_SHAPE);
      lnm_trainer_destroy(tr);
    } else {
      ++g_failures;
      std::printf("FAIL lnm_trainer_create: %s\n", lnm_last_error());
    }
  }
  // training with channel adapters
  {
    const size_t sb = lnm_trainer_state_bytes(L, base);
    std::vector<char> state(sb + 512);
    char* st = state.data() + (256 - reinterpret_cast<uintptr_t>(state.data()) % 256) % 256;
    const size_t na = lnm_adapters_param_count(base), ab = lnm_trainer_adapters_state_bytes(base);
    std::vector<char> astate(ab + 512);
    char* ast = astate.data() + (256 - reinterpret_cast<uintptr_t>(astate.data()) % 256) % 256;
    std::vector<float> ap(na, 0.01f), back(na);
    CHECK(lnm_trainer_adapters_state_bytes(17) == 0);
    lnm_trainer tr = nullptr;
    if (lnm_trainer_create(ctx, L, base, prm_host.data(), np, st, sb, nullptr, &tr) == LNM_OK) {
      const int B = 2, H = 32, W = 32;
      const size_t plain = lnm_trainer_workspace_bytes(tr, B, H, W);
      CHECK(plain == lnm_train_workspace_bytes(L, base, B, H, W));
      EXPECT(lnm_trainer_read_adapters(tr, back.data(), na, nullptr), LNM_ERR_ARG);
      EXPECT(lnm_trainer_attach_adapters(tr, ap.data(), na - 1, ast, ab, nullptr), LNM_ERR_SHAPE);
      EXPECT(lnm_trainer_attach_adapters(tr, ap.data(), na, ast, ab - 1, nullptr), LNM_ERR_SHAPE);
      EXPECT(lnm_trainer_attach_adapters(tr, ap.data(), na, ast + 4, ab, nullptr), LNM_ERR_ARG);
      EXPECT(lnm_trainer_attach_adapters(nullptr, ap.data(), na, ast, ab, nullptr), LNM_ERR_ARG);
      EXPECT(lnm_trainer_attach_adapters(tr, ap.data(), na, ast, ab, nullptr), LNM_OK);
      EXPECT(lnm_trainer_attach_adapters(tr, ap.data(), na, ast, ab, nullptr), LNM_ERR_ARG);
      const size_t tw = lnm_trainer_workspace_bytes(tr, B, H, W);
      CHECK(tw > plain);
      std::vector<char> tws(tw);
      std::vector<float> g(B * H * W * 3), t(B * H * W * 6), ag(na);
      EXPECT(lnm_train_step(ctx, tr, B, H, W, g.data(), t.data(), 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, tws.data(), tw,
                            nullptr),
             LNM_OK);
      EXPECT(lnm_train_step(ctx, tr, B, H, W, g.data(), t.data(), 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, tws.data(),
                            plain, nullptr),
             LNM_ERR_SHAPE);
      EXPECT(lnm_trainer_read_adapters(tr, back.data(), na + 1, nullptr), LNM_ERR_SHAPE);
      CHECK(lnm_trainer_read_adapters(tr, back.data(), na, nullptr) == LNM_OK && back == ap);
      CHECK(lnm_trainer_adapter_grad(tr, ag.data(), na, nullptr) == LNM_OK);
      std::vector<float> lmo(B * H * W * 6);
      EXPECT(lnm_trainer_infer(ctx, tr, B, H, W, g.data(), lmo.data(), tws.data(), tw, nullptr), LNM_ERR_UNSUPPORTED);
      EXPECT(lnm_trainer_adapter_grad(tr, nullptr, na, nullptr), LNM_ERR_ARG);
      lnm_trainer_destroy(tr);
    } else {
      ++g_failures;
      std::printf("FAIL lnm_trainer_create: %s\n", lnm_last_error());
    }
    // adapters come before the first step
    if (lnm_trainer_create(ctx, L, base, prm_host.data(), np, st, sb, nullptr, &tr) == LNM_OK) {
      const int B = 1, H = 16, W = 16;
      const size_t tw = lnm_trainer_workspace_bytes(tr, B, H, W);
      std::vector<char> tws(tw);
      std::vector<float> g(B * H * W * 3), t(B * H * W * 6);
      EXPECT(lnm_train_step(ctx, tr, B, H, W, g.data(), t.data(), 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, tws.data(), tw,
                            nullptr),
             LNM_OK);
      EXPECT(lnm_trainer_attach_adapters(tr, ap.data(), na, ast, ab, nullptr), LNM_ERR_ARG);
      lnm_trainer_destroy(tr);
    }
  }
  // profiling
  {
    int32_t n = 0;
    double ms = 0.0;
    EXPECT(lnm_profile_read(ctx, LNM_K_COUNT, &n, &ms), LNM_ERR_ARG);
  }
  lnm_net_destroy(net);
  lnm_ctx_destroy(ctx);
  std::printf("%d checks, %d failures\n", g_checks, g_failures);
  return g_failures ? 1 : 0;
}
