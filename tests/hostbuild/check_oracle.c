/* Runs every function of the fp64 oracle once on small inputs (ragged sizes,
 * perspective and orthographic views, both quadratures, both light sets,
 * the network forward and backward, adapters, shading and shadows) so that
 * tests/test_host_sanitized.py can execute the oracle under
 * AddressSanitizer and UndefinedBehaviorSanitizer.  The values themselves
 * are pinned elsewhere (tests/test_oracle_*.py); here only finiteness is
 * checked.  Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t orc_splitmix64(uint64_t state);
double orc_jitter(uint64_t seed, uint32_t frame, uint32_t pixel);
double orc_sigma_vol(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* p);
int orc_march(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* cam, double step_voxels,
              double depth_tau, double ert_eps, int jitter_on, uint64_t jitter_seed, uint32_t frame, int quadrature,
              const double* light_w, int light_set, int unit_radiance, int stride, double* guide, double* d_margin,
              long long* counters);
double orc_front_identity_gap(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* cam,
                              double step_voxels, int jitter_on, uint64_t seed);
int orc_reference_lightmaps(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* cam,
                            double step_voxels, double ert_eps, double* lm);
int orc_composite(int H, int W, const double* lm, const double* guide, const double* cam, const double* lights,
                  int n_lights, double* rgba);
void orc_shadow_map_sphere(int S, double E, const double* origin, const double* light, const double* centre,
                           double radius, double* depth);
void orc_shadow_visibility(int H, int W, const double* guide, const double* cam, const double* light, int S, double E,
                           const double* origin, const double* depth, double bias, double* vis, double* margin);
int orc_composite_shadowed(int H, int W, const double* lm, const double* guide, const double* cam,
                           const double* lights, int n_lights, const double* vis, double* rgba);
long orc_unet_param_count(int levels, int base);
int orc_unet_forward(int levels, int base, const float* params, long n_params, int B, int H, int W,
                     const double* guide, double* lightmaps, double* logits);
int orc_unet_loss_grad(int levels, int base, const float* params, long n_params, int B, int H, int W,
                       const double* guide, const double* target, double* loss, double* grad);
int orc_unet_features(int levels, int base, const float* params, long n_params, int B, int H, int W,
                      const double* guide, double* feat);
long orc_adapter_param_count(int c);
int orc_adapters_forward(int c, const float* params, long n_params, int B, int H, int W, const double* feat,
                         double* lightmaps, double* extra);
int orc_adapters_loss_grad(int levels, int base, const float* params, long n_params, const float* ad_params,
                           long n_ad, int B, int H, int W, const double* guide, const double* target, double* loss,
                           double* grad, double* grad_ad);
void orc_adam(long n, double* p, const double* g, double* m, double* v, int t, double lr, double b1, double b2,
              double eps);

static int failures = 0;
static void check_finite(const char* what, const double* x, long n) {
  for (long i = 0; i < n; ++i)
    if (!isfinite(x[i])) {
      printf("FAIL %s: entry %ld is not finite\n", what, i);
      ++failures;
      return;
    }
}

static uint64_t rng = 12345;
static double urand(void) {
  rng = orc_splitmix64(rng);
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
  /* a ragged 9 x 7 x 5 grid of random densities */
  const int nx = 9, ny = 7, nz = 5, W = 12, H = 10;
  float* rho = malloc(sizeof(float) * nx * ny * nz);
  for (int i = 0; i < nx * ny * nz; ++i) rho[i] = (float)(2.0 * urand());
  const double persp[16] = {1, 2.4, 0.6, 0.3, 0.5, 0.45, 0.5, 0.1, 1.0, 0.2, 50.0, 0.8, W, H, 0, 0};
  const double ortho[16] = {0, 0.45, -2.0, 0.7, 0.5, 0.5, 0.5, 0, 0, 1, 60.0, 0.8, W, H, 0, 0};
  const double w[3] = {1.0, 0.7, 0.4};
  double* guide = malloc(sizeof(double) * W * H * 3);
  double* margin = malloc(sizeof(double) * W * H);
  long long cnt[2];
  for (int cam = 0; cam < 2; ++cam)
    for (int quad = 0; quad < 2; ++quad)
      for (int set = 0; set < 2; ++set) {
        if (orc_march(rho, nx, ny, nz, 8.0, cam ? ortho : persp, 1.5, 0.1, 1e-6, 1, 7, 3, quad, w, set, 0, 1, guide,
                      margin, cnt)) {
          printf("FAIL orc_march\n");
          ++failures;
        }
        check_finite("orc_march guide", guide, W * H * 3);
      }
  double p[3] = {0.4, 0.55, 0.5};
  double s = orc_sigma_vol(rho, nx, ny, nz, 8.0, p);
  check_finite("orc_sigma_vol", &s, 1);
  double gap = orc_front_identity_gap(rho, nx, ny, nz, 8.0, persp, 1.0, 1, 5);
  check_finite("orc_front_identity_gap", &gap, 1);
  double j = orc_jitter(3, 4, 5);
  check_finite("orc_jitter", &j, 1);
  double* lm = malloc(sizeof(double) * W * H * 6);
  if (orc_reference_lightmaps(rho, nx, ny, nz, 8.0, persp, 0.5, 1e-6, lm)) ++failures;
  check_finite("orc_reference_lightmaps", lm, W * H * 6);

  /* shading and shadows */
  const double lights[12] = {0.3, 1.0, -0.2, 1.0, 0.9, 0.8, -1.0, 0.2, 0.4, 0.2, 0.3, 0.4};
  double* rgba = malloc(sizeof(double) * W * H * 4);
  if (orc_composite(H, W, lm, guide, persp, lights, 2, rgba)) ++failures;
  check_finite("orc_composite", rgba, W * H * 4);
  const int S = 16;
  const double origin[3] = {0.5, 0.5, 0.5}, centre[3] = {0.5, 0.45, 0.5};
  double* depth = malloc(sizeof(double) * S * S);
  orc_shadow_map_sphere(S, 0.9, origin, lights, centre, 0.15, depth);
  double* vis = malloc(sizeof(double) * 2 * W * H);
  double* vmargin = malloc(sizeof(double) * W * H);
  orc_shadow_visibility(H, W, guide, persp, lights, S, 0.9, origin, depth, 0.01, vis, vmargin);
  orc_shadow_visibility(H, W, guide, persp, lights + 6, S, 0.9, origin, depth, 0.01, vis + W * H, vmargin);
  check_finite("orc_shadow_visibility", vis, 2 * W * H);
  if (orc_composite_shadowed(H, W, lm, guide, persp, lights, 2, vis, rgba)) ++failures;
  check_finite("orc_composite_shadowed", rgba, W * H * 4);

  /* network: 3 levels of base 16 on a 2 x 12 x 8 batch (ragged width) */
  const int L = 3, base = 16, B = 2, h = 12, wd = 8;
  const long np = orc_unet_param_count(L, base);
  float* prm = malloc(sizeof(float) * np);
  for (long i = 0; i < np; ++i) prm[i] = (float)(0.2 * (urand() - 0.5));
  double* g = malloc(sizeof(double) * B * h * wd * 3);
  for (int i = 0; i < B * h * wd * 3; ++i) g[i] = urand();
  double* out = malloc(sizeof(double) * B * h * wd * 6);
  double* logits = malloc(sizeof(double) * B * h * wd * 6);
  if (orc_unet_forward(L, base, prm, np, B, h, wd, g, out, logits)) ++failures;
  check_finite("orc_unet_forward", out, B * h * wd * 6);
  double loss, *grad = malloc(sizeof(double) * np);
  if (orc_unet_loss_grad(L, base, prm, np, B, h, wd, g, out, &loss, grad)) ++failures;
  check_finite("orc_unet_loss_grad", grad, np);
  double* feat = malloc(sizeof(double) * B * h * wd * base);
  if (orc_unet_features(L, base, prm, np, B, h, wd, g, feat)) ++failures;
  check_finite("orc_unet_features", feat, B * h * wd * base);
  const long na = orc_adapter_param_count(base);
  float* ap = malloc(sizeof(float) * na);
  for (long i = 0; i < na; ++i) ap[i] = (float)(0.2 * (urand() - 0.5));
  double* extra = malloc(sizeof(double) * B * h * wd * 2);
  if (orc_adapters_forward(base, ap, na, B, h, wd, feat, out, extra)) ++failures;
  check_finite("orc_adapters_forward", out, B * h * wd * 6);
  double* gad = malloc(sizeof(double) * na);
  double* tgt = malloc(sizeof(double) * B * h * wd * 6);
  for (int i = 0; i < B * h * wd * 6; ++i) tgt[i] = urand();
  if (orc_adapters_loss_grad(L, base, prm, np, ap, na, B, h, wd, g, tgt, &loss, grad, gad)) ++failures;
  check_finite("orc_adapters_loss_grad trunk", grad, np);
  check_finite("orc_adapters_loss_grad adapters", gad, na);
  double* pd = malloc(sizeof(double) * np);
  double* m = calloc(np, sizeof(double));
  double* v = calloc(np, sizeof(double));
  for (long i = 0; i < np; ++i) pd[i] = prm[i];
  orc_adam(np, pd, grad, m, v, 1, 1e-3, 0.9, 0.999, 1e-8);
  check_finite("orc_adam", pd, np);

  free(rho), free(guide), free(margin), free(lm), free(rgba), free(depth), free(vis), free(vmargin), free(prm);
  free(g), free(out), free(logits), free(grad), free(feat), free(ap), free(extra), free(pd), free(m), free(v);
  free(gad), free(tgt);
  printf("oracle under sanitizers: %d failures\n", failures);
  return failures ? 1 : 0;
}
