/*
 * FP64 CPU oracle of the neural six-way lightmaps hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two meet
 * only through the seeded inputs of the `synth` package.
 *
 * Everything is plain fp64 loops in the order the paper states the method:
 *   - zero-border, cell-centred trilinear sampling of the density grid
 *     (the paper's "3D texture", Section 4.2);
 *   - camera rays, the three surrogate guiding lights front = w,
 *     top = w x z, bottom = -w x z (Section 4.2, Eq. approx), or the
 *     left/right pair of the guiding-light ablation (Section 5);
 *   - the coarse-step guiding-map march of Algorithm 1 producing
 *     (L~_scattering, T, D) per pixel, with per-ray jitter;
 *   - fine-step six-way reference lightmaps (training targets standing in for
 *     the paper's offline single-scatter references, Section 5);
 *   - the U-Net forward and backward passes (Section 4.3), the pixel MSE in
 *     sRGB space (Section 4.4) and Adam (Section 5, "Training");
 *   - the four NAFBlock channel adapters on the decoder output (Section 4.3);
 *   - the six-way directional interpolation used for shading (Section 3),
 *     and the depth-based obstacle shadowing (Section 4.5).
 *
 * Readings of silent or garbled passages (all listed in the design notes):
 *   - A_n: Algorithm 1 writes T_{n-1} sigma_s with no step length.  The default
 *     quadrature takes A_n = T_{n-1} (1 - exp(-sigma_n h)) ("alpha"), which is
 *     the exact integral for piecewise-constant sigma; quadrature 1 takes the
 *     literal Riemann term T_{n-1} sigma_n h.
 *   - c_0 <- 1 is read as T_0 = 1; "A^. L^. P^." as the light transmittance T^.
 *   - jitter is one offset per ray: samples at t_n = (n + u) h, n >= 1.
 *   - sigma_t = sigma_s (albedo 1), isotropic phase (4 pi P = 1), unit light
 *     intensities scaled by the caller's weights (w_front, w_top, w_bottom).
 *   - early ray termination (not in the paper): the primary march stops after a
 *     sample whose transmittance falls below eps_T and reports T = 0; a
 *     secondary march stops once its optical depth exceeds -ln eps_T and
 *     reports 0.  eps_T = 0 disables both.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ hash */
/* SplitMix64 finaliser (Steele, Lea and Flood 2014; Vigna's reference
 * splitmix64.c): the output for state s is mix(s + 0x9E3779B97F4A7C15). */
ORC_EXPORT uint64_t orc_splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Per-ray jitter u in [0, 1): 24 random bits, exact in fp32 and fp64. */
ORC_EXPORT double orc_jitter(uint64_t seed, uint32_t frame, uint32_t pixel) {
  uint64_t key = seed ^ ((uint64_t)frame << 32) ^ (uint64_t)pixel;
  return (double)(orc_splitmix64(key) >> 40) * (1.0 / 16777216.0);
}

/* ---------------------------------------------------------------- vectors */
static void v_sub(const double* a, const double* b, double* o) { for (int i = 0; i < 3; ++i) o[i] = a[i] - b[i]; }
static double v_dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void v_cross(const double* a, const double* b, double* o) {
  double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
static double v_norm(const double* a) { return sqrt(v_dot(a, a)); }
static void v_normalize(double* a) { double n = v_norm(a); a[0] /= n; a[1] /= n; a[2] /= n; }

/* ----------------------------------------------------------------- volume */
typedef struct {
  const float* rho; /* [nz][ny][nx], x fastest */
  int nx, ny, nz;
  double sigma_scale;
} Vol;

static double rho_at(const Vol* v, long i, long j, long k) {
  if (i < 0 || j < 0 || k < 0 || i >= v->nx || j >= v->ny || k >= v->nz) return 0.0;
  return (double)v->rho[((size_t)k * v->ny + (size_t)j) * v->nx + (size_t)i];
}

/* sigma(p) = sigma_scale * trilinear interpolation of the voxel-centred grid,
 * reading 0 outside it; continuous, and 0 on and outside the support box
 * [-dx/2, 1 + dx/2] per axis. */
ORC_EXPORT double orc_sigma_vol(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* p);
static double sample_sigma(const Vol* v, const double* p) {
  double g[3] = {p[0] * v->nx - 0.5, p[1] * v->ny - 0.5, p[2] * v->nz - 0.5};
  if (g[0] <= -1.0 || g[1] <= -1.0 || g[2] <= -1.0 || g[0] >= v->nx || g[1] >= v->ny || g[2] >= v->nz) return 0.0;
  double f0 = floor(g[0]), f1 = floor(g[1]), f2 = floor(g[2]);
  long i = (long)f0, j = (long)f1, k = (long)f2;
  double fx = g[0] - f0, fy = g[1] - f1, fz = g[2] - f2;
  double s = 0.0;
  for (int dk = 0; dk < 2; ++dk)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        double w = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
        s += w * rho_at(v, i + di, j + dj, k + dk);
      }
  return v->sigma_scale * s;
}
double orc_sigma_vol(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* p) {
  Vol v = {rho, nx, ny, nz, sigma_scale};
  return sample_sigma(&v, p);
}

/* Parametric interval [t0, t1] (t >= 0) of o + t d inside the support box. */
static int clip_support(const Vol* v, const double* o, const double* d, double* t0, double* t1) {
  int n[3] = {v->nx, v->ny, v->nz};
  double lo = 0.0, hi = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double bmin = -0.5 / n[a], bmax = 1.0 + 0.5 / n[a];
    if (d[a] == 0.0) {
      if (o[a] < bmin || o[a] > bmax) return 0;
      continue;
    }
    double ta = (bmin - o[a]) / d[a], tb = (bmax - o[a]) / d[a];
    if (ta > tb) { double t = ta; ta = tb; tb = t; }
    if (ta > lo) lo = ta;
    if (tb < hi) hi = tb;
  }
  if (hi < lo) return 0;
  *t0 = lo; *t1 = hi;
  return 1;
}

/* ----------------------------------------------------------------- camera */
/* cam[16] = {projection, eye xyz, target xyz, up xyz, fov_y_deg,
 *            ortho_half_extent, width, height, (unused) x2}
 * projection 0 = orthographic, 1 = perspective. */
typedef struct {
  int proj, W, H;
  double eye[3], f[3], r[3], u[3];
  double tan_half, half_extent;
} Cam;

static void cam_setup(const double* c, Cam* k) {
  k->proj = (int)c[0];
  double eye[3] = {c[1], c[2], c[3]}, tgt[3] = {c[4], c[5], c[6]}, up[3] = {c[7], c[8], c[9]};
  memcpy(k->eye, eye, sizeof eye);
  v_sub(tgt, eye, k->f); v_normalize(k->f);
  v_cross(k->f, up, k->r); v_normalize(k->r);
  v_cross(k->r, k->f, k->u);
  k->tan_half = tan(0.5 * c[10] * M_PI / 180.0);
  k->half_extent = c[11];
  k->W = (int)c[12]; k->H = (int)c[13];
}

/* Ray through the centre of pixel (i, j); row j = 0 is the top of the image. */
static void cam_ray(const Cam* k, int i, int j, double* o, double* d) {
  double sx = 2.0 * (i + 0.5) / k->W - 1.0, sy = 1.0 - 2.0 * (j + 0.5) / k->H;
  double aspect = (double)k->W / k->H;
  if (k->proj == 1) {
    for (int a = 0; a < 3; ++a) {
      o[a] = k->eye[a];
      d[a] = k->f[a] + k->tan_half * (sx * aspect * k->r[a] + sy * k->u[a]);
    }
    v_normalize(d);
  } else {
    for (int a = 0; a < 3; ++a) {
      o[a] = k->eye[a] + k->half_extent * (sx * aspect * k->r[a] + sy * k->u[a]);
      d[a] = k->f[a];
    }
  }
}

/* Surrogate side-light direction top = normalize(w x z_world), bottom = -top.
 * If w is (anti)parallel to z the limit direction normalize(w x x_world) is
 * used. */
static void top_light(const double* w, double* top) {
  double z[3] = {0, 0, 1}, x[3] = {1, 0, 0};
  v_cross(w, z, top);
  if (v_norm(top) < 1e-6) v_cross(w, x, top);
  v_normalize(top);
}

/* The ablation's alternative side lights (Section 5, guiding light
 * directions): left = normalize(w x top), right = -left, i.e. the two
 * directions perpendicular to both the view and the top/bottom pair. */
static void left_light(const double* w, double* left) {
  double top[3];
  top_light(w, top);
  v_cross(w, top, left);
  v_normalize(left);
}

/* Transmittance from x toward unit direction l through the support box:
 * exp(-h sum_{k>=1} sigma(x + k h l)) over the in-box points, or 0 once the
 * partial optical depth exceeds tau_max. */
static double light_transmittance(const Vol* v, const double* x, const double* l, double h, double tau_max,
                                  long long* nsamp) {
  double s0, s1;
  if (!clip_support(v, x, l, &s0, &s1)) return 1.0;
  long kmax = (long)floor(s1 / h);
  double tau = 0.0;
  for (long k = 1; k <= kmax; ++k) {
    double p[3] = {x[0] + k * h * l[0], x[1] + k * h * l[1], x[2] + k * h * l[2]};
    tau += h * sample_sigma(v, p);
    ++*nsamp;
    if (tau > tau_max) return 0.0;
  }
  return exp(-tau);
}

/* ------------------------------------------------------------------ march */
/*
 * Guiding map (Algorithm 1).  guide[H][W][3] = (L~_scattering, T, D).
 * d_margin[H][W] (optional): min |sigma_n - tau_D| over the samples that took
 * part in the depth decision, so a comparison can exempt pixels whose D sits
 * on the threshold.
 * counters[2] (optional): primary and secondary sample counts.
 * unit_radiance != 0 replaces L_n by 1 (diagnostic for the identity
 * sum A_n = 1 - T).
 * stride > 1 computes only pixels whose row and column are multiples of it
 * (the others are left untouched), for spot checks of large images.
 * light_set 0 uses the (top, bottom) side lights, 1 the (left, right) pair;
 * light_w weighs (front, first side, second side).
 */
ORC_EXPORT int orc_march(const float* rho, int nx, int ny, int nz, double sigma_scale, const double* cam,
                         double step_voxels, double depth_tau, double ert_eps, int jitter_on, uint64_t jitter_seed,
                         uint32_t frame, int quadrature, const double* light_w, int light_set, int unit_radiance,
                         int stride, double* guide, double* d_margin, long long* counters) {
  if (!rho || !cam || !guide || nx < 1 || ny < 1 || nz < 1 || step_voxels <= 0.0 || ert_eps < 0.0 || stride < 1 ||
      light_set < 0 || light_set > 1)
    return 1;
  Vol v = {rho, nx, ny, nz, sigma_scale};
  Cam k;
  cam_setup(cam, &k);
  int nmax = nx > ny ? nx : ny;
  if (nz > nmax) nmax = nz;
  const double h = step_voxels / nmax;
  const double tau_max = ert_eps > 0.0 ? -log(ert_eps) : INFINITY;
  long long c_primary = 0, c_secondary = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : c_primary, c_secondary)
  for (int j = 0; j < k.H; j += stride) {
    for (int i = 0; i < k.W; i += stride) {
      double o[3], d[3], w[3], top[3], bot[3];
      cam_ray(&k, i, j, o, d);
      for (int a = 0; a < 3; ++a) w[a] = -d[a];
      if (light_set == 1)
        left_light(w, top); /* the side pair is then (left, right) */
      else
        top_light(w, top);
      for (int a = 0; a < 3; ++a) bot[a] = -top[a];
      uint32_t pix = (uint32_t)j * (uint32_t)k.W + (uint32_t)i;
      double u = jitter_on ? orc_jitter(jitter_seed, frame, pix) : 0.0;
      double Ls = 0.0, tau = 0.0, T_prev = 1.0, T_out = 1.0, D = 0.0, margin = INFINITY;
      double t0, t1;
      if (clip_support(&v, o, d, &t0, &t1)) {
        long n0 = (long)ceil(t0 / h - u), n1 = (long)floor(t1 / h - u);
        if (n0 < 1) n0 = 1;
        for (long n = n0; n <= n1; ++n) {
          double t = (n + u) * h;
          double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
          double sig = sample_sigma(&v, x);
          ++c_primary;
          if (D == 0.0) {
            double m = fabs(sig - depth_tau);
            if (m < margin) margin = m;
            if (sig > depth_tau) D = n * h;
          }
          tau += sig * h;
          double T = exp(-tau);
          double A = quadrature == 1 ? T_prev * sig * h : T_prev - T;
          double L;
          if (unit_radiance) {
            L = 1.0;
          } else {
            long long ns = 0;
            double Tt = light_w[1] != 0.0 ? light_transmittance(&v, x, top, h, tau_max, &ns) : 0.0;
            double Tb = light_w[2] != 0.0 ? light_transmittance(&v, x, bot, h, tau_max, &ns) : 0.0;
            c_secondary += ns;
            /* front light: the march toward w retraces the primary samples
             * before x_n, so its transmittance is T_{n-1}. */
            L = light_w[0] * T_prev + light_w[1] * Tt + light_w[2] * Tb;
          }
          Ls += A * L;
          T_prev = T;
          T_out = T;
          if (tau > tau_max) { T_out = 0.0; break; }
        }
      }
      double* g = guide + 3 * (size_t)pix;
      g[0] = Ls; g[1] = T_out; g[2] = D;
      if (d_margin) d_margin[pix] = margin;
    }
  }
  if (counters) { counters[0] = c_primary; counters[1] = c_secondary; }
  return 0;
}

/* Front-light transmittance by an explicit march toward w (debug form of the
 * T^front = T_{n-1} identity); returns the largest |difference| over the image. */
ORC_EXPORT double orc_front_identity_gap(const float* rho, int nx, int ny, int nz, double sigma_scale,
                                         const double* cam, double step_voxels, int jitter_on, uint64_t seed) {
  Vol v = {rho, nx, ny, nz, sigma_scale};
  Cam k;
  cam_setup(cam, &k);
  int nmax = nx > ny ? nx : ny;
  if (nz > nmax) nmax = nz;
  const double h = step_voxels / nmax;
  double worst = 0.0;
  for (int j = 0; j < k.H; ++j)
    for (int i = 0; i < k.W; ++i) {
      double o[3], d[3], w[3];
      cam_ray(&k, i, j, o, d);
      for (int a = 0; a < 3; ++a) w[a] = -d[a];
      uint32_t pix = (uint32_t)j * (uint32_t)k.W + (uint32_t)i;
      double u = jitter_on ? orc_jitter(seed, 0, pix) : 0.0, t0, t1, tau = 0.0;
      if (!clip_support(&v, o, d, &t0, &t1)) continue;
      long n0 = (long)ceil(t0 / h - u), n1 = (long)floor(t1 / h - u);
      if (n0 < 1) n0 = 1;
      for (long n = n0; n <= n1; ++n) {
        double t = (n + u) * h;
        double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        long long ns = 0;
        double Tf = light_transmittance(&v, x, w, h, INFINITY, &ns);
        double gap = fabs(Tf - exp(-tau));
        if (gap > worst) worst = gap;
        tau += h * sample_sigma(&v, x);
      }
    }
  return worst;
}

/* ------------------------------------------------------ reference lightmaps */
/*
 * Six-way reference lightmaps lm[H][W][6], order (+X, -X, +Y, -Y, +Z, -Z) of
 * the camera frame X = right, Y = up, Z = toward the camera (= -forward).
 * L_a = sum_n A_n T^a_n with the alpha quadrature, no jitter, step
 * step_voxels (fine), and T^a_n the transmittance from x_n toward axis a.
 */
ORC_EXPORT int orc_reference_lightmaps(const float* rho, int nx, int ny, int nz, double sigma_scale,
                                       const double* cam, double step_voxels, double ert_eps, double* lm) {
  if (!rho || !cam || !lm || step_voxels <= 0.0) return 1;
  Vol v = {rho, nx, ny, nz, sigma_scale};
  Cam k;
  cam_setup(cam, &k);
  int nmax = nx > ny ? nx : ny;
  if (nz > nmax) nmax = nz;
  const double h = step_voxels / nmax;
  const double tau_max = ert_eps > 0.0 ? -log(ert_eps) : INFINITY;
  double axes[6][3];
  for (int a = 0; a < 3; ++a) {
    axes[0][a] = k.r[a]; axes[1][a] = -k.r[a];
    axes[2][a] = k.u[a]; axes[3][a] = -k.u[a];
    axes[4][a] = -k.f[a]; axes[5][a] = k.f[a];
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < k.H; ++j) {
    for (int i = 0; i < k.W; ++i) {
      double o[3], d[3], acc[6] = {0, 0, 0, 0, 0, 0}, t0, t1, tau = 0.0, T_prev = 1.0;
      cam_ray(&k, i, j, o, d);
      if (clip_support(&v, o, d, &t0, &t1)) {
        long n0 = (long)ceil(t0 / h), n1 = (long)floor(t1 / h);
        if (n0 < 1) n0 = 1;
        for (long n = n0; n <= n1; ++n) {
          double t = n * h;
          double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
          double sig = sample_sigma(&v, x);
          tau += sig * h;
          double T = exp(-tau), A = T_prev - T;
          if (A > 0.0) {
            for (int a = 0; a < 6; ++a) {
              long long ns = 0;
              acc[a] += A * light_transmittance(&v, x, axes[a], h, tau_max, &ns);
            }
          }
          T_prev = T;
          if (tau > tau_max) break;
        }
      }
      double* out = lm + 6 * ((size_t)j * k.W + i);
      for (int a = 0; a < 6; ++a) out[a] = acc[a];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------- sRGB */
/* IEC 61966-2-1 transfer curve. */
ORC_EXPORT double orc_srgb_encode(double c) {
  return c <= 0.0031308 ? 12.92 * c : 1.055 * pow(c, 1.0 / 2.4) - 0.055;
}
ORC_EXPORT double orc_srgb_decode(double s) {
  return s <= 0.04045 ? s / 12.92 : pow((s + 0.055) / 1.055, 2.4);
}

/* -------------------------------------------------------------- composite */
/*
 * Shading from six-way lightmaps (Section 3): for each light with direction
 * l (world, toward the light) and colour c, rgb += c * sum_p |l_p| lin(L_p^{sign l_p})
 * where l_p are the components of l in the camera frame (right, up, toward
 * camera), lin decodes the network's sRGB output, and alpha = 1 - T.
 * lights[n][6] = (dir xyz, rgb).  rgba[H][W][4].
 */
ORC_EXPORT int orc_composite(int H, int W, const double* lm, const double* guide, const double* cam,
                             const double* lights, int n_lights, double* rgba) {
  Cam k;
  cam_setup(cam, &k);
  double lc[16][3];
  if (n_lights > 16) return 1;
  for (int q = 0; q < n_lights; ++q) {
    const double* l = lights + 6 * q;
    double z[3] = {-k.f[0], -k.f[1], -k.f[2]};
    lc[q][0] = v_dot(l, k.r); lc[q][1] = v_dot(l, k.u); lc[q][2] = v_dot(l, z);
  }
  for (long p = 0; p < (long)H * W; ++p) {
    const double* L = lm + 6 * p;
    double rgb[3] = {0, 0, 0};
    for (int q = 0; q < n_lights; ++q) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) {
        double comp = lc[q][a];
        double val = comp >= 0.0 ? L[2 * a] : L[2 * a + 1];
        s += fabs(comp) * orc_srgb_decode(val);
      }
      for (int c = 0; c < 3; ++c) rgb[c] += lights[6 * q + 3 + c] * s;
    }
    rgba[4 * p + 0] = rgb[0]; rgba[4 * p + 1] = rgb[1]; rgba[4 * p + 2] = rgb[2];
    rgba[4 * p + 3] = 1.0 - guide[3 * p + 1];
  }
  return 0;
}

/* ------------------------------------------------------- obstacle shadows */
/*
 * Depth-based screen-space obstacle shadowing (Section 4.5).  A directional
 * light with unit direction l (toward the light) gets an orthographic
 * light space: e1 = normalize(a x l) with a = y (x when |l . y| > 0.99),
 * e2 = l x e1, coordinates (u, v, z) = ((p - origin) . e1, . e2, . l).  Its
 * shadow map is an S x S grid over u, v in [-E, E] storing the largest z of
 * the obstacle along each texel centre's light ray (the occluder surface
 * nearest the light), -inf where the obstacle is absent.  A pixel's smoke
 * surface point P = o + D d (D from the guiding map; no surface when D = 0)
 * is shadowed when the texel containing (u, v) holds an occluder depth
 * greater than z(P) + bias.
 */
static void light_basis(const double* l, double* e1, double* e2) {
  double a[3] = {0, 1, 0};
  if (fabs(l[1]) > 0.99) { a[0] = 1; a[1] = 0; }
  v_cross(a, l, e1);
  v_normalize(e1);
  v_cross(l, e1, e2);
}

/* shadow map of a sphere (centre, radius): depth[j][i] over u (i) and v (j) */
ORC_EXPORT void orc_shadow_map_sphere(int S, double E, const double* origin, const double* light, const double* centre,
                                      double radius, double* depth) {
  double l[3] = {light[0], light[1], light[2]}, e1[3], e2[3], c[3];
  v_normalize(l);
  light_basis(l, e1, e2);
  v_sub(centre, origin, c);
  const double cu = v_dot(c, e1), cv = v_dot(c, e2), cz = v_dot(c, l);
  for (int j = 0; j < S; ++j)
    for (int i = 0; i < S; ++i) {
      const double u = -E + 2.0 * E * (i + 0.5) / S, v = -E + 2.0 * E * (j + 0.5) / S;
      const double q = radius * radius - (u - cu) * (u - cu) - (v - cv) * (v - cv);
      depth[(size_t)j * S + i] = q >= 0.0 ? cz + sqrt(q) : -INFINITY;
    }
}

/* visibility[H][W] in {0, 1} of each pixel's smoke surface for one light.
 * margin (optional, [H][W]) receives how far the decision is from flipping,
 * in world units: the smaller of the distance of (u, v) to the nearest texel
 * edge and |occluder depth - (z + bias)|; +inf where D = 0. */
ORC_EXPORT void orc_shadow_visibility(int H, int W, const double* guide, const double* cam, const double* light, int S,
                                      double E, const double* origin, const double* depth, double bias,
                                      double* vis, double* margin) {
  Cam k;
  cam_setup(cam, &k);
  double l[3] = {light[0], light[1], light[2]}, e1[3], e2[3];
  v_normalize(l);
  light_basis(l, e1, e2);
  const double texel = 2.0 * E / S;
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      const size_t p = (size_t)j * W + i;
      const double D = guide[3 * p + 2];
      double v = 1.0, mg = INFINITY;
      if (D > 0.0) {
        double o[3], d[3], P[3], q[3];
        cam_ray(&k, i, j, o, d);
        for (int a = 0; a < 3; ++a) P[a] = o[a] + D * d[a];
        v_sub(P, origin, q);
        const double u = v_dot(q, e1), w = v_dot(q, e2), z = v_dot(q, l);
        const double su = (u + E) / (2.0 * E) * S, sw = (w + E) / (2.0 * E) * S;
        const int ti = (int)floor(su), tj = (int)floor(sw);
        mg = fmin(fabs(su - nearbyint(su)), fabs(sw - nearbyint(sw))) * texel;
        if (ti >= 0 && ti < S && tj >= 0 && tj < S) {
          const double occ = depth[(size_t)tj * S + ti];
          if (occ > z + bias) v = 0.0;
          if (isfinite(occ)) mg = fmin(mg, fabs(occ - (z + bias)));
        }
      }
      vis[p] = v;
      if (margin) margin[p] = mg;
    }
}

/* Shading of orc_composite with each light's term multiplied by its
 * visibility (vis[n_lights][H][W]). */
ORC_EXPORT int orc_composite_shadowed(int H, int W, const double* lm, const double* guide, const double* cam,
                                      const double* lights, int n_lights, const double* vis, double* rgba) {
  if (n_lights > 16) return 1;
  for (int q = 0; q < n_lights; ++q) {
    double* one = malloc(sizeof(double) * (size_t)H * W * 4);
    orc_composite(H, W, lm, guide, cam, lights + 6 * q, 1, one);
    for (size_t p = 0; p < (size_t)H * W; ++p) {
      for (int c = 0; c < 3; ++c) rgba[4 * p + c] = (q ? rgba[4 * p + c] : 0.0) + vis[(size_t)q * H * W + p] * one[4 * p + c];
      rgba[4 * p + 3] = one[4 * p + 3];
    }
    free(one);
  }
  if (n_lights == 0) orc_composite(H, W, lm, guide, cam, lights, 0, rgba);
  return 0;
}

/* ------------------------------------------------------------------ U-Net */
/*
 * Tensors are NCHW fp64 here.  Convolution is cross-correlation with stride 1
 * and zero padding k/2: out[b,o,y,x] = bias[o] + sum_{c,dy,dx}
 * W[o,c,dy,dx] in[b,c,y+dy-k/2,x+dx-k/2].
 */
typedef struct {
  int ci, co, k;
  const float* w; /* [co][ci][k][k] */
  const float* b; /* [co] */
  long offset;    /* index of w in the flat parameter vector */
} Layer;

#define MAXL 64
typedef struct {
  int levels, base, n;
  Layer L[MAXL];
  long n_params;
} Net;

static int net_setup(int levels, int base, const float* params, long n_params, Net* net) {
  if (levels < 1 || base < 1 || 2 * (2 * levels - 1) + 1 > MAXL) return 1;
  int n = 0, cin = 3;
  long off = 0;
  int width[16];
  for (int l = 0; l < levels; ++l) width[l] = base << l;
#define ADD(CI, CO, K)                                                     \
  do {                                                                     \
    net->L[n].ci = (CI); net->L[n].co = (CO); net->L[n].k = (K);           \
    net->L[n].offset = off; net->L[n].w = params + off;                    \
    off += (long)(CO) * (CI) * (K) * (K);                                  \
    net->L[n].b = params + off; off += (CO); ++n;                          \
  } while (0)
  for (int l = 0; l < levels - 1; ++l) { ADD(cin, width[l], 3); ADD(width[l], width[l], 3); cin = width[l]; }
  ADD(cin, width[levels - 1], 3);
  ADD(width[levels - 1], width[levels - 1], 3);
  for (int l = levels - 2; l >= 0; --l) { ADD(width[l] + width[l + 1], width[l], 3); ADD(width[l], width[l], 3); }
  ADD(width[0], 6, 1);
#undef ADD
  net->levels = levels; net->base = base; net->n = n; net->n_params = off;
  if (n_params >= 0 && off != n_params) return 2;
  return 0;
}

ORC_EXPORT long orc_unet_param_count(int levels, int base) {
  Net net;
  if (net_setup(levels, base, NULL, -1, &net)) return -1;
  return net.n_params;
}

static void conv_fwd(const double* in, int B, int H, int W, const Layer* l, double* out) {
  const int ci = l->ci, co = l->co, k = l->k, p = k / 2;
#pragma omp parallel for collapse(2) schedule(static)
  for (int b = 0; b < B; ++b)
    for (int o = 0; o < co; ++o)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          double s = l->b[o];
          for (int c = 0; c < ci; ++c)
            for (int dy = 0; dy < k; ++dy) {
              int yy = y + dy - p;
              if (yy < 0 || yy >= H) continue;
              for (int dx = 0; dx < k; ++dx) {
                int xx = x + dx - p;
                if (xx < 0 || xx >= W) continue;
                s += (double)l->w[((o * ci + c) * k + dy) * k + dx] * in[(((size_t)b * ci + c) * H + yy) * W + xx];
              }
            }
          out[(((size_t)b * co + o) * H + y) * W + x] = s;
        }
}

/* dW, db accumulated into grad (flat, same layout as the params); din written
 * (not accumulated) when non-NULL. */
static void conv_bwd(const double* in, const double* dout, int B, int H, int W, const Layer* l, double* grad,
                     double* din) {
  const int ci = l->ci, co = l->co, k = l->k, p = k / 2;
  double* gw = grad + l->offset;
  double* gb = gw + (long)co * ci * k * k;
#pragma omp parallel for schedule(static)
  for (int o = 0; o < co; ++o) {
    double sb = 0.0;
    for (int b = 0; b < B; ++b)
      for (size_t q = 0; q < (size_t)H * W; ++q) sb += dout[((size_t)b * co + o) * H * W + q];
    gb[o] += sb;
    for (int c = 0; c < ci; ++c)
      for (int dy = 0; dy < k; ++dy)
        for (int dx = 0; dx < k; ++dx) {
          double s = 0.0;
          for (int b = 0; b < B; ++b)
            for (int y = 0; y < H; ++y) {
              int yy = y + dy - p;
              if (yy < 0 || yy >= H) continue;
              for (int x = 0; x < W; ++x) {
                int xx = x + dx - p;
                if (xx < 0 || xx >= W) continue;
                s += dout[(((size_t)b * co + o) * H + y) * W + x] * in[(((size_t)b * ci + c) * H + yy) * W + xx];
              }
            }
          gw[((o * ci + c) * k + dy) * k + dx] += s;
        }
  }
  if (!din) return;
#pragma omp parallel for collapse(2) schedule(static)
  for (int b = 0; b < B; ++b)
    for (int c = 0; c < ci; ++c)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          double s = 0.0;
          for (int o = 0; o < co; ++o)
            for (int dy = 0; dy < k; ++dy) {
              int yy = y - dy + p;
              if (yy < 0 || yy >= H) continue;
              for (int dx = 0; dx < k; ++dx) {
                int xx = x - dx + p;
                if (xx < 0 || xx >= W) continue;
                s += (double)l->w[((o * ci + c) * k + dy) * k + dx] * dout[(((size_t)b * co + o) * H + yy) * W + xx];
              }
            }
          din[(((size_t)b * ci + c) * H + y) * W + x] = s;
        }
}

static void relu_inplace(double* a, size_t n) { for (size_t i = 0; i < n; ++i) if (a[i] < 0.0) a[i] = 0.0; }

static void maxpool2(const double* in, int BC, int H, int W, double* out) {
  int Ho = H / 2, Wo = W / 2;
  for (long q = 0; q < BC; ++q)
    for (int y = 0; y < Ho; ++y)
      for (int x = 0; x < Wo; ++x) {
        const double* s = in + (size_t)q * H * W;
        double m = s[(2 * y) * W + 2 * x];
        if (s[(2 * y) * W + 2 * x + 1] > m) m = s[(2 * y) * W + 2 * x + 1];
        if (s[(2 * y + 1) * W + 2 * x] > m) m = s[(2 * y + 1) * W + 2 * x];
        if (s[(2 * y + 1) * W + 2 * x + 1] > m) m = s[(2 * y + 1) * W + 2 * x + 1];
        out[((size_t)q * Ho + y) * Wo + x] = m;
      }
}

/* The gradient of each 2x2 window goes to its first maximum in raster order. */
static void maxpool2_bwd(const double* in, const double* dout, int BC, int H, int W, double* din) {
  int Ho = H / 2, Wo = W / 2;
  memset(din, 0, sizeof(double) * (size_t)BC * H * W);
  for (long q = 0; q < BC; ++q)
    for (int y = 0; y < Ho; ++y)
      for (int x = 0; x < Wo; ++x) {
        const double* s = in + (size_t)q * H * W;
        size_t idx[4] = {(size_t)(2 * y) * W + 2 * x, (size_t)(2 * y) * W + 2 * x + 1, (size_t)(2 * y + 1) * W + 2 * x,
                         (size_t)(2 * y + 1) * W + 2 * x + 1};
        int best = 0;
        for (int t = 1; t < 4; ++t) if (s[idx[t]] > s[idx[best]]) best = t;
        din[(size_t)q * H * W + idx[best]] += dout[((size_t)q * Ho + y) * Wo + x];
      }
}

/* Nearest-neighbour 2x upsampling of [B][C][h][w] written into channels
 * [c_off, c_off + C) of a [B][Ctot][2h][2w] tensor. */
static void upsample2_into(const double* in, int B, int C, int h, int w, double* out, int Ctot, int c_off) {
  for (int b = 0; b < B; ++b)
    for (int c = 0; c < C; ++c)
      for (int y = 0; y < 2 * h; ++y)
        for (int x = 0; x < 2 * w; ++x)
          out[(((size_t)b * Ctot + c_off + c) * 2 * h + y) * 2 * w + x] = in[(((size_t)b * C + c) * h + y / 2) * w + x / 2];
}

static void copy_channels_into(const double* in, int B, int C, int H, int W, double* out, int Ctot, int c_off) {
  for (int b = 0; b < B; ++b)
    memcpy(out + ((size_t)b * Ctot + c_off) * H * W, in + (size_t)b * C * H * W, sizeof(double) * (size_t)C * H * W);
}

/* Saved forward state: the input and the post-ReLU output of every conv, and
 * the pooled tensors. */
typedef struct {
  double* x_in[MAXL];  /* input of conv layer i (NCHW) */
  double* y_out[MAXL]; /* output of conv layer i (after ReLU; logits for the head) */
  int hh[MAXL], ww[MAXL];
  double* pred; /* sigmoid output, NCHW */
} Fwd;

static void fwd_free(Fwd* f, int n) {
  for (int i = 0; i < n; ++i) { free(f->x_in[i]); free(f->y_out[i]); }
  free(f->pred);
}

static void unet_forward_saved(const Net* net, int B, int H, int W, const double* guide_nhwc, Fwd* f) {
  memset(f, 0, sizeof *f);
  const int L = net->levels;
  int li = 0, h = H, w = W;
  double* x = malloc(sizeof(double) * (size_t)B * 3 * H * W);
  for (int b = 0; b < B; ++b)
    for (int c = 0; c < 3; ++c)
      for (size_t q = 0; q < (size_t)H * W; ++q) x[((size_t)b * 3 + c) * H * W + q] = guide_nhwc[((size_t)b * H * W + q) * 3 + c];
  int skip_layer[16];
  /* encoder and bottleneck */
  for (int l = 0; l < L; ++l) {
    for (int rep = 0; rep < 2; ++rep) {
      const Layer* ly = &net->L[li];
      f->x_in[li] = x; f->hh[li] = h; f->ww[li] = w;
      double* y = malloc(sizeof(double) * (size_t)B * ly->co * h * w);
      conv_fwd(x, B, h, w, ly, y);
      relu_inplace(y, (size_t)B * ly->co * h * w);
      f->y_out[li] = y;
      x = malloc(sizeof(double) * (size_t)B * ly->co * h * w);
      memcpy(x, y, sizeof(double) * (size_t)B * ly->co * h * w);
      ++li;
    }
    if (l < L - 1) {
      skip_layer[l] = li - 1;
      double* pooled = malloc(sizeof(double) * (size_t)B * net->L[li - 1].co * (h / 2) * (w / 2));
      maxpool2(x, B * net->L[li - 1].co, h, w, pooled);
      free(x);
      x = pooled;
      h /= 2; w /= 2;
    }
  }
  /* decoder */
  for (int l = L - 2; l >= 0; --l) {
    const Layer* sk = &net->L[skip_layer[l]];
    int cs = sk->co, cu = net->L[li - 1].co, ct = cs + cu;
    double* cat = malloc(sizeof(double) * (size_t)B * ct * (2 * h) * (2 * w));
    copy_channels_into(f->y_out[skip_layer[l]], B, cs, 2 * h, 2 * w, cat, ct, 0);
    upsample2_into(x, B, cu, h, w, cat, ct, cs);
    free(x);
    x = cat;
    h *= 2; w *= 2;
    for (int rep = 0; rep < 2; ++rep) {
      const Layer* ly = &net->L[li];
      f->x_in[li] = x; f->hh[li] = h; f->ww[li] = w;
      double* y = malloc(sizeof(double) * (size_t)B * ly->co * h * w);
      conv_fwd(x, B, h, w, ly, y);
      relu_inplace(y, (size_t)B * ly->co * h * w);
      f->y_out[li] = y;
      x = malloc(sizeof(double) * (size_t)B * ly->co * h * w);
      memcpy(x, y, sizeof(double) * (size_t)B * ly->co * h * w);
      ++li;
    }
  }
  /* head: 1x1 conv to 6 logits, sigmoid */
  const Layer* hd = &net->L[li];
  f->x_in[li] = x; f->hh[li] = h; f->ww[li] = w;
  double* z = malloc(sizeof(double) * (size_t)B * 6 * h * w);
  conv_fwd(x, B, h, w, hd, z);
  f->y_out[li] = z;
  f->pred = malloc(sizeof(double) * (size_t)B * 6 * h * w);
  for (size_t q = 0; q < (size_t)B * 6 * h * w; ++q) f->pred[q] = 1.0 / (1.0 + exp(-z[q]));
}

static void nchw_to_nhwc(const double* in, int B, int C, int H, int W, double* out) {
  for (int b = 0; b < B; ++b)
    for (int c = 0; c < C; ++c)
      for (size_t q = 0; q < (size_t)H * W; ++q) out[((size_t)b * H * W + q) * C + c] = in[((size_t)b * C + c) * H * W + q];
}

/* Forward pass: guide[B][H][W][3] -> lightmaps[B][H][W][6] (sigmoid output);
 * logits (pre-sigmoid, same layout) if non-NULL.  H, W divisible by
 * 2^(levels-1). */
ORC_EXPORT int orc_unet_forward(int levels, int base, const float* params, long n_params, int B, int H, int W,
                                const double* guide, double* lightmaps, double* logits) {
  Net net;
  int st = net_setup(levels, base, params, n_params, &net);
  if (st) return st;
  int div = 1 << (levels - 1);
  if (B < 1 || H < 1 || W < 1 || H % div || W % div) return 3;
  Fwd f;
  unet_forward_saved(&net, B, H, W, guide, &f);
  nchw_to_nhwc(f.pred, B, 6, H, W, lightmaps);
  if (logits) nchw_to_nhwc(f.y_out[net.n - 1], B, 6, H, W, logits);
  fwd_free(&f, net.n);
  return 0;
}

/* Backward through the trunk (every layer but the head), from g, the
 * gradient with respect to the head's input (the last decoder layer's
 * output, NCHW; freed here), adding each layer's parameter gradient to grad. */
static void trunk_backward(const Net* net_p, const Fwd* fp, int B, double* g, double* grad) {
  const Net net = *net_p;
  const Fwd f = *fp;
  const int L = net.levels;
  int li = net.n - 2;
  /* gradient flowing into each encoder skip from the decoder concat */
  double* skip_grad[16] = {0};
  int skip_layer[16];
  {
    int q = 0;
    for (int lv = 0; lv < L - 1; ++lv) { q += 2; skip_layer[lv] = q - 1; }
  }
  /* decoder, level 0 upward */
  for (int lv = 0; lv <= L - 2; ++lv) {
    int h = f.hh[li], w = f.ww[li];
    for (int rep = 0; rep < 2; ++rep) {
      const Layer* ly = &net.L[li];
      /* ReLU: gradient passes where the output is positive */
      const double* y = f.y_out[li];
      for (size_t q = 0; q < (size_t)B * ly->co * h * w; ++q) if (!(y[q] > 0.0)) g[q] = 0.0;
      double* gi = malloc(sizeof(double) * (size_t)B * ly->ci * h * w);
      conv_bwd(f.x_in[li], g, B, h, w, ly, grad, gi);
      free(g);
      g = gi;
      --li;
    }
    /* g is the gradient of concat(skip, up): split */
    int cs = net.L[skip_layer[lv]].co, ct = net.L[li + 1].ci, cu = ct - cs;
    skip_grad[lv] = malloc(sizeof(double) * (size_t)B * cs * h * w);
    double* gu = calloc((size_t)B * cu * (h / 2) * (w / 2), sizeof(double));
    for (int b = 0; b < B; ++b) {
      memcpy(skip_grad[lv] + (size_t)b * cs * h * w, g + (size_t)b * ct * h * w, sizeof(double) * (size_t)cs * h * w);
      for (int c = 0; c < cu; ++c)
        for (int y = 0; y < h; ++y)
          for (int x = 0; x < w; ++x)
            gu[(((size_t)b * cu + c) * (h / 2) + y / 2) * (w / 2) + x / 2] += g[(((size_t)b * ct + cs + c) * h + y) * w + x];
    }
    free(g);
    g = gu;
  }
  /* bottleneck and encoder, from the deepest level up */
  for (int lv = L - 1; lv >= 0; --lv) {
    int h = f.hh[li], w = f.ww[li];
    for (int rep = 0; rep < 2; ++rep) {
      const Layer* ly = &net.L[li];
      const double* y = f.y_out[li];
      for (size_t q = 0; q < (size_t)B * ly->co * h * w; ++q) if (!(y[q] > 0.0)) g[q] = 0.0;
      double* gi = li > 0 ? malloc(sizeof(double) * (size_t)B * ly->ci * h * w) : NULL;
      conv_bwd(f.x_in[li], g, B, h, w, ly, grad, gi);
      free(g);
      g = gi;
      --li;
    }
    if (lv > 0) {
      /* g: gradient of the pooled output of level lv-1; route through the
       * max-pool and add the decoder's skip gradient */
      int sl = skip_layer[lv - 1], cs = net.L[sl].co, H2 = f.hh[sl], W2 = f.ww[sl];
      double* gs = malloc(sizeof(double) * (size_t)B * cs * H2 * W2);
      maxpool2_bwd(f.y_out[sl], g, B * cs, H2, W2, gs);
      for (size_t q = 0; q < (size_t)B * cs * H2 * W2; ++q) gs[q] += skip_grad[lv - 1][q];
      free(g);
      g = gs;
    }
  }
  free(g);
  for (int lv = 0; lv < L - 1; ++lv) free(skip_grad[lv]);
}

/* Loss (mean squared error over B*H*W*6 against target_srgb[B][H][W][6]) and
 * its gradient with respect to every parameter (grad[n_params], written). */
ORC_EXPORT int orc_unet_loss_grad(int levels, int base, const float* params, long n_params, int B, int H, int W,
                                  const double* guide, const double* target, double* loss, double* grad) {
  Net net;
  int st = net_setup(levels, base, params, n_params, &net);
  if (st) return st;
  int div = 1 << (levels - 1);
  if (B < 1 || H < 1 || W < 1 || H % div || W % div) return 3;
  Fwd f;
  unet_forward_saved(&net, B, H, W, guide, &f);
  const size_t npix = (size_t)B * H * W;
  const double inv = 1.0 / (double)(npix * 6);
  double* t = malloc(sizeof(double) * npix * 6);
  /* target to NCHW */
  for (int b = 0; b < B; ++b)
    for (int c = 0; c < 6; ++c)
      for (size_t q = 0; q < (size_t)H * W; ++q) t[((size_t)b * 6 + c) * H * W + q] = target[((size_t)b * H * W + q) * 6 + c];
  double l = 0.0;
  double* dz = malloc(sizeof(double) * npix * 6);
  for (size_t q = 0; q < npix * 6; ++q) {
    double e = f.pred[q] - t[q];
    l += e * e;
    dz[q] = 2.0 * e * inv * f.pred[q] * (1.0 - f.pred[q]);
  }
  *loss = l * inv;
  memset(grad, 0, sizeof(double) * (size_t)net.n_params);
  free(t);
  /* backward through the head, then the trunk */
  const int li = net.n - 1;
  double* g = malloc(sizeof(double) * npix * net.L[li].ci);
  conv_bwd(f.x_in[li], dz, B, f.hh[li], f.ww[li], &net.L[li], grad, g);
  free(dz);
  trunk_backward(&net, &f, B, g, grad);
  fwd_free(&f, net.n);
  return 0;
}

/* Decoder output features of the U-Net (the input of its head):
 * feat[B][H][W][base], after the last ReLU.  params as orc_unet_forward. */
ORC_EXPORT int orc_unet_features(int levels, int base, const float* params, long n_params, int B, int H, int W,
                                 const double* guide, double* feat) {
  Net net;
  int st = net_setup(levels, base, params, n_params, &net);
  if (st) return st;
  int div = 1 << (levels - 1);
  if (B < 1 || H < 1 || W < 1 || H % div || W % div) return 3;
  Fwd f;
  unet_forward_saved(&net, B, H, W, guide, &f);
  nchw_to_nhwc(f.x_in[net.n - 1], B, base, H, W, feat);
  fwd_free(&f, net.n);
  return 0;
}

/* ------------------------------------------------------- channel adapters */
/*
 * Four channel adapters on the decoder output (Section 4.3): one per output
 * group (front/back, left/right, up/down, alpha/emissive), each a NAFBlock
 * of width c followed by a 1x1 head to that group's two channels and a
 * sigmoid.  The NAFBlock is the published one (Chen et al. 2022, "Simple
 * Baselines for Image Restoration") with both expansion factors 2:
 *   x = LN1(in); x = conv1x1(c -> 2c); x = depthwise conv3x3 (2c, zero pad);
 *   x = x[:c] * x[c:] (simple gate); x = x * (W_sca mean_{H,W}(x) + b_sca)
 *   (simplified channel attention, mean over each image); x = conv1x1(c -> c);
 *   y = in + beta * x;
 *   x = LN2(y); x = conv1x1(c -> 2c); x = x[:c] * x[c:]; x = conv1x1(c -> c);
 *   out = y + gamma * x.
 * LN is a layer norm over the channels of each pixel (biased variance,
 * eps 1e-6) with per-channel weight and bias.
 * Parameters of one adapter, in order: ln1 w[c] b[c]; conv1 W[2c][c] b[2c];
 * dw W[2c][3][3] b[2c]; sca W[c][c] b[c]; conv3 W[c][c] b[c]; beta[c];
 * ln2 w[c] b[c]; conv4 W[2c][c] b[2c]; conv5 W[c][c] b[c]; gamma[c];
 * head W[2][c] b[2].  The four adapters follow each other in group order.
 * Outputs: group 0 -> lightmaps (+Z, -Z), 1 -> (+X, -X), 2 -> (+Y, -Y),
 * 3 -> (alpha, emissive).
 */
ORC_EXPORT long orc_adapter_param_count(int c) { return 4L * (7L * c * c + 35L * c + 2); }

static void layer_norm_pixel(const double* x, int c, const float* w, const float* b, double* out) {
  double mu = 0.0, var = 0.0;
  for (int i = 0; i < c; ++i) mu += x[i];
  mu /= c;
  for (int i = 0; i < c; ++i) var += (x[i] - mu) * (x[i] - mu);
  var /= c;
  const double r = 1.0 / sqrt(var + 1e-6);
  for (int i = 0; i < c; ++i) out[i] = (x[i] - mu) * r * w[i] + b[i];
}

/* out[o] = b[o] + sum_i W[o][i] x[i] */
static void dense(const double* x, int ci, int co, const float* W, const float* b, double* out) {
  for (int o = 0; o < co; ++o) {
    double s = b[o];
    for (int i = 0; i < ci; ++i) s += (double)W[(size_t)o * ci + i] * x[i];
    out[o] = s;
  }
}

/* One NAFBlock + head on feat[B][H][W][c] -> two sigmoid outputs [B][H][W][2]. */
static void adapter_forward(int c, const float* P, int B, int H, int W, const double* feat, double* out2) {
  const float *ln1w = P, *ln1b = ln1w + c, *c1w = ln1b + c, *c1b = c1w + 2 * c * c, *dww = c1b + 2 * c,
              *dwb = dww + 18 * c, *scaw = dwb + 2 * c, *scab = scaw + c * c, *c3w = scab + c, *c3b = c3w + c * c,
              *beta = c3b + c, *ln2w = beta + c, *ln2b = ln2w + c, *c4w = ln2b + c, *c4b = c4w + 2 * c * c,
              *c5w = c4b + 2 * c, *c5b = c5w + c * c, *gamma = c5b + c, *hw = gamma + c, *hb = hw + 2 * c;
  const size_t HW = (size_t)H * W;
  double* u = malloc(sizeof(double) * HW * 2 * c); /* conv1 output of one image */
  double* g = malloc(sizeof(double) * HW * c);     /* gated, then attended */
  double* t = malloc(sizeof(double) * 2 * c);
  double* t2 = malloc(sizeof(double) * 2 * c);
  double* pooled = malloc(sizeof(double) * c);
  double* sca = malloc(sizeof(double) * c);
  for (int b = 0; b < B; ++b) {
    const double* f = feat + (size_t)b * HW * c;
    for (size_t q = 0; q < HW; ++q) {
      layer_norm_pixel(f + q * c, c, ln1w, ln1b, t);
      dense(t, c, 2 * c, c1w, c1b, u + q * 2 * c);
    }
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        for (int ch = 0; ch < 2 * c; ++ch) {
          double s = dwb[ch];
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              const int yy = y + dy - 1, xx = x + dx - 1;
              if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
              s += (double)dww[ch * 9 + dy * 3 + dx] * u[((size_t)yy * W + xx) * 2 * c + ch];
            }
          t[ch] = s;
        }
        for (int ch = 0; ch < c; ++ch) g[((size_t)y * W + x) * c + ch] = t[ch] * t[c + ch];
      }
    for (int ch = 0; ch < c; ++ch) {
      double s = 0.0;
      for (size_t q = 0; q < HW; ++q) s += g[q * c + ch];
      pooled[ch] = s / (double)HW;
    }
    dense(pooled, c, c, scaw, scab, sca);
    for (size_t q = 0; q < HW; ++q) {
      double* gq = g + q * c;
      for (int ch = 0; ch < c; ++ch) gq[ch] *= sca[ch];
      dense(gq, c, c, c3w, c3b, t);
      double yv[512];
      for (int ch = 0; ch < c; ++ch) yv[ch] = f[q * c + ch] + (double)beta[ch] * t[ch];
      layer_norm_pixel(yv, c, ln2w, ln2b, t);
      dense(t, c, 2 * c, c4w, c4b, t2);
      for (int ch = 0; ch < c; ++ch) t[ch] = t2[ch] * t2[c + ch];
      dense(t, c, c, c5w, c5b, t2);
      for (int ch = 0; ch < c; ++ch) yv[ch] += (double)gamma[ch] * t2[ch];
      double z[2];
      dense(yv, c, 2, hw, hb, z);
      for (int k = 0; k < 2; ++k) out2[((size_t)b * HW + q) * 2 + k] = 1.0 / (1.0 + exp(-z[k]));
    }
  }
  free(u); free(g); free(t); free(t2); free(pooled); free(sca);
}

/* Adapters on feat[B][H][W][c]: lightmaps[B][H][W][6] (+X, -X, +Y, -Y, +Z,
 * -Z) and extra[B][H][W][2] (alpha, emissive).  c <= 512. */
ORC_EXPORT int orc_adapters_forward(int c, const float* params, long n_params, int B, int H, int W,
                                    const double* feat, double* lightmaps, double* extra) {
  if (c < 1 || c > 512 || n_params != orc_adapter_param_count(c) || B < 1 || H < 1 || W < 1) return 1;
  static const int dst[4][2] = {{4, 5}, {0, 1}, {2, 3}, {-1, -2}};
  const long per = 7L * c * c + 35L * c + 2;
  const size_t n = (size_t)B * H * W;
  double* o2 = malloc(sizeof(double) * n * 2);
  for (int grp = 0; grp < 4; ++grp) {
    adapter_forward(c, params + grp * per, B, H, W, feat, o2);
    for (size_t q = 0; q < n; ++q)
      for (int k = 0; k < 2; ++k) {
        if (dst[grp][k] >= 0)
          lightmaps[q * 6 + dst[grp][k]] = o2[q * 2 + k];
        else
          extra[q * 2 + k] = o2[q * 2 + k];
      }
  }
  free(o2);
  return 0;
}

/* ------------------------------------------------- channel adapters: training */
/*
 * The adapters' backward pass, for training them with the network (Section
 * 4.3 puts them on the decoder output; Section 5 trains the whole model on
 * the lightmap loss).  adapter_forward_saved takes the same steps in the
 * same order as adapter_forward and keeps every intermediate; the backward
 * pass applies the chain rule to them in reverse.  The layer norm's
 * gradient is the textbook one: with xh = (x - mu) r, r = 1 / sqrt(var +
 * eps) and dxh the gradient at xh, dx = r (dxh - mean(dxh) - xh mean(dxh
 * xh)).  The depthwise conv's input gradient is the transposed
 * correlation (each tap sends dw * g back to the input pixel it read).
 */
typedef struct {
  double *xh1, *r1;        /* layer norm 1: normalised input [n][c], 1 / sigma [n] */
  double *u, *d;           /* conv1 output, depthwise output [n][2c] */
  double *gt;              /* simple gate [n][c] */
  double *m, *s;           /* image mean of gt, attention scale [B][c] */
  double *t3, *y;          /* conv3 output, first residual [n][c] */
  double *xh2, *r2;        /* layer norm 2: normalised y [n][c], 1 / sigma [n] */
  double *e, *h, *t5, *z;  /* conv4 output [n][2c], its gate, conv5 output, block output [n][c] */
  double *out;             /* sigmoid outputs [n][2] */
} AdSaved;

static void adsaved_free(AdSaved* S) {
  free(S->xh1); free(S->r1); free(S->u); free(S->d); free(S->gt); free(S->m); free(S->s); free(S->t3); free(S->y);
  free(S->xh2); free(S->r2); free(S->e); free(S->h); free(S->t5); free(S->z); free(S->out);
}

/* the tensors of one adapter's parameter (or gradient) slice */
#define AD_OFFSETS(c)                                                                                          \
  const long o_ln1w = 0, o_ln1b = (c), o_c1w = 2L * (c), o_c1b = o_c1w + 2L * (c) * (c), o_dww = o_c1b + 2L * (c), \
             o_dwb = o_dww + 18L * (c), o_scaw = o_dwb + 2L * (c), o_scab = o_scaw + (long)(c) * (c),             \
             o_c3w = o_scab + (c), o_c3b = o_c3w + (long)(c) * (c), o_beta = o_c3b + (c), o_ln2w = o_beta + (c),   \
             o_ln2b = o_ln2w + (c), o_c4w = o_ln2b + (c), o_c4b = o_c4w + 2L * (c) * (c), o_c5w = o_c4b + 2L * (c), \
             o_c5b = o_c5w + (long)(c) * (c), o_gamma = o_c5b + (c), o_hw = o_gamma + (c), o_hb = o_hw + 2L * (c)

/* layer norm over c values with the normalised values and 1 / sigma kept */
static void layer_norm_saved(const double* x, int c, const float* w, const float* b, double* xh, double* r,
                             double* out) {
  double mu = 0.0, var = 0.0;
  for (int i = 0; i < c; ++i) mu += x[i];
  mu /= c;
  for (int i = 0; i < c; ++i) var += (x[i] - mu) * (x[i] - mu);
  var /= c;
  *r = 1.0 / sqrt(var + 1e-6);
  for (int i = 0; i < c; ++i) {
    xh[i] = (x[i] - mu) * *r;
    out[i] = xh[i] * w[i] + b[i];
  }
}

static void adapter_forward_saved(int c, const float* P, int B, int H, int W, const double* feat, AdSaved* S) {
  AD_OFFSETS(c);
  const size_t HW = (size_t)H * W, n = (size_t)B * HW;
  S->xh1 = malloc(sizeof(double) * n * c); S->r1 = malloc(sizeof(double) * n);
  S->u = malloc(sizeof(double) * n * 2 * c); S->d = malloc(sizeof(double) * n * 2 * c);
  S->gt = malloc(sizeof(double) * n * c);
  S->m = malloc(sizeof(double) * B * c); S->s = malloc(sizeof(double) * B * c);
  S->t3 = malloc(sizeof(double) * n * c); S->y = malloc(sizeof(double) * n * c);
  S->xh2 = malloc(sizeof(double) * n * c); S->r2 = malloc(sizeof(double) * n);
  S->e = malloc(sizeof(double) * n * 2 * c); S->h = malloc(sizeof(double) * n * c);
  S->t5 = malloc(sizeof(double) * n * c); S->z = malloc(sizeof(double) * n * c);
  S->out = malloc(sizeof(double) * n * 2);
  double* t = malloc(sizeof(double) * 2 * c);
  double* a = malloc(sizeof(double) * c);
  for (int b = 0; b < B; ++b) {
    const size_t q0 = (size_t)b * HW;
    for (size_t q = q0; q < q0 + HW; ++q) {
      layer_norm_saved(feat + q * c, c, P + o_ln1w, P + o_ln1b, S->xh1 + q * c, S->r1 + q, t);
      dense(t, c, 2 * c, P + o_c1w, P + o_c1b, S->u + q * 2 * c);
    }
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const size_t q = q0 + (size_t)y * W + x;
        for (int ch = 0; ch < 2 * c; ++ch) {
          double sum = P[o_dwb + ch];
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              const int yy = y + dy - 1, xx = x + dx - 1;
              if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
              sum += (double)P[o_dww + ch * 9 + dy * 3 + dx] * S->u[(q0 + (size_t)yy * W + xx) * 2 * c + ch];
            }
          S->d[q * 2 * c + ch] = sum;
        }
        for (int ch = 0; ch < c; ++ch) S->gt[q * c + ch] = S->d[q * 2 * c + ch] * S->d[q * 2 * c + c + ch];
      }
    for (int ch = 0; ch < c; ++ch) {
      double sum = 0.0;
      for (size_t q = q0; q < q0 + HW; ++q) sum += S->gt[q * c + ch];
      S->m[(size_t)b * c + ch] = sum / (double)HW;
    }
    dense(S->m + (size_t)b * c, c, c, P + o_scaw, P + o_scab, S->s + (size_t)b * c);
    for (size_t q = q0; q < q0 + HW; ++q) {
      for (int ch = 0; ch < c; ++ch) a[ch] = S->gt[q * c + ch] * S->s[(size_t)b * c + ch];
      dense(a, c, c, P + o_c3w, P + o_c3b, S->t3 + q * c);
      for (int ch = 0; ch < c; ++ch) S->y[q * c + ch] = feat[q * c + ch] + (double)P[o_beta + ch] * S->t3[q * c + ch];
      layer_norm_saved(S->y + q * c, c, P + o_ln2w, P + o_ln2b, S->xh2 + q * c, S->r2 + q, t);
      dense(t, c, 2 * c, P + o_c4w, P + o_c4b, S->e + q * 2 * c);
      for (int ch = 0; ch < c; ++ch) S->h[q * c + ch] = S->e[q * 2 * c + ch] * S->e[q * 2 * c + c + ch];
      dense(S->h + q * c, c, c, P + o_c5w, P + o_c5b, S->t5 + q * c);
      for (int ch = 0; ch < c; ++ch) S->z[q * c + ch] = S->y[q * c + ch] + (double)P[o_gamma + ch] * S->t5[q * c + ch];
      double zz[2];
      dense(S->z + q * c, c, 2, P + o_hw, P + o_hb, zz);
      for (int k = 0; k < 2; ++k) S->out[q * 2 + k] = 1.0 / (1.0 + exp(-zz[k]));
    }
  }
  free(t); free(a);
}

/* dx += r (dxh - mean(dxh) - xh mean(dxh xh)) over c values */
static void layer_norm_bwd(const double* xh, double r, const double* dxh, int c, double* dx) {
  double m1 = 0.0, m2 = 0.0;
  for (int i = 0; i < c; ++i) {
    m1 += dxh[i];
    m2 += dxh[i] * xh[i];
  }
  m1 /= c;
  m2 /= c;
  for (int i = 0; i < c; ++i) dx[i] += r * (dxh[i] - m1 - xh[i] * m2);
}

/* dout[n][2]: the loss gradient at this adapter's two sigmoid outputs.
 * Adds the parameter gradient to G (this adapter's slice, laid out as P)
 * and the gradient with respect to the features to dfeat[n][c]. */
static void adapter_backward(int c, const float* P, int B, int H, int W, const AdSaved* S, const double* dout,
                             double* G, double* dfeat) {
  AD_OFFSETS(c);
  const size_t HW = (size_t)H * W, n = (size_t)B * HW;
  double* dgt = malloc(sizeof(double) * n * c);
  double* du = calloc(n * 2 * c, sizeof(double));
  double* ds = calloc((size_t)B * c, sizeof(double));
  double *dz = malloc(sizeof(double) * c), *dy = malloc(sizeof(double) * c), *dt = malloc(sizeof(double) * c),
         *dh = malloc(sizeof(double) * c), *de = malloc(sizeof(double) * 2 * c), *dxh = malloc(sizeof(double) * c),
         *da = malloc(sizeof(double) * c);
  for (size_t q = 0; q < n; ++q) {
    const size_t b = q / HW;
    const double *z = S->z + q * c, *t5 = S->t5 + q * c, *h = S->h + q * c, *e = S->e + q * 2 * c,
                 *xh2 = S->xh2 + q * c, *t3 = S->t3 + q * c, *gt = S->gt + q * c, *sv = S->s + b * c;
    /* sigmoid, then the head */
    double dop[2];
    for (int k = 0; k < 2; ++k) {
      const double o = S->out[q * 2 + k];
      dop[k] = dout[q * 2 + k] * o * (1.0 - o);
      G[o_hb + k] += dop[k];
      for (int ch = 0; ch < c; ++ch) G[o_hw + k * c + ch] += dop[k] * z[ch];
    }
    for (int ch = 0; ch < c; ++ch) dz[ch] = (double)P[o_hw + ch] * dop[0] + (double)P[o_hw + c + ch] * dop[1];
    /* z = y + gamma t5 */
    for (int ch = 0; ch < c; ++ch) {
      G[o_gamma + ch] += dz[ch] * t5[ch];
      dt[ch] = (double)P[o_gamma + ch] * dz[ch];
      dy[ch] = dz[ch];
    }
    /* t5 = W5 h + b5 */
    for (int o = 0; o < c; ++o) {
      G[o_c5b + o] += dt[o];
      for (int i = 0; i < c; ++i) G[o_c5w + (long)o * c + i] += dt[o] * h[i];
    }
    for (int i = 0; i < c; ++i) {
      double sum = 0.0;
      for (int o = 0; o < c; ++o) sum += (double)P[o_c5w + (long)o * c + i] * dt[o];
      dh[i] = sum;
    }
    /* h = e[:c] e[c:] */
    for (int i = 0; i < c; ++i) {
      de[i] = dh[i] * e[c + i];
      de[c + i] = dh[i] * e[i];
    }
    /* e = W4 n2 + b4, n2 = xh2 w2 + b2 */
    for (int o = 0; o < 2 * c; ++o) {
      G[o_c4b + o] += de[o];
      for (int i = 0; i < c; ++i) G[o_c4w + (long)o * c + i] += de[o] * (xh2[i] * P[o_ln2w + i] + P[o_ln2b + i]);
    }
    for (int i = 0; i < c; ++i) {
      double sum = 0.0;
      for (int o = 0; o < 2 * c; ++o) sum += (double)P[o_c4w + (long)o * c + i] * de[o];
      G[o_ln2w + i] += sum * xh2[i];
      G[o_ln2b + i] += sum;
      dxh[i] = sum * P[o_ln2w + i];
    }
    layer_norm_bwd(xh2, S->r2[q], dxh, c, dy);
    /* y = feat + beta t3 */
    for (int ch = 0; ch < c; ++ch) {
      dfeat[q * c + ch] += dy[ch];
      G[o_beta + ch] += dy[ch] * t3[ch];
      dt[ch] = (double)P[o_beta + ch] * dy[ch];
    }
    /* t3 = W3 a + b3, a = gt s */
    for (int o = 0; o < c; ++o) {
      G[o_c3b + o] += dt[o];
      for (int i = 0; i < c; ++i) G[o_c3w + (long)o * c + i] += dt[o] * (gt[i] * sv[i]);
    }
    for (int i = 0; i < c; ++i) {
      double sum = 0.0;
      for (int o = 0; o < c; ++o) sum += (double)P[o_c3w + (long)o * c + i] * dt[o];
      da[i] = sum;
      dgt[q * c + i] = sum * sv[i];
      ds[b * c + i] += sum * gt[i];
    }
  }
  /* s = Wsca m + bsca, m = mean of gt over the image */
  for (int b = 0; b < B; ++b) {
    const double *dsb = ds + (size_t)b * c, *mb = S->m + (size_t)b * c;
    for (int o = 0; o < c; ++o) {
      G[o_scab + o] += dsb[o];
      for (int i = 0; i < c; ++i) G[o_scaw + (long)o * c + i] += dsb[o] * mb[i];
    }
    for (int i = 0; i < c; ++i) {
      double sum = 0.0;
      for (int o = 0; o < c; ++o) sum += (double)P[o_scaw + (long)o * c + i] * dsb[o];
      da[i] = sum / (double)HW;
    }
    for (size_t q = (size_t)b * HW; q < (size_t)(b + 1) * HW; ++q)
      for (int i = 0; i < c; ++i) dgt[q * c + i] += da[i];
  }
  /* gt = d[:c] d[c:]; d = depthwise(u) + dwb (zero padded) */
  for (int b = 0; b < B; ++b) {
    const size_t q0 = (size_t)b * HW;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const size_t q = q0 + (size_t)y * W + x;
        for (int ch = 0; ch < 2 * c; ++ch) {
          const int i = ch < c ? ch : ch - c;
          const double g = dgt[q * c + i] * S->d[q * 2 * c + (ch < c ? c + i : i)];
          G[o_dwb + ch] += g;
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              const int yy = y + dy - 1, xx = x + dx - 1;
              if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
              const size_t nb = (q0 + (size_t)yy * W + xx) * 2 * c + ch;
              G[o_dww + ch * 9 + dy * 3 + dx] += g * S->u[nb];
              du[nb] += (double)P[o_dww + ch * 9 + dy * 3 + dx] * g;
            }
        }
      }
  }
  /* u = W1 n1 + b1, n1 = xh1 w1 + b1 */
  for (size_t q = 0; q < n; ++q) {
    const double* xh1 = S->xh1 + q * c;
    const double* duq = du + q * 2 * c;
    for (int o = 0; o < 2 * c; ++o) {
      G[o_c1b + o] += duq[o];
      for (int i = 0; i < c; ++i) G[o_c1w + (long)o * c + i] += duq[o] * (xh1[i] * P[o_ln1w + i] + P[o_ln1b + i]);
    }
    for (int i = 0; i < c; ++i) {
      double sum = 0.0;
      for (int o = 0; o < 2 * c; ++o) sum += (double)P[o_c1w + (long)o * c + i] * duq[o];
      G[o_ln1w + i] += sum * xh1[i];
      G[o_ln1b + i] += sum;
      dxh[i] = sum * P[o_ln1w + i];
    }
    layer_norm_bwd(xh1, S->r1[q], dxh, c, dfeat + q * c);
  }
  free(dgt); free(du); free(ds); free(dz); free(dy); free(dt); free(dh); free(de); free(dxh); free(da);
}

/* The network with the four adapters in place of its plain head, trained
 * jointly: lightmaps from the adapters (groups 0-2; group 3's alpha and
 * emissive have no target here and take no gradient), loss = mean squared
 * error over B*H*W*6 against target_srgb[B][H][W][6] as orc_unet_loss_grad,
 * and its gradient with respect to the trunk's parameters (grad[n_params];
 * the unused head's entries are 0) and the adapters' (grad_ad[n_ad]). */
ORC_EXPORT int orc_adapters_loss_grad(int levels, int base, const float* params, long n_params,
                                      const float* ad_params, long n_ad, int B, int H, int W, const double* guide,
                                      const double* target, double* loss, double* grad, double* grad_ad) {
  Net net;
  int st = net_setup(levels, base, params, n_params, &net);
  if (st) return st;
  const int c = base;
  if (c > 512 || n_ad != orc_adapter_param_count(c)) return 1;
  int div = 1 << (levels - 1);
  if (B < 1 || H < 1 || W < 1 || H % div || W % div) return 3;
  static const int dst[4][2] = {{4, 5}, {0, 1}, {2, 3}, {-1, -2}};
  const long per = 7L * c * c + 35L * c + 2;
  const size_t HW = (size_t)H * W, n = (size_t)B * HW;
  Fwd f;
  unet_forward_saved(&net, B, H, W, guide, &f);
  double* feat = malloc(sizeof(double) * n * c);
  nchw_to_nhwc(f.x_in[net.n - 1], B, c, H, W, feat);
  AdSaved S[4];
  for (int g = 0; g < 4; ++g) adapter_forward_saved(c, ad_params + g * per, B, H, W, feat, &S[g]);
  const double inv = 1.0 / (double)(n * 6);
  double l = 0.0;
  double* dout = malloc(sizeof(double) * n * 2);
  double* dfeat = calloc(n * c, sizeof(double));
  memset(grad, 0, sizeof(double) * (size_t)net.n_params);
  memset(grad_ad, 0, sizeof(double) * (size_t)n_ad);
  for (int g = 0; g < 4; ++g) {
    for (size_t q = 0; q < n; ++q)
      for (int k = 0; k < 2; ++k) {
        dout[q * 2 + k] = 0.0;
        if (dst[g][k] < 0) continue;
        const double e = S[g].out[q * 2 + k] - target[q * 6 + dst[g][k]];
        l += e * e;
        dout[q * 2 + k] = 2.0 * e * inv;
      }
    adapter_backward(c, ad_params + g * per, B, H, W, &S[g], dout, grad_ad + g * per, dfeat);
  }
  *loss = l * inv;
  /* the trunk, from the features' gradient (to NCHW) */
  double* gf = malloc(sizeof(double) * n * c);
  for (int b = 0; b < B; ++b)
    for (int ch = 0; ch < c; ++ch)
      for (size_t q = 0; q < HW; ++q) gf[((size_t)b * c + ch) * HW + q] = dfeat[((size_t)b * HW + q) * c + ch];
  trunk_backward(&net, &f, B, gf, grad);
  for (int g = 0; g < 4; ++g) adsaved_free(&S[g]);
  free(feat); free(dout); free(dfeat);
  fwd_free(&f, net.n);
  return 0;
}

/* Adam with bias correction, step t >= 1; p, m, v updated in place. */
ORC_EXPORT void orc_adam(long n, double* p, const double* g, double* m, double* v, int t, double lr, double b1, double b2,
                         double eps) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (long i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

ORC_EXPORT int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
