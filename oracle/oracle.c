/*
 * FP64 CPU oracle for screen-space path guiding with per-pixel parametric
 * mixture models (arXiv 2112.09728).  TEST INFRASTRUCTURE ONLY: it defines what
 * the GPU path must compute and is never called by the product path.
 *
 * Paper passages followed (section titles of the paper):
 *   Eq. (2) and its paragraph (Sec. 1)    the per-pixel mixture D = pi*N(M^-1(w)) + (1-pi)*BRDF
 *   Sec. 1, same paragraph               M is the Shirley-Chiu area-preserving square->hemisphere map
 *   Sec. 3.1 (Path tracing pass)          NN fetch of Gamma with motion vectors; new models with
 *                                         pi = 0.05, k = 0, sampled from the BRDF; zeta < pi selects
 *                                         Box-Muller + N(mu, Sigma) + M, otherwise the BRDF;
 *                                         depth/normal stopping tests and the change of hemisphere
 *   Sec. 3.2 (Training pass)              E-step posterior BRDF vs Gaussian, M-step with temporal
 *                                         filtering by the epoch k, neighbour samples, BRDF-strategy
 *                                         samples only, pi clamped to [0.05, 0.95]
 *   Fig. 2 caption                        samples weighted by the luminance of L_i f_r cos
 *   Sec. 2 (Previous Work)                online weighted EM of parametric mixtures
 *   Sec. 4.2 (Performance)                N = (1 - k/kMax)*15 + 5 close samples per pixel
 *   Sec. 5 (Current Pitfalls)             BRDF-only sampling for near-zero roughness
 * Where the paper is silent the reading taken is stated at the function.
 *
 * Everything is double precision, scalar and unblocked, except the few
 * decisions that turn floating point into an integer from single-precision
 * inputs (the reprojection address, the depth and normal tests and pixel
 * validity); those are taken in single precision with an explicit operation
 * order, which is the precision the GPU path decides them in.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define NCH 8

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
 * as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplications, with the
 * key advanced by the Weyl constants between rounds.  The paper only asks for
 * "a uniform random variable"; a counter-based generator makes the draws a
 * pure function of (pixel, frame, stream, call, view, seed). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw the four words of (pixel i, stream, call) for this frame and view. */
static void rng_words(const orc_params *P, uint32_t i, uint32_t stream, uint32_t call,
                      uint32_t w[4]) {
  uint32_t ctr[4] = {i, P->frame, (stream << 16) | call, P->view};
  uint32_t key[2] = {(uint32_t)(P->seed & 0xFFFFFFFFu), (uint32_t)(P->seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* 24-bit uniform in [0, 1): exactly representable in single and double. */
static double uniform24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------------- */
/* Vectors and the shading frame. */
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void normalize3(double v[3]) {
  double s = 1.0 / sqrt(dot3(v, v));
  v[0] *= s; v[1] *= s; v[2] *= s;
}

/* Orthonormal basis around a unit normal: the branchless construction of Duff,
 * Burgess, Christensen, Hery, Kensler, Liani, Villemin, "Building an
 * Orthonormal Basis, Revisited" (JCGT 2017). */
static void onb(const double n[3], double t[3], double b[3]) {
  double sign = copysign(1.0, n[2]);
  double a = -1.0 / (sign + n[2]);
  double c = n[0] * n[1] * a;
  t[0] = 1.0 + sign * n[0] * n[0] * a;
  t[1] = sign * c;
  t[2] = -sign * n[0];
  b[0] = c;
  b[1] = sign + n[1] * n[1] * a;
  b[2] = -n[1];
}

void orc_onb_n(int64_t n, const double *nrm, double *t, double *b) {
  for (int64_t i = 0; i < n; ++i) onb(nrm + 3 * i, t + 3 * i, b + 3 * i);
}

typedef struct frame_t { double t[3], b[3], n[3]; } frame_t;

static frame_t make_frame(const float *normal, int64_t plane, int64_t idx) {
  frame_t f;
  f.n[0] = normal[idx];
  f.n[1] = normal[plane + idx];
  f.n[2] = normal[2 * plane + idx];
  normalize3(f.n);
  onb(f.n, f.t, f.b);
  return f;
}
static void to_local(const frame_t *f, const double w[3], double l[3]) {
  l[0] = dot3(w, f->t);
  l[1] = dot3(w, f->b);
  l[2] = dot3(w, f->n);
}
static void to_world(const frame_t *f, const double l[3], double w[3]) {
  for (int c = 0; c < 3; ++c) w[c] = l[0] * f->t[c] + l[1] * f->b[c] + l[2] * f->n[c];
}

/* ------------------------------------------------------------------------- */
/* The map M of Eq. (2): Shirley and Chiu, "A Low Distortion Map Between Disk
 * and Square" (JGT 1997) takes the unit square to the unit disk (concentric
 * map), and the equal-area lift (x, y) -> (x sqrt(2 - r^2), y sqrt(2 - r^2),
 * 1 - r^2) takes the disk to the hemisphere.  Both steps preserve area up to a
 * constant, so d(omega) = 2 pi du. */
static void sq2hemi(const double u[2], double w[3]) {
  double a = 2.0 * u[0] - 1.0, b = 2.0 * u[1] - 1.0;
  double r, phi;
  if (a == 0.0 && b == 0.0) {
    w[0] = 0.0; w[1] = 0.0; w[2] = 1.0;
    return;
  }
  if (fabs(a) > fabs(b)) {
    r = a;
    phi = (PI / 4.0) * (b / a);
  } else {
    r = b;
    phi = PI / 2.0 - (PI / 4.0) * (a / b);
  }
  double s = r * sqrt(2.0 - r * r);
  w[0] = s * cos(phi);
  w[1] = s * sin(phi);
  w[2] = 1.0 - r * r;
}

/* Inverse of M for a direction on the upper hemisphere (w is normalised
 * first).  The squared disk radius is (w_x^2 + w_y^2)/(1 + w_z), which equals
 * 1 - w_z without its cancellation near the pole; the inverse concentric map
 * follows Shirley and Chiu's four angular sectors. */
static void hemi2sq(const double w_in[3], double u[2]) {
  double w[3] = {w_in[0], w_in[1], w_in[2]};
  normalize3(w);
  double rho2 = (w[0] * w[0] + w[1] * w[1]) / (1.0 + w[2]);
  double rho = sqrt(rho2);
  double s = sqrt(2.0 - rho2);
  double dx = w[0] / s, dy = w[1] / s;
  double a, b;
  if (rho == 0.0) {
    a = 0.0; b = 0.0;
  } else {
    double phi = atan2(dy, dx);
    if (phi < -PI / 4.0) phi += 2.0 * PI;
    if (phi < PI / 4.0) {
      a = rho;
      b = phi * a / (PI / 4.0);
    } else if (phi < 3.0 * PI / 4.0) {
      b = rho;
      a = -(phi - PI / 2.0) * b / (PI / 4.0);
    } else if (phi < 5.0 * PI / 4.0) {
      a = -rho;
      b = (phi - PI) * a / (PI / 4.0);
    } else {
      b = -rho;
      a = -(phi - 3.0 * PI / 2.0) * b / (PI / 4.0);
    }
  }
  u[0] = 0.5 * (a + 1.0);
  u[1] = 0.5 * (b + 1.0);
}

void orc_sq2hemi_n(int64_t n, const double *u, double *w) {
  for (int64_t i = 0; i < n; ++i) sq2hemi(u + 2 * i, w + 3 * i);
}
void orc_hemi2sq_n(int64_t n, const double *w, double *u) {
  for (int64_t i = 0; i < n; ++i) hemi2sq(w + 3 * i, u + 2 * i);
}

/* ------------------------------------------------------------------------- */
/* The BRDF of the synthetic materials (the paper's second mixture component is
 * "based on BRDF distribution"; its materials are not available, so the
 * workload uses Lambert + GGX): in the local frame with wo_z > 0,
 *   f_r(wi) = albedo/pi + F(wo.h) D(h) G1(wi) G1(wo) / (4 wi_z wo_z)
 * with the GGX distribution D, the separable Smith G1 and Schlick's F (Walter,
 * Marschner, Li, Torrance, EGSR 2007).  The BRDF-sampling density picks the
 * cosine lobe with probability s_d and the GGX normal distribution otherwise:
 *   p_b(wi) = s_d wi_z/pi + (1 - s_d) D(h) h_z / (4 wo.h),  wi_z > 0. */
static double ggx_D(const double h[3], double alpha) {
  double a2 = alpha * alpha;
  double d = h[0] * h[0] + h[1] * h[1] + a2 * h[2] * h[2];
  return a2 / (PI * d * d);
}
static double smith_G1(const double v[3], double alpha) {
  return 2.0 * v[2] / (v[2] + sqrt(alpha * alpha * (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]));
}
static void half_vector(const double wo[3], const double wi[3], double h[3]) {
  h[0] = wo[0] + wi[0]; h[1] = wo[1] + wi[1]; h[2] = wo[2] + wi[2];
  normalize3(h);
}
static double brdf_f(const double wo_in[3], const double wi_in[3], double alpha, double albedo,
                     double f0) {
  double wo[3] = {wo_in[0], wo_in[1], wo_in[2]}, wi[3] = {wi_in[0], wi_in[1], wi_in[2]};
  normalize3(wo);
  normalize3(wi);
  if (wi[2] <= 0.0 || wo[2] <= 0.0) return 0.0;
  double h[3];
  half_vector(wo, wi, h);
  double woh = dot3(wo, h);
  double F = f0 + (1.0 - f0) * pow(1.0 - woh, 5.0);
  return albedo / PI +
         F * ggx_D(h, alpha) * smith_G1(wi, alpha) * smith_G1(wo, alpha) / (4.0 * wi[2] * wo[2]);
}
static double brdf_pdf(const double wo_in[3], const double wi_in[3], double alpha, double s_d) {
  double wo[3] = {wo_in[0], wo_in[1], wo_in[2]}, wi[3] = {wi_in[0], wi_in[1], wi_in[2]};
  normalize3(wo);
  normalize3(wi);
  if (wi[2] <= 0.0) return 0.0;
  double h[3];
  half_vector(wo, wi, h);
  double woh = dot3(wo, h);
  return s_d * wi[2] / PI + (1.0 - s_d) * ggx_D(h, alpha) * h[2] / (4.0 * woh);
}
/* BRDF sampling: cosine lobe (Malley) if xi_l < s_d, otherwise a GGX normal
 * with tan^2(theta_h) = alpha^2 xi_1/(1 - xi_1), phi_h = 2 pi xi_2 (Walter et
 * al. 2007) reflected about h.  Returns 0 when the draw leaves the upper
 * hemisphere (a null sample). */
static int brdf_sample(const double wo_in[3], double alpha, double s_d, double xl, double x1,
                       double x2, double wi[3], double *margin) {
  double wo[3] = {wo_in[0], wo_in[1], wo_in[2]};
  normalize3(wo);
  if (xl < s_d) {
    double r = sqrt(x1), phi = 2.0 * PI * x2;
    wi[0] = r * cos(phi);
    wi[1] = r * sin(phi);
    wi[2] = sqrt(1.0 - x1);
    if (margin) *margin = fmin(fabs(xl - s_d), wi[2]);
    return wi[2] > 0.0;
  }
  double t2 = alpha * alpha * x1 / (1.0 - x1);
  double ch = 1.0 / sqrt(1.0 + t2);
  double sh = sqrt(t2) * ch;
  double phi = 2.0 * PI * x2;
  double h[3] = {sh * cos(phi), sh * sin(phi), ch};
  double woh = dot3(wo, h);
  for (int c = 0; c < 3; ++c) wi[c] = 2.0 * woh * h[c] - wo[c];
  if (margin) *margin = fmin(fabs(xl - s_d), fmin(fabs(wi[2]), fabs(woh)));
  return wi[2] > 0.0 && woh > 0.0;
}

void orc_brdf_f_n(int64_t n, const double *wo, const double *wi, const double *alpha,
                  const double *albedo, double f0, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = brdf_f(wo + 3 * i, wi + 3 * i, alpha[i], albedo[i], f0);
}
void orc_brdf_pdf_n(int64_t n, const double *wo, const double *wi, const double *alpha,
                    double s_diffuse, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = brdf_pdf(wo + 3 * i, wi + 3 * i, alpha[i], s_diffuse);
}
void orc_brdf_sample_n(int64_t n, const double *wo, const double *alpha, double s_diffuse,
                       const double *xi, double *wi, int32_t *valid) {
  for (int64_t i = 0; i < n; ++i)
    valid[i] = brdf_sample(wo + 3 * i, alpha[i], s_diffuse, xi[3 * i], xi[3 * i + 1],
                           xi[3 * i + 2], wi + 3 * i, NULL);
}

/* ------------------------------------------------------------------------- */
/* The Gaussian component of Eq. (2) lives on the unit square of M.  The
 * covariance is regularised as Sigma + eps*I (the paper gives no floor) and
 * factored by Cholesky, with the Schur complement floored at eps against
 * rounding; N is the plain, untruncated bivariate normal density. */
typedef struct gauss_t { double mx, my, l11, l21, l22; } gauss_t;

static gauss_t gauss_setup(const double g[5], double eps) {
  gauss_t G;
  G.mx = g[0];
  G.my = g[1];
  double a = g[2] + eps, b = g[3], c = g[4] + eps;
  G.l11 = sqrt(fmax(a, eps));
  G.l21 = b / G.l11;
  G.l22 = sqrt(fmax(c - G.l21 * G.l21, eps));
  return G;
}
static double gauss_pdf_sq(const gauss_t *G, const double u[2]) {
  double z1 = (u[0] - G->mx) / G->l11;
  double z2 = (u[1] - G->my - G->l21 * z1) / G->l22;
  return exp(-0.5 * (z1 * z1 + z2 * z2)) / (2.0 * PI * G->l11 * G->l22);
}
/* Solid-angle density of the guided lobe: N(M^-1(w)) / (2 pi), the 2 pi being
 * the constant Jacobian of M; zero below the horizon. */
static double guide_pdf(const gauss_t *G, const double l[3]) {
  if (l[2] <= 0.0) return 0.0;
  double u[2];
  hemi2sq(l, u);
  return gauss_pdf_sq(G, u) / (2.0 * PI);
}
/* Box-Muller (Sec. 3.1): two N(0,1) variables from (xi_1, xi_2), mapped to
 * N(mu, Sigma) by the lower Cholesky factor.  1 - xi_1 keeps the log finite. */
static void gauss_sample(const gauss_t *G, double x1, double x2, double u[2]) {
  double rho = sqrt(-2.0 * log(1.0 - x1));
  double z1 = rho * cos(2.0 * PI * x2), z2 = rho * sin(2.0 * PI * x2);
  u[0] = G->mx + G->l11 * z1;
  u[1] = G->my + G->l21 * z1 + G->l22 * z2;
}

void orc_gauss_pdf_sq_n(const double g[5], double eps, int64_t n, const double *u, double *out) {
  gauss_t G = gauss_setup(g, eps);
  for (int64_t i = 0; i < n; ++i) out[i] = gauss_pdf_sq(&G, u + 2 * i);
}
void orc_gauss_sample_n(const double g[5], double eps, int64_t n, const double *xi, double *u) {
  gauss_t G = gauss_setup(g, eps);
  for (int64_t i = 0; i < n; ++i) gauss_sample(&G, xi[2 * i], xi[2 * i + 1], u + 2 * i);
}
void orc_guide_pdf_n(const double g[5], double eps, int64_t n, const double *w, double *out) {
  gauss_t G = gauss_setup(g, eps);
  for (int64_t i = 0; i < n; ++i) out[i] = guide_pdf(&G, w + 3 * i);
}

/* ------------------------------------------------------------------------- */
/* Per-pixel inputs. */
typedef struct pixel_t {
  frame_t f;
  double wo[3];    /* local view direction */
  double alpha, albedo;
  int valid;       /* omega_o above the surface */
  int guided;      /* valid and rough enough to guide (Sec. 5) */
} pixel_t;

/* Single-precision dot product with a fixed operation order; used only for
 * decisions, which the GPU path takes in the same precision. */
static float dot3f(float a0, float a1, float a2, float b0, float b1, float b2) {
  return fmaf(a2, b2, fmaf(a1, b1, a0 * b0));
}

static int pixel_valid(const orc_view *v, int64_t idx) {
  int64_t pl = (int64_t)v->height * v->pitch;
  const float *n = v->normal, *o = v->view_dir;
  return dot3f(n[idx], n[pl + idx], n[2 * pl + idx], o[idx], o[pl + idx], o[2 * pl + idx]) > 0.0f;
}

static pixel_t load_pixel(const orc_params *P, const orc_view *v, int64_t idx) {
  pixel_t px;
  int64_t pl = (int64_t)v->height * v->pitch;
  px.f = make_frame(v->normal, pl, idx);
  double o[3] = {v->view_dir[idx], v->view_dir[pl + idx], v->view_dir[2 * pl + idx]};
  normalize3(o);
  to_local(&px.f, o, px.wo);
  double r = (double)v->roughness[idx];
  px.alpha = r * r;
  px.albedo = (double)v->albedo[idx];
  px.valid = pixel_valid(v, idx);
  px.guided = px.valid && (v->roughness[idx] >= P->rough_min);
  return px;
}

static void gamma_get(const double *gamma, int64_t pl, int64_t idx, double g[NCH]) {
  for (int c = 0; c < NCH; ++c) g[c] = gamma[c * pl + idx];
}
static void gamma_put(double *gamma, int64_t pl, int64_t idx, const double g[NCH]) {
  for (int c = 0; c < NCH; ++c) gamma[c * pl + idx] = g[c];
}

/* State of a new model (Sec. 3.1): pi = 0.05 and k = 0 from the paper; the
 * remaining channels are this build's reading: mu at the centre of the square
 * (the normal direction), Sigma the covariance of U[0,1]^2, evidence W = 0. */
static void gamma_reset(const orc_params *P, double g[NCH]) {
  g[0] = 0.5; g[1] = 0.5;
  g[2] = 1.0 / 12.0; g[3] = 0.0; g[4] = 1.0 / 12.0;
  g[5] = (double)P->pi_init;
  g[6] = 0.0; g[7] = 0.0;
}

/* Mixing weight used for sampling and for D: guiding is off while k = 0 (a new
 * model samples the BRDF, Sec. 3.1) and for pixels that are not guided. */
static double pi_effective(const pixel_t *px, const double g[NCH]) {
  return (px->guided && g[7] >= 1.0) ? g[5] : 0.0;
}

static gauss_t pixel_gauss(const orc_params *P, const double g[NCH]) {
  return gauss_setup(g, (double)P->eps_sigma);
}

/* ------------------------------------------------------------------------- */
/* Reprojection (Sec. 3.1): the model is fetched from the previous frame with
 * nearest-neighbour filtering through the motion vectors, rejected by the
 * depth and normal tests and re-expressed in the hemisphere of the current
 * surface.  Readings: source q = floor(p + 1/2 - mv); reject when
 * |z - z_q| > tau_z z or n.n_q < tau_n; a rejected or invalid history, a
 * non-finite state or an unguided pixel starts a new model; the lobe mean is
 * carried to the new hemisphere through M (w = M(mu) in the old frame, mu' =
 * M^-1 of w in the new frame, new model if w falls below the new horizon),
 * and Sigma, pi, W and k are kept. */
void orc_reproject(const orc_params *P, const orc_view *cur, const orc_view *prev,
                   const double *gamma_prev, double *gamma_out, int32_t *src_index,
                   orc_rect r) {
  const int W = cur->width, H = cur->height;
  const int64_t pl = (int64_t)H * cur->pitch;
  const int64_t ppl = prev ? (int64_t)prev->height * prev->pitch : 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * cur->pitch + x;
      double g[NCH];
      int32_t src = -1;
      pixel_t px = load_pixel(P, cur, idx);
      int keep = (P->frame > 0) && gamma_prev != NULL && prev != NULL && px.guided;
      if (keep && cur->disocc && cur->disocc[idx]) keep = 0;
      int qx = 0, qy = 0;
      if (keep) {
        float mx = cur->motion ? cur->motion[idx] : 0.0f;
        float my = cur->motion ? cur->motion[pl + idx] : 0.0f;
        float fx = ((float)x + 0.5f) - mx;
        float fy = ((float)y + 0.5f) - my;
        /* floor(f) lies in [0, n) exactly when f does; the comparison also
           sends a non-finite motion vector to a new model */
        if (fx >= 0.0f && fy >= 0.0f && fx < (float)prev->width && fy < (float)prev->height) {
          qx = (int)floorf(fx);
          qy = (int)floorf(fy);
        } else {
          keep = 0;
        }
      }
      int64_t qidx = 0;
      if (keep) {
        qidx = (int64_t)qy * prev->pitch + qx;
        float zp = cur->depth[idx], zq = prev->depth[qidx];
        if (fabsf(zp - zq) > P->tau_depth * zp) keep = 0;
        const float *n = cur->normal, *m = prev->normal;
        float nd = dot3f(n[idx], n[pl + idx], n[2 * pl + idx], m[qidx], m[ppl + qidx],
                         m[2 * ppl + qidx]);
        if (nd < P->tau_normal) keep = 0;
      }
      if (keep) {
        gamma_get(gamma_prev, ppl, qidx, g);
        for (int c = 0; c < NCH; ++c)
          if (!isfinite(g[c])) keep = 0;
      }
      if (keep) {
        int same = 1;
        for (int c = 0; c < 3; ++c)
          if (cur->normal[c * pl + idx] != prev->normal[c * ppl + qidx]) same = 0;
        if (!same) {
          frame_t fq = make_frame(prev->normal, ppl, qidx);
          double mu[2] = {fmin(fmax(g[0], 0.0), 1.0), fmin(fmax(g[1], 0.0), 1.0)};
          double lq[3], w[3], lp[3];
          sq2hemi(mu, lq);
          to_world(&fq, lq, w);
          to_local(&px.f, w, lp);
          if (lp[2] <= 0.0) {
            keep = 0;
          } else {
            double u[2];
            hemi2sq(lp, u);
            g[0] = u[0];
            g[1] = u[1];
          }
        }
      }
      if (keep) {
        src = (int32_t)(qy * prev->width + qx);
      } else {
        gamma_reset(P, g);
      }
      gamma_put(gamma_out, pl, idx, g);
      if (src_index) src_index[idx] = src;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Mixture density of Eq. (2) at a local direction, with the readings: the
 * second term is (1 - pi) times the BRDF-sampling density, and the Gaussian
 * term is N(M^-1(w))/(2 pi).  pg and pb receive the two component densities. */
static double mixture_pdf(const orc_params *P, const pixel_t *px, const double g[NCH],
                          const double l[3], double *pg_out, double *pb_out) {
  double pg = 0.0, pb = 0.0;
  if (px->valid && l[2] > 0.0) {
    gauss_t G = pixel_gauss(P, g);
    pg = guide_pdf(&G, l);
    pb = brdf_pdf(px->wo, l, px->alpha, (double)P->s_diffuse);
  }
  double pe = pi_effective(px, g);
  if (pg_out) *pg_out = pg;
  if (pb_out) *pb_out = pb;
  return pe * pg + (1.0 - pe) * pb;
}

/* Guided sampling with one-sample MIS (Sec. 3.1 and Eq. (2)): for each sample
 * the four words of stream 0 give (zeta, xi_l, xi_1, xi_2); zeta < pi selects
 * the Gaussian (Box-Muller, Cholesky, then M), otherwise the BRDF.  A Gaussian
 * draw outside the unit square is a null sample (this build's reading: the
 * density is not renormalised, so such a draw contributes zero).  The record
 * holds the world direction, D(w), p_b(w) and the strategy. */
void orc_sample(const orc_params *P, const orc_view *v, const double *gamma, int32_t spp,
                double *dir, double *pdf_mix, double *pdf_brdf, uint8_t *strategy,
                double *margin, orc_rect r) {
  const int W = v->width, H = v->height;
  const int64_t pl = (int64_t)H * v->pitch;
  const int64_t spl = (int64_t)spp * pl;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      double g[NCH];
      gamma_get(gamma, pl, idx, g);
      gauss_t G = pixel_gauss(P, g);
      double pe = pi_effective(&px, g);
      for (int s = 0; s < spp; ++s) {
        const int64_t o = (int64_t)s * pl + idx;
        uint8_t code = 0;
        double l[3] = {0, 0, 0}, mg = INFINITY;
        if (px.valid) {
          uint32_t w4[4];
          rng_words(P, (uint32_t)(y * W + x), 0, (uint32_t)s, w4);
          double zeta = uniform24(w4[0]), xl = uniform24(w4[1]);
          double x1 = uniform24(w4[2]), x2 = uniform24(w4[3]);
          if (pe > 0.0) mg = fabs(zeta - pe);
          if (zeta < pe) {
            double u[2];
            gauss_sample(&G, x1, x2, u);
            double dist = fmin(fmin(fabs(u[0]), fabs(1.0 - u[0])), fmin(fabs(u[1]), fabs(1.0 - u[1])));
            mg = fmin(mg, dist);
            if (u[0] >= 0.0 && u[0] <= 1.0 && u[1] >= 0.0 && u[1] <= 1.0) {
              sq2hemi(u, l);
              code = 2;
            } else {
              code = 3;
            }
          } else {
            double m2 = INFINITY;
            int ok = brdf_sample(px.wo, px.alpha, (double)P->s_diffuse, xl, x1, x2, l, &m2);
            mg = fmin(mg, m2);
            code = ok ? 1 : 4;
          }
        }
        double w[3] = {0, 0, 0}, D = 0.0, pb = 0.0;
        if (code == 1 || code == 2) {
          to_world(&px.f, l, w);
          D = mixture_pdf(P, &px, g, l, NULL, &pb);
        }
        for (int c = 0; c < 3; ++c) dir[c * spl + o] = w[c];
        pdf_mix[o] = D;
        pdf_brdf[o] = pb;
        strategy[o] = code;
        if (margin) margin[o] = mg;
      }
    }
  }
}

/* Densities of given world directions (n_per_px per pixel): D(w), and
 * optionally the unweighted guided density and the BRDF-sampling density. */
void orc_pdf(const orc_params *P, const orc_view *v, const double *gamma, int32_t n_per_px,
             const double *dir, double *pdf_mix, double *pdf_guide, double *pdf_brdf,
             orc_rect r) {
  const int H = v->height;
  const int64_t pl = (int64_t)H * v->pitch;
  const int64_t spl = (int64_t)n_per_px * pl;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      double g[NCH];
      gamma_get(gamma, pl, idx, g);
      for (int j = 0; j < n_per_px; ++j) {
        const int64_t o = (int64_t)j * pl + idx;
        double w[3] = {dir[o], dir[spl + o], dir[2 * spl + o]}, l[3];
        double pg = 0.0, pb = 0.0, D = 0.0;
        if (px.valid && dot3(w, w) > 0.0) {
          normalize3(w);
          to_local(&px.f, w, l);
          D = mixture_pdf(P, &px, g, l, &pg, &pb);
        }
        pdf_mix[o] = D;
        if (pdf_guide) pdf_guide[o] = pg;
        if (pdf_brdf) pdf_brdf[o] = pb;
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Stand-in for the traced incident radiance (the paper traces the scene; this
 * build has no geometry): a constant ambient term plus spherical-Gaussian
 * lights, each gated by a per-pixel visibility bit:
 *   L(p, w) = ambient + sum_l V(p, l) c_l exp(lambda_l (w.xi_l - 1)).
 * with w and xi_l taken as unit vectors.  Null and missing samples carry no
 * radiance. */
void orc_light(int32_t n_lights, const float *lights, double ambient, const uint8_t *vis,
               int32_t width, int32_t height, int32_t pitch, int32_t spp, const double *dir,
               const uint8_t *strategy, double *radiance, orc_rect r) {
  const int64_t pl = (int64_t)height * pitch;
  const int64_t spl = (int64_t)spp * pl;
  (void)width;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * pitch + x;
      for (int s = 0; s < spp; ++s) {
        const int64_t o = (int64_t)s * pl + idx;
        double L = 0.0;
        if (strategy[o] == 1 || strategy[o] == 2) {
          double w[3] = {dir[o], dir[spl + o], dir[2 * spl + o]};
          normalize3(w);
          L = ambient;
          for (int k = 0; k < n_lights; ++k) {
            if (!((vis[idx] >> k) & 1u)) continue;
            const float *lt = lights + 5 * k;
            double ax[3] = {lt[0], lt[1], lt[2]};
            normalize3(ax);
            L += (double)lt[4] * exp((double)lt[3] * (dot3(w, ax) - 1.0));
          }
        }
        radiance[o] = L;
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Training set of a pixel (Sec. 3.2, Sec. 4.2, Fig. 2 caption): the pixel's own
 * BRDF-strategy samples in sample order, then N(k) = 5 + floor(15 (kMax - k) /
 * kMax) picks among the samples of the (2R+1)^2 - 1 surrounding pixels, drawn
 * with replacement from stream 1 (16 bits per pick, eight picks per call); a
 * pick is used when it lies in the image and is a BRDF-strategy sample. */
static int n_picks(const orc_params *P, int k) {
  if (k < 0) k = 0;
  if (k > P->k_max) k = P->k_max;
  return 5 + (15 * (P->k_max - k)) / P->k_max;
}

int32_t orc_training_set(const orc_params *P, const orc_view *v, int32_t spp,
                         const uint8_t *strategy, int32_t x, int32_t y, int32_t k,
                         int32_t *q_index, int32_t *s_index, int32_t *keep, int32_t cap) {
  const int W = v->width, H = v->height;
  const int64_t pl = (int64_t)H * v->pitch;
  const int R = P->radius, side = 2 * R + 1, C = side * side - 1;
  int32_t n = 0;
  for (int s = 0; s < spp && n < cap; ++s) {
    int64_t o = (int64_t)s * pl + (int64_t)y * v->pitch + x;
    q_index[n] = y * W + x;
    s_index[n] = s;
    keep[n] = strategy[o] == 1;
    ++n;
  }
  int N = n_picks(P, k);
  uint32_t w4[4] = {0, 0, 0, 0};
  for (int m = 0; m < N && n < cap; ++m) {
    if (m % 8 == 0) rng_words(P, (uint32_t)(y * W + x), 1, (uint32_t)(m / 8), w4);
    uint32_t word = w4[(m / 2) % 4];
    uint32_t h16 = (m % 2 == 0) ? (word & 0xFFFFu) : (word >> 16);
    uint32_t c = (uint32_t)(((uint64_t)h16 * (uint64_t)(C * spp)) >> 16);
    int o = (int)(c / (uint32_t)spp), s = (int)(c % (uint32_t)spp);
    if (o >= C / 2) o += 1; /* skip the centre of the window */
    int qx = x + (o % side) - R, qy = y + (o / side) - R;
    int inside = qx >= 0 && qy >= 0 && qx < W && qy < H;
    q_index[n] = inside ? qy * W + qx : -1;
    s_index[n] = s;
    keep[n] = inside && strategy[(int64_t)s * pl + (int64_t)qy * v->pitch + qx] == 1;
    ++n;
  }
  return n;
}

/* Weighted statistics of the Gaussian component over a batch (E-step
 * responsibilities gam, sample weights w):
 *   B0 = sum w, B1 = sum w gam, m = sum w gam u / B1,
 *   S = sum w gam (u - m)(u - m)^T / B1   (two passes, as defined). */
void orc_batch_stats(int64_t n, const double *u, const double *w, const double *gam,
                     double out[7]) {
  double B0 = 0.0, B1 = 0.0, mx = 0.0, my = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    B0 += w[j];
    B1 += w[j] * gam[j];
    mx += w[j] * gam[j] * u[2 * j];
    my += w[j] * gam[j] * u[2 * j + 1];
  }
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  if (B1 > 0.0) {
    mx /= B1;
    my /= B1;
    for (int64_t j = 0; j < n; ++j) {
      double dx = u[2 * j] - mx, dy = u[2 * j + 1] - my, c = w[j] * gam[j];
      sxx += c * dx * dx;
      sxy += c * dx * dy;
      syy += c * dy * dy;
    }
    sxx /= B1;
    sxy /= B1;
    syy /= B1;
  } else {
    mx = my = 0.0;
  }
  out[0] = B0; out[1] = B1; out[2] = mx; out[3] = my;
  out[4] = sxx; out[5] = sxy; out[6] = syy;
}

static double clamp_pi(const orc_params *P, double p) {
  if (P->flags & ORC_NO_CLAMP) return p;
  return fmin(fmax(p, (double)P->pi_lo), (double)P->pi_hi);
}

/* M-step with temporal filtering by the epoch k (Sec. 3.2), in this build's
 * reading: the stored state is the pooled weighted estimate with total
 * evidence W and Gaussian evidence pi W; a new batch enters with step
 * eta = 1/(k+1) (a running average that becomes an exponential average once k
 * reaches kMax):
 *   s_w = (1-eta) W + eta B0,  s_o = (1-eta) pi W,  s_n = eta B1,
 *   mu  = (s_o mu + s_n m)/(s_o + s_n),
 *   Sigma = (s_o Sigma + s_n S)/(s_o + s_n) + s_o s_n/(s_o + s_n)^2 (mu - m)(mu - m)^T
 *   (the pooled covariance of Chan, Golub and LeVeque),
 *   pi = clamp((s_o + s_n)/s_w, 0.05, 0.95) (Sec. 3.2), W = s_w, k = min(k+1, kMax).
 * An empty batch (B0 <= 0) leaves the state unchanged. */
void orc_merge(const orc_params *P, const double g_in[8], const double st[7], double g_out[8]) {
  double g[NCH];
  memcpy(g, g_in, sizeof(g));
  const double B0 = st[0], B1 = st[1];
  if (!(B0 > 0.0)) {
    memcpy(g_out, g, sizeof(g));
    return;
  }
  double k = g[7];
  double eta = 1.0 / (k + 1.0);
  double sw = (1.0 - eta) * g[6] + eta * B0;
  double so = (1.0 - eta) * g[5] * g[6];
  double sn = eta * B1;
  double sg = so + sn;
  if (sg > 0.0 && B1 > 0.0) {
    double al = so / sg, be = sn / sg;
    double dx = g[0] - st[2], dy = g[1] - st[3];
    double mux = al * g[0] + be * st[2];
    double muy = al * g[1] + be * st[3];
    double sxx = al * g[2] + be * st[4] + al * be * dx * dx;
    double sxy = al * g[3] + be * st[5] + al * be * dx * dy;
    double syy = al * g[4] + be * st[6] + al * be * dy * dy;
    g[0] = mux; g[1] = muy; g[2] = sxx; g[3] = sxy; g[4] = syy;
  }
  g[5] = clamp_pi(P, sg / sw);
  g[6] = sw;
  g[7] = fmin(k + 1.0, (double)P->k_max);
  memcpy(g_out, g, sizeof(g));
}

/* E-step quantities of one training sample at pixel px (Sec. 3.2, Fig. 2
 * caption): local direction l, square coordinate u = M^-1(l), importance
 * weight w = L f_r(l) l_z / p_src (the luminance of L_i f_r cos over the
 * density the sample was drawn with) and the posterior gam of the Gaussian
 * against the BRDF under the model's pi.  Returns 0 for a sample below the
 * pixel's horizon. */
static int estep_sample(const orc_params *P, const pixel_t *px, const gauss_t *G, double pi,
                        const double wdir[3], double L, double p_src, double u[2], double *w,
                        double *gam, double *pg_out, double *pb_out) {
  double wn[3] = {wdir[0], wdir[1], wdir[2]}, l[3];
  if (!(dot3(wn, wn) > 0.0) || !(p_src > 0.0)) return 0;
  normalize3(wn);
  to_local(&px->f, wn, l);
  if (l[2] <= 0.0) return 0;
  hemi2sq(l, u);
  double f = brdf_f(px->wo, l, px->alpha, px->albedo, (double)P->f0);
  *w = L * f * l[2] / p_src;
  double pg = gauss_pdf_sq(G, u) / (2.0 * PI);
  double pb = brdf_pdf(px->wo, l, px->alpha, (double)P->s_diffuse);
  double a = pi * pg, b = (1.0 - pi) * pb;
  *gam = (a + b > 0.0) ? a / (a + b) : 0.0;
  if (pg_out) *pg_out = pg;
  if (pb_out) *pb_out = pb;
  return 1;
}

#define MAX_SET 64

typedef struct tset_t {
  int n;
  double dir[MAX_SET][3];
  double L[MAX_SET], psrc[MAX_SET];
  int64_t pix[MAX_SET], rec[MAX_SET]; /* source pixel (plane index) and record offset */
} tset_t;

static void gather_set(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
                       const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
                       int x, int y, int k, tset_t *T) {
  const int W = v->width, H = v->height;
  const int64_t pl = (int64_t)H * v->pitch, spl = (int64_t)spp * pl;
  int32_t qi[MAX_SET], si[MAX_SET], keep[MAX_SET];
  int n = orc_training_set(P, v, spp, strategy, x, y, k, qi, si, keep, MAX_SET);
  T->n = 0;
  for (int j = 0; j < n; ++j) {
    if (!keep[j]) continue;
    int qx = qi[j] % W, qy = qi[j] / W;
    int64_t o = (int64_t)si[j] * pl + (int64_t)qy * v->pitch + qx;
    T->dir[T->n][0] = dir[o];
    T->dir[T->n][1] = dir[spl + o];
    T->dir[T->n][2] = dir[2 * spl + o];
    T->L[T->n] = radiance[o];
    T->psrc[T->n] = pdf_brdf[o];
    T->pix[T->n] = (int64_t)qy * v->pitch + qx;
    T->rec[T->n] = o;
    T->n++;
  }
  (void)H;
}

/* Rejection of a stale history (the paper leaves stronger rejection of
 * reprojected models open, Sec. 5): with the E-step's densities of the
 * batch, compare the weighted log-likelihood under the reprojected model,
 *   l_m = sum w log(pi p_g + (1 - pi) p_b),
 * with the one under a new model (the reset lobe, pi = pi_init),
 *   l_r = sum w log(pi_init p_g,new + (1 - pi_init) p_b);
 * the history is stale when l_m - l_r < -stale_tau sum w. */
static double mixture_at(const gauss_t *G, double pi, const double u[2], double pb) {
  return pi * gauss_pdf_sq(G, u) / (2.0 * PI) + (1.0 - pi) * pb;
}

static int stale_history(const orc_params *P, const double g[NCH], int n, double u[][2], const double *w,
                         const double *pb) {
  double g0[NCH];
  gamma_reset(P, g0);
  const gauss_t G = pixel_gauss(P, g), G0 = pixel_gauss(P, g0);
  double lm = 0.0, lr = 0.0, ws = 0.0;
  for (int j = 0; j < n; ++j) {
    const double dm = mixture_at(&G, g[5], u[j], pb[j]);
    const double dr = mixture_at(&G0, g0[5], u[j], pb[j]);
    if (!(w[j] > 0.0) || !(dm > 0.0) || !(dr > 0.0)) continue;
    lm += w[j] * log(dm);
    lr += w[j] * log(dr);
    ws += w[j];
  }
  return ws > 0.0 && (lm - lr) < -(double)P->stale_tau * ws;
}

/* The margin of that decision per pixel: (l_m - l_r) / sum w + stale_tau
 * (negative: the history is reset); NaN where the test does not apply (not
 * guided, k < 1, or no weight).  Test infrastructure for decisions taken in
 * different precisions. */
void orc_stale_margin(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
                      const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
                      const double *gamma, double *out, orc_rect r) {
  const int64_t pl = (int64_t)v->height * v->pitch;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    tset_t *T = (tset_t *)malloc(sizeof(tset_t));
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      out[idx] = NAN;
      pixel_t px = load_pixel(P, v, idx);
      double g[NCH];
      gamma_get(gamma, pl, idx, g);
      if (!px.guided || (int)g[7] < 1) continue;
      gather_set(P, v, spp, dir, pdf_brdf, strategy, radiance, x, y, (int)g[7], T);
      gauss_t G = pixel_gauss(P, g);
      double u[MAX_SET][2], w[MAX_SET], gam[MAX_SET], pg[MAX_SET], pb[MAX_SET];
      int n = 0;
      for (int j = 0; j < T->n; ++j)
        if (estep_sample(P, &px, &G, g[5], T->dir[j], T->L[j], T->psrc[j], u[n], &w[n], &gam[n], &pg[n], &pb[n]))
          ++n;
      double g0[NCH];
      gamma_reset(P, g0);
      const gauss_t G0 = pixel_gauss(P, g0);
      double lm = 0.0, lr = 0.0, ws = 0.0;
      for (int j = 0; j < n; ++j) {
        const double dm = mixture_at(&G, g[5], u[j], pb[j]);
        const double dr = mixture_at(&G0, g0[5], u[j], pb[j]);
        if (!(w[j] > 0.0) || !(dm > 0.0) || !(dr > 0.0)) continue;
        lm += w[j] * log(dm);
        lr += w[j] * log(dr);
        ws += w[j];
      }
      if (ws > 0.0) out[idx] = (lm - lr) / ws + (double)P->stale_tau;
    }
    free(T);
  }
}

/* Online EM update (Sec. 3.2): E-step over the training set with the
 * reprojected model, then the stepwise merge.  With batch != 0 the E- and
 * M-steps are iterated on the same training set with eta = 1 (plain batch EM:
 * mu, Sigma and pi are replaced by the batch estimate; W and k are kept). */
void orc_em(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
            const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
            double *gamma, int32_t iterations, int32_t batch, double *stats, orc_rect r) {
  const int H = v->height;
  const int64_t pl = (int64_t)H * v->pitch;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    tset_t *T = (tset_t *)malloc(sizeof(tset_t));
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      if (stats) {
        stats[idx] = 0.0;
        stats[pl + idx] = 0.0;
      }
      if (!px.guided) continue;
      double g[NCH];
      gamma_get(gamma, pl, idx, g);
      gather_set(P, v, spp, dir, pdf_brdf, strategy, radiance, x, y, (int)g[7], T);
      int iters = batch ? iterations : 1;
      for (int it = 0; it < iters; ++it) {
        gauss_t G = pixel_gauss(P, g);
        double u[MAX_SET][2], w[MAX_SET], gam[MAX_SET], pg[MAX_SET], pb[MAX_SET];
        int n = 0;
        for (int j = 0; j < T->n; ++j) {
          if (estep_sample(P, &px, &G, g[5], T->dir[j], T->L[j], T->psrc[j], u[n], &w[n],
                           &gam[n], &pg[n], &pb[n]))
            ++n;
        }
        if (!batch && (P->flags & ORC_STALE_RESET) && (int)g[7] >= 1 &&
            stale_history(P, g, n, u, w, pb)) {
          /* the history explains the batch worse than a new model: start over */
          gamma_reset(P, g);
          G = pixel_gauss(P, g);
          n = 0;
          for (int j = 0; j < T->n; ++j) {
            if (estep_sample(P, &px, &G, g[5], T->dir[j], T->L[j], T->psrc[j], u[n], &w[n],
                             &gam[n], NULL, NULL))
              ++n;
          }
        }
        double st[7];
        orc_batch_stats(n, &u[0][0], w, gam, st);
        if (stats) {
          stats[idx] = st[0];
          stats[pl + idx] = st[1];
        }
        if (!batch) {
          orc_merge(P, g, st, g);
        } else if (st[0] > 0.0) {
          if (st[1] > 0.0) {
            g[0] = st[2]; g[1] = st[3]; g[2] = st[4]; g[3] = st[5]; g[4] = st[6];
          }
          g[5] = clamp_pi(P, st[1] / st[0]);
        }
      }
      gamma_put(gamma, pl, idx, g);
    }
    free(T);
  }
}

/* ------------------------------------------------------------------------- */
/* Radiance-weighted negative log-likelihood of the mixture over a pixel's
 * training set, and its gradient.  Parameters theta per pixel:
 *   (mu_x, mu_y, l11, l21, l22, logit pi, unused, k), Sigma = L L^T,
 * the Gaussian using Sigma + eps I as everywhere else.  With d = u - mu,
 * v = (Sigma + eps I)^-1 d and gam the posterior of the Gaussian:
 *   dNLL/dmu = -sum w gam v,
 *   dNLL/dSigma = G = -1/2 sum w gam (v v^T - (Sigma + eps I)^-1),  dNLL/dL = 2 G L,
 *   dNLL/dlogit = -sum w (gam - pi).
 * The gradient is scaled by grad_out (1 when NULL); channels 6 and 7 are 0. */
void orc_nll(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
             const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
             const double *theta, const double *grad_out, double *grad, double *nll,
             orc_rect r) {
  const int H = v->height;
  const int64_t pl = (int64_t)H * v->pitch;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    tset_t *T = (tset_t *)malloc(sizeof(tset_t));
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      double th[NCH], gr[NCH] = {0, 0, 0, 0, 0, 0, 0, 0}, loss = 0.0;
      gamma_get(theta, pl, idx, th);
      if (px.guided) {
        gather_set(P, v, spp, dir, pdf_brdf, strategy, radiance, x, y, (int)th[7], T);
        double eps = (double)P->eps_sigma;
        double l11 = th[2], l21 = th[3], l22 = th[4];
        double sig[5] = {th[0], th[1], l11 * l11, l11 * l21, l21 * l21 + l22 * l22};
        gauss_t G = gauss_setup(sig, eps);
        double pi = 1.0 / (1.0 + exp(-th[5]));
        double a = sig[2] + eps, b = sig[3], c = sig[4] + eps;
        double det = a * c - b * b;
        double ia = c / det, ib = -b / det, ic = a / det; /* (Sigma + eps I)^-1 */
        double gmx = 0, gmy = 0, Gxx = 0, Gxy = 0, Gyy = 0, gl = 0;
        for (int j = 0; j < T->n; ++j) {
          double u[2], w, gam, pg, pb;
          if (!estep_sample(P, &px, &G, pi, T->dir[j], T->L[j], T->psrc[j], u, &w, &gam, &pg,
                            &pb))
            continue;
          double D = pi * pg + (1.0 - pi) * pb;
          loss -= w * log(D);
          double dx = u[0] - th[0], dy = u[1] - th[1];
          double vx = ia * dx + ib * dy, vy = ib * dx + ic * dy;
          gmx -= w * gam * vx;
          gmy -= w * gam * vy;
          Gxx -= 0.5 * w * gam * (vx * vx - ia);
          Gxy -= 0.5 * w * gam * (vx * vy - ib);
          Gyy -= 0.5 * w * gam * (vy * vy - ic);
          gl -= w * (gam - pi);
        }
        double s = grad_out ? grad_out[idx] : 1.0;
        gr[0] = s * gmx;
        gr[1] = s * gmy;
        gr[2] = s * 2.0 * (Gxx * l11 + Gxy * l21);
        gr[3] = s * 2.0 * (Gxy * l11 + Gyy * l21);
        gr[4] = s * 2.0 * (Gyy * l22);
        gr[5] = s * gl;
      }
      if (grad) gamma_put(grad, pl, idx, gr);
      if (nll) nll[idx] = loss;
    }
    free(T);
  }
}

/* ------------------------------------------------------------------------- */
/* The first-bounce estimator the guided samples feed (Eq. (1) estimated by
 * Monte Carlo with the density D of Eq. (2)): per pixel the mean over its
 * samples of f_r(w) L(w) cos(theta) / D(w), a null sample (strategy 0, 3 or
 * 4) contributing zero.  Pixels with omega_o below the surface give 0. */
void orc_estimate(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
                  const double *pdf_mix, const uint8_t *strategy, const double *radiance, double *out,
                  orc_rect r) {
  const int64_t pl = (int64_t)v->height * v->pitch;
  const int64_t spl = (int64_t)spp * pl;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      const pixel_t px = load_pixel(P, v, idx);
      double acc = 0.0;
      if (px.valid) {
        for (int s = 0; s < spp; ++s) {
          const int64_t o = (int64_t)s * pl + idx;
          if (!(strategy[o] == 1 || strategy[o] == 2) || !(pdf_mix[o] > 0.0)) continue;
          double w[3] = {dir[o], dir[spl + o], dir[2 * spl + o]}, l[3];
          normalize3(w);
          to_local(&px.f, w, l);
          if (l[2] <= 0.0) continue;
          acc += brdf_f(px.wo, l, px.alpha, px.albedo, (double)P->f0) * radiance[o] * l[2] / pdf_mix[o];
        }
        acc /= spp;
      }
      out[idx] = acc;
    }
  }
}

/* Reference value of the same integral, L_o = int f_r L cos dw over the upper
 * hemisphere, for a list of pixels: Monte Carlo in FP64 with n samples per
 * pixel drawn from the equal mixture of BRDF sampling and sampling of each
 * visible spherical-Gaussian light lobe (balance heuristic: every sample is
 * weighted by the mixture density).  An SG lobe exp(lambda (w.xi - 1)) is
 * sampled exactly: cos = 1 + ln(u + (1 - u) e^(-2 lambda)) / lambda about xi,
 * with density lambda exp(lambda (w.xi - 1)) / (2 pi (1 - e^(-2 lambda))).
 * Random words: Philox4x32-10 with counter (pixel, frame, 7 * 2^16 + sample,
 * view), one call per sample.  Returns the mean and its standard error. */
static double sg_pdf(const double w[3], const double ax[3], double lambda) {
  return lambda * exp(lambda * (dot3(w, ax) - 1.0)) / (2.0 * PI * (1.0 - exp(-2.0 * lambda)));
}

void orc_reference(const orc_params *P, const orc_view *v, int32_t n_lights, const float *lights,
                   double ambient, const uint8_t *vis, int32_t n_samples, int64_t n_px, const int64_t *px_index,
                   double *mean, double *stderr_out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n_px; ++i) {
    const int64_t idx = px_index[i];
    const int64_t y = idx / v->pitch, x = idx % v->pitch;
    const pixel_t px = load_pixel(P, v, idx);
    if (!px.valid) {
      mean[i] = 0.0;
      stderr_out[i] = 0.0;
      continue;
    }
    double ax[8][3], lam[8], cl[8];
    int m = 0;
    for (int k = 0; k < n_lights && k < 8; ++k) {
      if (!((vis[idx] >> k) & 1u)) continue;
      const float *lt = lights + 5 * k;
      ax[m][0] = lt[0]; ax[m][1] = lt[1]; ax[m][2] = lt[2];
      normalize3(ax[m]);
      lam[m] = lt[3];
      cl[m] = lt[4];
      ++m;
    }
    const int J = 1 + m;
    double s1 = 0.0, s2 = 0.0;
    for (int n = 0; n < n_samples; ++n) {
      uint32_t wds[4];
      rng_words(P, (uint32_t)(y * v->width + x), 7u, (uint32_t)n, wds);
      const double u0 = uniform24(wds[0]), u1 = uniform24(wds[1]), u2 = uniform24(wds[2]),
                   u3 = uniform24(wds[3]);
      int j = (int)(u0 * J);
      if (j >= J) j = J - 1;
      double l[3], w[3];
      int ok = 1;
      if (j == 0) {
        ok = brdf_sample(px.wo, px.alpha, (double)P->s_diffuse, u1, u2, u3, l, NULL);
        if (ok) {
          normalize3(l);
          to_world(&px.f, l, w);
        }
      } else {
        const int k = j - 1;
        const double c = 1.0 + log(u1 + (1.0 - u1) * exp(-2.0 * lam[k])) / lam[k];
        const double sn = sqrt(fmax(0.0, 1.0 - c * c)), phi = 2.0 * PI * u2;
        double t[3], b[3];
        onb(ax[k], t, b);
        for (int q = 0; q < 3; ++q) w[q] = c * ax[k][q] + sn * (cos(phi) * t[q] + sin(phi) * b[q]);
        normalize3(w);
        to_local(&px.f, w, l);
        ok = l[2] > 0.0;
      }
      double val = 0.0;
      if (ok && l[2] > 0.0) {
        double q = brdf_pdf(px.wo, l, px.alpha, (double)P->s_diffuse);
        double L = ambient;
        for (int k = 0; k < m; ++k) {
          q += sg_pdf(w, ax[k], lam[k]);
          L += cl[k] * exp(lam[k] * (dot3(w, ax[k]) - 1.0));
        }
        q /= J;
        if (q > 0.0) val = brdf_f(px.wo, l, px.alpha, px.albedo, (double)P->f0) * L * l[2] / q;
      }
      s1 += val;
      s2 += val * val;
    }
    const double mu = s1 / n_samples;
    mean[i] = mu;
    stderr_out[i] = sqrt(fmax(0.0, s2 / n_samples - mu * mu) / n_samples);
  }
}

/* ------------------------------------------------------------------------- */
/* K Gaussian lobes per pixel (the single lobe of Eq. (2) generalised; the
 * paper names one 2-D Gaussian as the limit of its model, Sec. 4.1):
 *   D(w) = sum_j pi_j N_j(M^-1 w) / (2 pi) + (1 - sum_j pi_j) p_b(w).
 * State planes [6K + 2]: lobe j at 6j: (mu_x, mu_y, S_xx, S_xy, S_yy, pi_j),
 * then W and k.  Readings of this extension: a new model's lobes share
 * Sigma = I/12 and pi_init/K but start at distinct means
 * mu_j = (0.5 + (j - (K-1)/2) / 4, 0.5) (identical lobes would stay
 * identical under EM; the means are dyadic, the same numbers in any
 * precision); zeta picks lobe j when it falls in [c_j, c_j + pi_j)
 * with c_j the sum of the earlier pi, else the BRDF; each lobe is merged with
 * its own evidence B1_j like the single lobe; the clamp raises each weight to
 * at least pi_lo / (4K) (a lobe at zero weight would never gain evidence
 * again) and then scales them so their sum lies in [pi_lo, pi_hi]. */
#define MAXK 4

static int nch_k(int K) { return 6 * K + 2; }

static void reset_k(const orc_params *P, int K, double *g) {
  for (int j = 0; j < K; ++j) {
    double *l = g + 6 * j;
    l[0] = 0.5 + 0.25 * (j - 0.5 * (K - 1));
    l[1] = 0.5;
    l[2] = 1.0 / 12.0; l[3] = 0.0; l[4] = 1.0 / 12.0;
    l[5] = (double)P->pi_init / K;
  }
  g[6 * K] = 0.0;
  g[6 * K + 1] = 0.0;
}

static double total_pi_k(const double *g, int K) {
  double t = 0.0;
  for (int j = 0; j < K; ++j) t += g[6 * j + 5];
  return t;
}

/* lobe weights used for sampling and D: zero while k = 0 or unguided */
static int guided_k(const pixel_t *px, const double *g, int K) { return px->guided && g[6 * K + 1] >= 1.0; }

static double mixture_k(const orc_params *P, const pixel_t *px, const double *g, int K, const double l[3],
                        double *pb_out) {
  double pb = 0.0, D = 0.0;
  if (px->valid && l[2] > 0.0) {
    pb = brdf_pdf(px->wo, l, px->alpha, (double)P->s_diffuse);
    double u[2];
    hemi2sq(l, u);
    double tot = 0.0;
    if (guided_k(px, g, K)) {
      for (int j = 0; j < K; ++j) {
        gauss_t G = gauss_setup(g + 6 * j, (double)P->eps_sigma);
        D += g[6 * j + 5] * (gauss_pdf_sq(&G, u) / (2.0 * PI));
        tot += g[6 * j + 5];
      }
    }
    D += (1.0 - tot) * pb;
  }
  if (pb_out) *pb_out = pb;
  return D;
}

void orc_reproject_k(const orc_params *P, int32_t K, const orc_view *cur, const orc_view *prev,
                     const double *gamma_prev, double *gamma_out, int32_t *src_index, orc_rect r) {
  const int NC = nch_k(K);
  const int64_t pl = (int64_t)cur->height * cur->pitch;
  const int64_t ppl = prev ? (int64_t)prev->height * prev->pitch : 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * cur->pitch + x;
      double g[6 * MAXK + 2];
      int32_t src = -1;
      pixel_t px = load_pixel(P, cur, idx);
      int keep = (P->frame > 0) && gamma_prev != NULL && prev != NULL && px.guided;
      if (keep && cur->disocc && cur->disocc[idx]) keep = 0;
      int qx = 0, qy = 0;
      if (keep) {
        float mx = cur->motion ? cur->motion[idx] : 0.0f;
        float my = cur->motion ? cur->motion[pl + idx] : 0.0f;
        float fx = ((float)x + 0.5f) - mx, fy = ((float)y + 0.5f) - my;
        if (fx >= 0.0f && fy >= 0.0f && fx < (float)prev->width && fy < (float)prev->height) {
          qx = (int)floorf(fx);
          qy = (int)floorf(fy);
        } else {
          keep = 0;
        }
      }
      int64_t qidx = 0;
      if (keep) {
        qidx = (int64_t)qy * prev->pitch + qx;
        float zp = cur->depth[idx], zq = prev->depth[qidx];
        if (fabsf(zp - zq) > P->tau_depth * zp) keep = 0;
        const float *n = cur->normal, *m = prev->normal;
        float nd = dot3f(n[idx], n[pl + idx], n[2 * pl + idx], m[qidx], m[ppl + qidx], m[2 * ppl + qidx]);
        if (nd < P->tau_normal) keep = 0;
      }
      if (keep) {
        for (int c = 0; c < NC; ++c) {
          g[c] = gamma_prev[c * ppl + qidx];
          if (!isfinite(g[c])) keep = 0;
        }
      }
      if (keep) {
        int same = 1;
        for (int c = 0; c < 3; ++c)
          if (cur->normal[c * pl + idx] != prev->normal[c * ppl + qidx]) same = 0;
        if (!same) {
          frame_t fq = make_frame(prev->normal, ppl, qidx);
          for (int j = 0; j < K && keep; ++j) {
            double *l = g + 6 * j;
            double mu[2] = {fmin(fmax(l[0], 0.0), 1.0), fmin(fmax(l[1], 0.0), 1.0)};
            double lq[3], w[3], lp[3];
            sq2hemi(mu, lq);
            to_world(&fq, lq, w);
            to_local(&px.f, w, lp);
            if (lp[2] <= 0.0) {
              keep = 0;
            } else {
              double u[2];
              hemi2sq(lp, u);
              l[0] = u[0];
              l[1] = u[1];
            }
          }
        }
      }
      if (keep)
        src = (int32_t)(qy * prev->width + qx);
      else
        reset_k(P, K, g);
      for (int c = 0; c < NC; ++c) gamma_out[c * pl + idx] = g[c];
      if (src_index) src_index[idx] = src;
    }
  }
}

void orc_sample_k(const orc_params *P, int32_t K, const orc_view *v, const double *gamma, int32_t spp,
                  double *dir, double *pdf_mix, double *pdf_brdf, uint8_t *strategy, double *margin,
                  orc_rect r) {
  const int NC = nch_k(K);
  const int W = v->width;
  const int64_t pl = (int64_t)v->height * v->pitch;
  const int64_t spl = (int64_t)spp * pl;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      double g[6 * MAXK + 2];
      for (int c = 0; c < NC; ++c) g[c] = gamma[c * pl + idx];
      const int gd = guided_k(&px, g, K);
      for (int s = 0; s < spp; ++s) {
        const int64_t o = (int64_t)s * pl + idx;
        uint8_t code = 0;
        double l[3] = {0, 0, 0}, mg = INFINITY;
        if (px.valid) {
          uint32_t w4[4];
          rng_words(P, (uint32_t)(y * W + x), 0, (uint32_t)s, w4);
          double zeta = uniform24(w4[0]), xl = uniform24(w4[1]);
          double x1 = uniform24(w4[2]), x2 = uniform24(w4[3]);
          int lobe = -1;
          double c = 0.0;
          if (gd) {
            for (int j = 0; j < K; ++j) {
              if (lobe < 0 && zeta >= c && zeta < c + g[6 * j + 5]) lobe = j;
              c += g[6 * j + 5];
              mg = fmin(mg, fabs(zeta - c));
            }
          }
          if (lobe >= 0) {
            gauss_t G = gauss_setup(g + 6 * lobe, (double)P->eps_sigma);
            double u[2];
            gauss_sample(&G, x1, x2, u);
            double dist = fmin(fmin(fabs(u[0]), fabs(1.0 - u[0])), fmin(fabs(u[1]), fabs(1.0 - u[1])));
            mg = fmin(mg, dist);
            if (u[0] >= 0.0 && u[0] <= 1.0 && u[1] >= 0.0 && u[1] <= 1.0) {
              sq2hemi(u, l);
              code = 2;
            } else {
              code = 3;
            }
          } else {
            double m2 = INFINITY;
            int ok = brdf_sample(px.wo, px.alpha, (double)P->s_diffuse, xl, x1, x2, l, &m2);
            mg = fmin(mg, m2);
            code = ok ? 1 : 4;
          }
        }
        double w[3] = {0, 0, 0}, D = 0.0, pb = 0.0;
        if (code == 1 || code == 2) {
          to_world(&px.f, l, w);
          D = mixture_k(P, &px, g, K, l, &pb);
        }
        for (int c = 0; c < 3; ++c) dir[c * spl + o] = w[c];
        pdf_mix[o] = D;
        pdf_brdf[o] = pb;
        strategy[o] = code;
        if (margin) margin[o] = mg;
      }
    }
  }
}

void orc_pdf_k(const orc_params *P, int32_t K, const orc_view *v, const double *gamma, int32_t n_per_px,
               const double *dirs, double *pdf_mix, orc_rect r) {
  const int NC = nch_k(K);
  const int64_t pl = (int64_t)v->height * v->pitch;
  const int64_t npl = (int64_t)n_per_px * pl;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      double g[6 * MAXK + 2];
      for (int c = 0; c < NC; ++c) g[c] = gamma[c * pl + idx];
      for (int s = 0; s < n_per_px; ++s) {
        const int64_t o = (int64_t)s * pl + idx;
        double w[3] = {dirs[o], dirs[npl + o], dirs[2 * npl + o]}, l[3];
        double D = 0.0;
        if (px.valid && dot3(w, w) > 0.0) {
          normalize3(w);
          to_local(&px.f, w, l);
          D = mixture_k(P, &px, g, K, l, NULL);
        }
        pdf_mix[o] = D;
      }
    }
  }
}

/* Online EM with K lobes: E-step responsibilities gam_j = pi_j p_gj / D
 * under the model's weights, per-lobe batch statistics (B1_j, mean, scatter
 * under the weights w gam_j), and the stepwise merge of each lobe with its
 * evidence; then the weight clamp of the extension's reading. */
/* The K-lobe update; with positions and hit distances (both non-NULL) every
 * training sample's direction is re-derived from its virtual point light:
 * y = x_q + t w_q, w = (y - x_p)/|y - x_p|, and w_q itself where t is not
 * finite (the sample left the scene; its light is at infinity). */
static void em_k_impl(const orc_params *P, int32_t K, const orc_view *v, int32_t spp, const double *dir,
                      const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
                      const float *position, const double *hit_dist, double *gamma, double *stats, orc_rect r) {
  const int NC = nch_k(K);
  const int64_t pl = (int64_t)v->height * v->pitch;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    tset_t *T = (tset_t *)malloc(sizeof(tset_t));
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      pixel_t px = load_pixel(P, v, idx);
      if (stats)
        for (int q = 0; q <= K; ++q) stats[q * pl + idx] = 0.0;
      if (!px.guided) continue;
      double g[6 * MAXK + 2];
      for (int c = 0; c < NC; ++c) g[c] = gamma[c * pl + idx];
      const double kk = g[6 * K + 1], Wv = g[6 * K];
      gather_set(P, v, spp, dir, pdf_brdf, strategy, radiance, x, y, (int)kk, T);
      if (position && hit_dist) {
        const double xp[3] = {position[idx], position[pl + idx], position[2 * pl + idx]};
        for (int j = 0; j < T->n; ++j) {
          const double t = hit_dist[T->rec[j]];
          if (!isfinite(t)) continue;
          const int64_t q = T->pix[j];
          double wq[3] = {T->dir[j][0], T->dir[j][1], T->dir[j][2]};
          normalize3(wq);
          for (int c = 0; c < 3; ++c) T->dir[j][c] = (double)position[c * pl + q] + t * wq[c] - xp[c];
        }
      }
      gauss_t G[MAXK];
      for (int j = 0; j < K; ++j) G[j] = gauss_setup(g + 6 * j, (double)P->eps_sigma);
      const double tot = total_pi_k(g, K);
      double u[MAX_SET][2], w[MAX_SET], gam[MAX_SET][MAXK];
      int n = 0;
      for (int j = 0; j < T->n; ++j) {
        double wn[3] = {T->dir[j][0], T->dir[j][1], T->dir[j][2]}, l[3];
        if (!(dot3(wn, wn) > 0.0) || !(T->psrc[j] > 0.0)) continue;
        normalize3(wn);
        to_local(&px.f, wn, l);
        if (l[2] <= 0.0) continue;
        hemi2sq(l, u[n]);
        w[n] = T->L[j] * brdf_f(px.wo, l, px.alpha, px.albedo, (double)P->f0) * l[2] / T->psrc[j];
        const double pb = brdf_pdf(px.wo, l, px.alpha, (double)P->s_diffuse);
        double a[MAXK], D = (1.0 - tot) * pb;
        for (int q = 0; q < K; ++q) {
          a[q] = g[6 * q + 5] * (gauss_pdf_sq(&G[q], u[n]) / (2.0 * PI));
          D += a[q];
        }
        for (int q = 0; q < K; ++q) gam[n][q] = D > 0.0 ? a[q] / D : 0.0;
        ++n;
      }
      double B0 = 0.0;
      for (int j = 0; j < n; ++j) B0 += w[j];
      if (stats) stats[idx] = B0;
      if (!(B0 > 0.0)) continue;
      const double eta = 1.0 / (kk + 1.0);
      const double sw = (1.0 - eta) * Wv + eta * B0;
      double pis[MAXK], ptot = 0.0;
      for (int q = 0; q < K; ++q) {
        double gq[MAX_SET], st[7];
        for (int j = 0; j < n; ++j) gq[j] = gam[j][q];
        orc_batch_stats(n, &u[0][0], w, gq, st);
        if (stats) stats[(q + 1) * pl + idx] = st[1];
        double *l = g + 6 * q;
        const double so = (1.0 - eta) * l[5] * Wv, sn = eta * st[1], sg = so + sn;
        if (sg > 0.0 && st[1] > 0.0) {
          const double al = so / sg, be = sn / sg;
          const double dx = l[0] - st[2], dy = l[1] - st[3];
          const double mux = al * l[0] + be * st[2], muy = al * l[1] + be * st[3];
          const double sxx = al * l[2] + be * st[4] + al * be * dx * dx;
          const double sxy = al * l[3] + be * st[5] + al * be * dx * dy;
          const double syy = al * l[4] + be * st[6] + al * be * dy * dy;
          l[0] = mux; l[1] = muy; l[2] = sxx; l[3] = sxy; l[4] = syy;
        }
        pis[q] = sg / sw;
        ptot += pis[q];
      }
      if (!(P->flags & ORC_NO_CLAMP)) {
        /* each weight raised to pi_lo / (4K) first, then all scaled so that
           their sum lies in [pi_lo, pi_hi] */
        const double floor_ = (double)P->pi_lo / (4.0 * K);
        double t = 0.0;
        for (int q = 0; q < K; ++q) {
          pis[q] = fmax(pis[q], floor_);
          t += pis[q];
        }
        const double scale = t > 0.0 ? fmin(fmax(t, (double)P->pi_lo), (double)P->pi_hi) / t : 0.0;
        for (int q = 0; q < K; ++q) pis[q] *= scale;
      }
      for (int q = 0; q < K; ++q) g[6 * q + 5] = pis[q];
      g[6 * K] = sw;
      g[6 * K + 1] = fmin(kk + 1.0, (double)P->k_max);
      for (int c = 0; c < NC; ++c) gamma[c * pl + idx] = g[c];
    }
    free(T);
  }
}

void orc_em_k(const orc_params *P, int32_t K, const orc_view *v, int32_t spp, const double *dir,
              const double *pdf_brdf, const uint8_t *strategy, const double *radiance, double *gamma,
              double *stats, orc_rect r) {
  em_k_impl(P, K, v, spp, dir, pdf_brdf, strategy, radiance, NULL, NULL, gamma, stats, r);
}

/* ------------------------------------------------------------------------- */
/* Positional reuse of virtual point lights (Fig. 2 caption, Sec. 3.1): the
 * trace stores with each sample the position y of its next surface
 * interaction, and a neighbour's sample trains pixel p along the direction
 * from x_p to that y, with the neighbour's radiance and source density (the
 * paper reuses the VPL as it is; no change-of-measure factor).  Positions
 * [3][H*pitch] are the pixels' world positions; hit_dist [spp][H*pitch] the
 * distance t to y along the sample's direction (+inf: no interaction). */
void orc_em_vpl(const orc_params *P, int32_t K, const orc_view *v, const float *position, int32_t spp,
                const double *dir, const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
                const double *hit_dist, double *gamma, double *stats, orc_rect r) {
  em_k_impl(P, K, v, spp, dir, pdf_brdf, strategy, radiance, position, hit_dist, gamma, stats, r);
}

/* Near-field stand-in for the trace (the workload of the positional reuse):
 * an emitting plane z = z_c above the surface, its emission a lattice of
 * Gaussian spots, lamp (i, j) at (sx, sy) with radius r and intensity c:
 *   E(y) = ambient + sum over the 3x3 lattice cells around y's cell of
 *          c exp(-|y_xy - s|^2 / (2 r^2)),
 * cell (i, j) = floor((y - origin) / period).  A live sample at x with world
 * direction w (normalised) hits the plane at t = (z_c - x_z) / w_z when
 * w_z > 0 (L = E(x + t w)); otherwise it leaves the scene (t = +inf, L =
 * ambient).  Null samples get L = 0 and t = 0. */
static double ceiling_emission(const orc_ceiling *C, double yx, double yy) {
  const double fx = (yx - C->x0) / C->period, fy = (yy - C->y0) / C->period;
  double E = C->ambient;
  /* no lamp lies within one cell of a point outside [-1, n + 1) */
  if (!(fx >= -1.0 && fx < C->nx + 1.0 && fy >= -1.0 && fy < C->ny + 1.0)) return E;
  const int ci = (int)floor(fx), cj = (int)floor(fy);
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      const int i = ci + di, j = cj + dj;
      if (i < 0 || j < 0 || i >= C->nx || j >= C->ny) continue;
      const float *l = C->lamps + 4 * ((int64_t)j * C->nx + i);
      const double dx = yx - l[0], dy = yy - l[1], rr = (double)l[2] * l[2];
      E += (double)l[3] * exp(-(dx * dx + dy * dy) / (2.0 * rr));
    }
  return E;
}

void orc_light_ceiling(const orc_ceiling *C, const orc_view *v, const float *position, int32_t spp,
                       const double *dir, const uint8_t *strategy, double *radiance, double *hit_dist,
                       orc_rect r) {
  const int64_t pl = (int64_t)v->height * v->pitch;
  const int64_t spl = (int64_t)spp * pl;
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = r.y0; y < r.y1; ++y) {
    for (int x = r.x0; x < r.x1; ++x) {
      const int64_t idx = (int64_t)y * v->pitch + x;
      const double xp[3] = {position[idx], position[pl + idx], position[2 * pl + idx]};
      for (int s = 0; s < spp; ++s) {
        const int64_t o = (int64_t)s * pl + idx;
        double L = 0.0, t = 0.0;
        if (strategy[o] == 1 || strategy[o] == 2) {
          double w[3] = {dir[o], dir[spl + o], dir[2 * spl + o]};
          normalize3(w);
          if (w[2] > 0.0) {
            t = (C->z - xp[2]) / w[2];
            L = ceiling_emission(C, xp[0] + t * w[0], xp[1] + t * w[1]);
          } else {
            t = INFINITY;
            L = C->ambient;
          }
        }
        radiance[o] = L;
        hit_dist[o] = t;
      }
    }
  }
}

/* Reference value of int f_r E(y(w)) cos dw for a list of pixels under the
 * ceiling: Monte Carlo in FP64 with n BRDF-sampling draws per pixel (Philox
 * counter (pixel, frame, 7 * 2^16 + sample, view)); null draws count zero.
 * Returns the mean and its standard error. */
void orc_reference_ceiling(const orc_params *P, const orc_view *v, const float *position, const orc_ceiling *C,
                           int32_t n_pixels, const int64_t *pixels, int64_t n, double *mean, double *stderr_out) {
  const int64_t pl = (int64_t)v->height * v->pitch;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t i = 0; i < n_pixels; ++i) {
    const int64_t pix = pixels[i];
    const int x = (int)(pix % v->width), y = (int)(pix / v->width);
    const int64_t idx = (int64_t)y * v->pitch + x;
    const pixel_t px = load_pixel(P, v, idx);
    const double xp[3] = {position[idx], position[pl + idx], position[2 * pl + idx]};
    double s1 = 0.0, s2 = 0.0;
    if (px.valid) {
      for (int64_t k = 0; k < n; ++k) {
        uint32_t w4[4];
        rng_words(P, (uint32_t)pix, 7, (uint32_t)k, w4);
        double l[3], m2;
        if (!brdf_sample(px.wo, px.alpha, (double)P->s_diffuse, uniform24(w4[1]), uniform24(w4[2]),
                         uniform24(w4[3]), l, &m2))
          continue;
        const double pb = brdf_pdf(px.wo, l, px.alpha, (double)P->s_diffuse);
        if (!(pb > 0.0)) continue;
        double w[3];
        to_world(&px.f, l, w);
        double E = C->ambient;
        if (w[2] > 0.0) {
          const double t = (C->z - xp[2]) / w[2];
          E = ceiling_emission(C, xp[0] + t * w[0], xp[1] + t * w[1]);
        }
        const double f = brdf_f(px.wo, l, px.alpha, px.albedo, (double)P->f0) * E * l[2] / pb;
        s1 += f;
        s2 += f * f;
      }
    }
    const double m = s1 / (double)n;
    mean[i] = m;
    stderr_out[i] = sqrt(fmax(s2 / (double)n - m * m, 0.0) / (double)n);
  }
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel regions (timing of the baseline). */
void orc_set_num_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
