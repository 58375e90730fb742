/*
 * FP64 CPU oracle for screen-space path guiding with per-pixel parametric
 * mixture models (Derevyannykh, "Real-Time Path-Guiding Based on Parametric
 * Mixture Models", arXiv 2112.09728).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain definition that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or helper with the HIP library: every formula here is written
 * out again from the paper (and from the published methods it names), in
 * double precision, one pixel at a time, in the order the paper describes.
 *
 * Conventions (all arrays are caller-owned host memory):
 *   - planes are row-major with a row pitch in elements; a [c][H*pitch] array
 *     holds channel c of pixel (x, y) at c*H*pitch + y*pitch + x;
 *   - per-sample arrays hold sample s of pixel (x, y) at (s*H + y)*pitch + x,
 *     and a 3-vector array has 3 such planes;
 *   - the mixture state Gamma of a pixel has 8 channels
 *       0 mu_x, 1 mu_y, 2 Sigma_xx, 3 Sigma_xy, 4 Sigma_yy, 5 pi, 6 W, 7 k;
 *   - strategy codes: 0 no sample (invalid pixel), 1 BRDF sample,
 *     2 guided sample, 3 guided draw outside the unit square (null sample),
 *     4 BRDF draw below the horizon (null sample);
 *   - frame-level calls compute only the pixels of `rect` (x0 <= x < x1,
 *     y0 <= y < y1) and read whatever neighbours they need from the full
 *     arrays, so a crop gives exactly the full-frame values on that crop.
 */
#ifndef PMM_ORACLE_H
#define PMM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_view {
  int32_t width, height, pitch;
  const float *normal;    /* [3][H*pitch] shading normal, world space          */
  const float *view_dir;  /* [3][H*pitch] omega_o, towards the camera          */
  const float *depth;     /* [H*pitch]                                         */
  const float *roughness; /* [H*pitch]; GGX alpha = roughness^2                */
  const float *albedo;    /* [H*pitch] diffuse albedo                          */
  const float *motion;    /* [2][H*pitch] in pixels, current minus previous;
                             NULL means zero motion                            */
  const uint8_t *disocc;  /* [H*pitch] nonzero = disoccluded; NULL = none      */
} orc_view;

enum { ORC_NO_CLAMP = 1, ORC_STALE_RESET = 4 };

typedef struct orc_params {
  uint64_t seed;
  uint32_t frame, view;
  int32_t k_max;        /* maximum training epoch kMax                         */
  int32_t radius;       /* neighbour window radius R                           */
  float pi_init;        /* mixing weight of a new model                        */
  float pi_lo, pi_hi;   /* clamp range of pi                                   */
  float eps_sigma;      /* covariance floor epsilon                            */
  float tau_depth;      /* relative depth tolerance of reprojection            */
  float tau_normal;     /* minimum normal dot product of reprojection          */
  float rough_min;      /* minimum roughness for guiding                       */
  float s_diffuse;      /* probability of the diffuse lobe in BRDF sampling   */
  float f0;             /* Schlick reflectance at normal incidence             */
  uint32_t flags;       /* ORC_NO_CLAMP, ORC_STALE_RESET                        */
  float stale_tau;      /* with ORC_STALE_RESET: reset a trained model whose
                           weighted log-likelihood of the batch is below a new
                           model's by more than stale_tau per unit weight     */
} orc_params;

typedef struct orc_rect { int32_t x0, y0, x1, y1; } orc_rect;

/* ---- primitives (exported for the pins) ---------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_sq2hemi_n(int64_t n, const double *u /*[n][2]*/, double *w /*[n][3]*/);
void orc_hemi2sq_n(int64_t n, const double *w /*[n][3]*/, double *u /*[n][2]*/);
void orc_onb_n(int64_t n, const double *nrm /*[n][3]*/, double *t, double *b);
/* BRDF in the local frame (z = normal). */
void orc_brdf_f_n(int64_t n, const double *wo, const double *wi, const double *alpha,
                  const double *albedo, double f0, double *out);
void orc_brdf_pdf_n(int64_t n, const double *wo, const double *wi, const double *alpha,
                    double s_diffuse, double *out);
void orc_brdf_sample_n(int64_t n, const double *wo, const double *alpha, double s_diffuse,
                       const double *xi /*[n][3] = (xi_l, xi_1, xi_2)*/,
                       double *wi /*[n][3]*/, int32_t *valid);
/* Gaussian on the unit square; g = (mu_x, mu_y, S_xx, S_xy, S_yy). */
void orc_gauss_pdf_sq_n(const double g[5], double eps, int64_t n, const double *u, double *out);
void orc_gauss_sample_n(const double g[5], double eps, int64_t n, const double *xi /*[n][2]*/,
                        double *u /*[n][2]*/);
/* Solid-angle density of the guided lobe for local directions. */
void orc_guide_pdf_n(const double g[5], double eps, int64_t n, const double *w, double *out);
/* Weighted batch statistics: out = (B0, B1, m_x, m_y, S_xx, S_xy, S_yy). */
void orc_batch_stats(int64_t n, const double *u, const double *w, const double *gam, double out[7]);
/* Stepwise M-step merge of one pixel's state with batch statistics. */
void orc_merge(const orc_params *P, const double g_in[8], const double stats[7], double g_out[8]);
/* Training set of one pixel: writes the candidate picks (own samples first)
   into q_index / s_index with keep = 1 when the candidate is used; returns the
   number of candidates written. */
int32_t orc_training_set(const orc_params *P, const orc_view *v, int32_t spp,
                         const uint8_t *strategy, int32_t x, int32_t y, int32_t k,
                         int32_t *q_index, int32_t *s_index, int32_t *keep, int32_t cap);

/* ---- frame-level steps ------------------------------------------------------ */
void orc_reproject(const orc_params *P, const orc_view *cur, const orc_view *prev,
                   const double *gamma_prev, double *gamma_out, int32_t *src_index,
                   orc_rect r);
void orc_sample(const orc_params *P, const orc_view *v, const double *gamma, int32_t spp,
                double *dir, double *pdf_mix, double *pdf_brdf, uint8_t *strategy,
                double *margin, orc_rect r);
void orc_pdf(const orc_params *P, const orc_view *v, const double *gamma, int32_t n_per_px,
             const double *dir, double *pdf_mix, double *pdf_guide, double *pdf_brdf,
             orc_rect r);
void orc_light(int32_t n_lights, const float *lights /*[n][5] axis xyz, sharpness, intensity*/,
               double ambient, const uint8_t *vis, int32_t width, int32_t height,
               int32_t pitch, int32_t spp, const double *dir, const uint8_t *strategy,
               double *radiance, orc_rect r);
/* stats (nullable) [2][H*pitch]: B0 and B1 of the pixel's last E-step. */
void orc_em(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
            const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
            double *gamma, int32_t iterations, int32_t batch, double *stats, orc_rect r);
void orc_nll(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
             const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
             const double *theta, const double *grad_out, double *grad, double *nll,
             orc_rect r);
/* Margin of the stale-history decision per pixel, (l_m - l_r)/sum w +
 * stale_tau (negative = reset), NaN where it does not apply. */
void orc_stale_margin(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
                      const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
                      const double *gamma, double *out, orc_rect r);
/* First-bounce estimate per pixel: mean over samples of f_r L cos / D
 * (null samples contribute zero). */
void orc_estimate(const orc_params *P, const orc_view *v, int32_t spp, const double *dir,
                  const double *pdf_mix, const uint8_t *strategy, const double *radiance, double *out,
                  orc_rect r);
/* Reference value of int f_r L cos over the hemisphere for listed pixels
 * (flat indices y*pitch + x): FP64 Monte Carlo with n_samples per pixel from
 * the mixture of BRDF and light-lobe sampling; mean and standard error. */
void orc_reference(const orc_params *P, const orc_view *v, int32_t n_lights, const float *lights,
                   double ambient, const uint8_t *vis, int32_t n_samples, int64_t n_px, const int64_t *px_index,
                   double *mean, double *stderr_out);
/* K Gaussian lobes per pixel (K <= 4): state planes [6K + 2] (per lobe
 * mu_x, mu_y, S_xx, S_xy, S_yy, pi_j; then W, k).  orc_em_k's stats (nullable)
 * [K+1][H*pitch] receive B0 and each lobe's B1_j of the E-step. */
void orc_reproject_k(const orc_params *P, int32_t K, const orc_view *cur, const orc_view *prev,
                     const double *gamma_prev, double *gamma_out, int32_t *src_index, orc_rect r);
void orc_sample_k(const orc_params *P, int32_t K, const orc_view *v, const double *gamma, int32_t spp,
                  double *dir, double *pdf_mix, double *pdf_brdf, uint8_t *strategy, double *margin,
                  orc_rect r);
void orc_pdf_k(const orc_params *P, int32_t K, const orc_view *v, const double *gamma, int32_t n_per_px,
               const double *dirs, double *pdf_mix, orc_rect r);
void orc_em_k(const orc_params *P, int32_t K, const orc_view *v, int32_t spp, const double *dir,
              const double *pdf_brdf, const uint8_t *strategy, const double *radiance, double *gamma,
              double *stats, orc_rect r);
/* Positional reuse of virtual point lights and its near-field workload. */
typedef struct orc_ceiling {
  double z, period, x0, y0, ambient; /* plane height, lattice period and origin */
  int32_t nx, ny;                    /* lattice cells                            */
  const float *lamps;                /* [ny][nx][4]: sx, sy, r, c                */
} orc_ceiling;
void orc_em_vpl(const orc_params *P, int32_t K, const orc_view *v, const float *position, int32_t spp,
                const double *dir, const double *pdf_brdf, const uint8_t *strategy, const double *radiance,
                const double *hit_dist, double *gamma, double *stats, orc_rect r);
void orc_light_ceiling(const orc_ceiling *C, const orc_view *v, const float *position, int32_t spp,
                       const double *dir, const uint8_t *strategy, double *radiance, double *hit_dist,
                       orc_rect r);
void orc_reference_ceiling(const orc_params *P, const orc_view *v, const float *position, const orc_ceiling *C,
                           int32_t n_pixels, const int64_t *pixels, int64_t n, double *mean, double *stderr_out);
int32_t orc_num_threads(void);
void orc_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
