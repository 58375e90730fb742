/*
 * libpmmguide: screen-space path guiding with per-pixel parametric mixture
 * models on AMD Instinct MI355X (gfx950).
 *
 * Method: M. Derevyannykh, "Real-Time Path-Guiding Based on Parametric
 * Mixture Models", arXiv 2112.09728.  Each pixel keeps a model Gamma of 8
 * values (Abstract): a 2-D Gaussian N(mu, Sigma) on the unit square, carried to
 * the hemisphere by the Shirley-Chiu area-preserving map M, mixed with the
 * BRDF by a weight pi (Eq. (2)).  Per frame the library
 *   1. reprojects Gamma from the previous frame through the motion vectors
 *      with nearest-neighbour filtering and depth/normal rejection, and
 *      re-expresses it in the current surface's hemisphere   (Sec. 3.1)
 *   2. samples first-bounce directions: zeta < pi takes Box-Muller + N(mu,
 *      Sigma) + M, otherwise the BRDF, and evaluates the one-sample MIS
 *      density D of each direction                          (Sec. 3.1, Eq. (2))
 *   3. trains Gamma by an online, radiance-weighted EM step from the pixel's
 *      own and neighbouring BRDF-strategy samples          (Sec. 3.2, Sec. 4.2)
 *
 * Conventions shared by every call
 *   - Every buffer is caller-owned DEVICE memory (e.g. a torch tensor's
 *     data_ptr()), except the structs themselves and pg_lights, which are
 *     read on the host during the call.  The library allocates nothing.
 *   - Planes are row-major with row pitch `pitch` (elements).  Channel c of
 *     pixel (x, y) of a [C][H*pitch] array is at c*H*pitch + y*pitch + x.
 *   - Per-sample arrays hold sample s of pixel (x, y) at (s*H + y)*pitch + x;
 *     the direction array has 3 such planes, [3][spp*H*pitch].
 *   - Gamma has 8 planes [8][H*pitch] in the storage type of pg_gamma.dtype:
 *       0 mu_x, 1 mu_y, 2 Sigma_xx, 3 Sigma_xy, 4 Sigma_yy, 5 pi, 6 W, 7 k
 *     (k the training epoch, W the running evidence).  All arithmetic is
 *     FP32 whatever the storage type; stores round to nearest-even and W
 *     saturates at the format's largest finite value.  FP16 and BF16
 *     states hold mu_x - 1/2 and mu_y - 1/2 in planes 0 and 1 (the means
 *     cluster near the centre of the square, where values near zero keep
 *     more significant bits); FP32 states hold mu.  k is stored in the
 *     state's type too, so every call given an FP16 state rejects k_max >
 *     2048 and every call given a BF16 state k_max > 256 (PG_ERR_ARG): above
 *     those the type no longer holds every integer up to k_max.
 *   - Strategy codes: 0 no sample (omega_o below the surface), 1 BRDF
 *     sample, 2 guided sample, 3 guided draw outside the unit square (null),
 *     4 BRDF draw below the horizon (null).  Null samples record zeros.
 *   - Calls enqueue work on `stream` (a hipStream_t; NULL = the null stream)
 *     and return without synchronising.  Results are bit-identical run to
 *     run and for every tile shape.
 *   - Errors: argument problems are found on the host before any launch and
 *     return PG_ERR_ARG (null required pointer, non-positive sizes, pitch <
 *     width, spp outside [1, 8], unknown dtype, forbidden aliasing);
 *     PG_ERR_UNSUPPORTED marks a valid request this build does not handle
 *     (radius other than 3, width or height above 16384, a pitch of 2^24
 *     or more, sizes beyond the 32-bit index range); a failed
 *     launch returns PG_ERR_HIP.  pg_last_error() then describes the error.
 *     Numeric trouble is never an error: a non-finite history starts a new
 *     model.
 */
#ifndef PMMGUIDE_H
#define PMMGUIDE_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum pg_status {
  PG_OK = 0,
  PG_ERR_ARG = 1,
  PG_ERR_UNSUPPORTED = 2,
  PG_ERR_HIP = 3
} pg_status;

typedef enum pg_dtype { PG_F32 = 0, PG_F16 = 1, PG_BF16 = 2 } pg_dtype;

enum {
  PG_NO_CLAMP = 1,    /* do not clamp pi after the M-step                     */
  PG_EM_BATCH = 2,    /* pg_em_update: iterate plain batch EM on a fixed set  */
  PG_STALE_RESET = 4  /* online update: reset a stale history (stale_tau)     */
};

/* One view's G-buffer (Sec. 3.1 "rasterized G-Buffer"); all FP32 device planes. */
typedef struct pg_view {
  int32_t width, height, pitch;
  const float *normal;    /* [3][H*pitch] shading normal, world space           */
  const float *view_dir;  /* [3][H*pitch] omega_o, unit, towards the camera     */
  const float *depth;     /* [H*pitch]                                          */
  const float *roughness; /* [H*pitch]; GGX alpha = roughness^2                 */
  const float *albedo;    /* [H*pitch] diffuse albedo                           */
  const float *motion;    /* [2][H*pitch] px, current position minus previous;
                             NULL = no motion                                   */
  const uint8_t *disocc;  /* [H*pitch] nonzero = disoccluded; NULL = none       */
} pg_view;

/* Per-pixel model planes, [8][H*pitch] of the view they belong to. */
typedef struct pg_gamma {
  int32_t dtype; /* pg_dtype */
  void *data;
} pg_gamma;

/* Sample records ("VPL" buffer Pi of Fig. 2, without the hit position). */
typedef struct pg_samples {
  int32_t spp;      /* samples per pixel, 1..8                                  */
  float *dir;       /* [3][spp*H*pitch] world direction                         */
  float *pdf_mix;   /* [spp*H*pitch] mixture density D(dir)                     */
  float *pdf_brdf;  /* [spp*H*pitch] BRDF-sampling density p_b(dir)             */
  uint8_t *strategy;/* [spp*H*pitch] strategy code                              */
  float *radiance;  /* [spp*H*pitch] incident radiance along dir               */
} pg_samples;

/* Method constants and per-call counters.  pg_params_default() fills the
 * values used throughout this library; the paper fixes pi_init = 0.05 and
 * k = 0 for a new model (Sec. 3.1), the clamp [0.05, 0.95] (Sec. 3.2) and
 * N(k) = (1 - k/kMax)*15 + 5 neighbour picks (Sec. 4.2); the others are this
 * library's readings where the paper gives no value. */
typedef struct pg_params {
  uint64_t seed;    /* RNG key                                                   */
  uint32_t frame;   /* frame index t: frame 0 starts every model anew            */
  uint32_t view;    /* view index (RNG counter word)                             */
  int32_t k_max;    /* kMax, 16                                                  */
  int32_t radius;   /* neighbour window radius R, 3 (7x7 window)                 */
  float pi_init;    /* 0.05                                                       */
  float pi_lo, pi_hi; /* 0.05, 0.95                                               */
  float eps_sigma;  /* covariance floor, 2.5e-4                                  */
  float tau_depth;  /* reject if |z - z_prev| > tau_depth * z, 0.1              */
  float tau_normal; /* reject if n . n_prev < tau_normal, 0.9                    */
  float rough_min;  /* guide only if roughness >= rough_min, 0.1                 */
  float s_diffuse;  /* probability of the cosine lobe in BRDF sampling, 0.5      */
  float f0;         /* Schlick reflectance at normal incidence, 0.04             */
  uint32_t flags;   /* PG_NO_CLAMP | PG_EM_BATCH | PG_STALE_RESET                 */
  int32_t tile_w, tile_h; /* training tile; 0 = library default; results do not
                             depend on it                                         */
  float stale_tau;  /* with PG_STALE_RESET: nats per unit weight (see
                       pg_em_update); ignored otherwise                           */
} pg_params;

/* Analytic stand-in for the traced incident radiance (the paper traces rays,
 * Fig. 2): L = ambient + sum_l V(p,l) c_l exp(lambda_l (w . xi_l - 1)). */
#define PG_MAX_LIGHTS 8
typedef struct pg_lights {
  int32_t count;                  /* <= PG_MAX_LIGHTS                          */
  float ambient;
  float light[PG_MAX_LIGHTS][5];  /* axis xi (unit, world), lambda, c          */
} pg_lights;

/* Fill *p with the library's constants (seed 0, frame 0, view 0). */
pg_status pg_params_default(pg_params *p);

/* Reprojection of Gamma (Sec. 3.1: NN fetch through motion vectors,
 * depth/normal stopping test, change of hemisphere; new model pi = 0.05,
 * k = 0).  For pixel p the source is q = floor(p + 1/2 - motion(p)); the model
 * restarts when frame == 0, p is disoccluded, q is outside the image,
 * |z(p) - z_prev(q)| > tau_depth z(p), n(p).n_prev(q) < tau_normal, a
 * channel of Gamma_prev(q) is not finite, or p is not guided (omega_o below
 * the surface or roughness < rough_min).  Otherwise Gamma_prev(q) is copied
 * and, when the normals differ, mu is moved so that M(mu) keeps its world
 * direction (the model restarts if that direction is below p's horizon).
 *   prev, prev_gamma: may be NULL only when frame == 0.
 *   out_gamma must not alias prev_gamma; both use cur's height and pitch.
 *   src_index (nullable) [H*pitch] int32: q.y*width_prev + q.x, or -1. */
pg_status pg_reproject(const pg_params *p, const pg_view *cur, const pg_view *prev,
                       pg_gamma prev_gamma, pg_gamma out_gamma, int32_t *src_index,
                       void *stream);

/* Guided sampling with one-sample MIS (Sec. 3.1 and Eq. (2)).  Sample s of
 * pixel (x, y) draws four words of Philox4x32-10 with counter
 * (y*width + x, frame, s, view) and key seed, giving zeta, xi_l, xi_1, xi_2
 * as (word >> 8) * 2^-24.  With pi_eff = pi when k >= 1 and the pixel is
 * guided (0 otherwise), zeta < pi_eff draws u = mu + L z (Box-Muller z,
 * Cholesky L of Sigma + eps I) and w = M(u) (null if u leaves [0,1]^2);
 * otherwise the BRDF is sampled with (xi_l, xi_1, xi_2).  Records the world
 * direction, D(w) = pi_eff N(M^-1 w)/(2 pi) + (1 - pi_eff) p_b(w), p_b(w) and
 * the strategy; out->radiance is not touched. */
pg_status pg_sample_mis(const pg_params *p, const pg_view *v, pg_gamma gamma,
                        const pg_samples *out, void *stream);

/* pg_reproject followed by pg_sample_mis in one launch: writes out_gamma
 * exactly as pg_reproject and the records exactly as pg_sample_mis would. */
pg_status pg_reproject_sample(const pg_params *p, const pg_view *cur, const pg_view *prev,
                              pg_gamma prev_gamma, pg_gamma out_gamma,
                              const pg_samples *out, void *stream);

/* Densities of given world directions (Eq. (2) under the same readings as
 * pg_sample_mis): for n_per_px directions per pixel, dir [3][n*H*pitch],
 * writes pdf_mix = D, and optionally pdf_guide = N(M^-1 w)/(2 pi) (the
 * unweighted guided density) and pdf_brdf = p_b.  Zero for pixels with
 * omega_o below the surface and for directions below the horizon. */
pg_status pg_pdf(const pg_params *p, const pg_view *v, pg_gamma gamma, int32_t n_per_px,
                 const float *dir, float *pdf_mix, float *pdf_guide, float *pdf_brdf,
                 void *stream);

/* Workload stand-in for the trace between sampling and training: writes
 * samples->radiance for strategies 1 and 2 (0 otherwise) from the analytic
 * light field; vis [H*pitch] holds bit l for light l.  `lights` is host
 * memory read during the call. */
pg_status pg_light_field(const pg_lights *lights, const pg_view *v, const uint8_t *vis,
                         const pg_samples *samples, void *stream);

/* Online weighted EM update of Gamma in place (Sec. 3.2, Sec. 4.2, Fig. 2).
 * For each guided pixel: training set = own samples with strategy 1 in
 * sample order, then N(k) = 5 + floor(15 (kMax - k)/kMax) picks with
 * replacement among the samples of the (2R+1)^2 - 1 surrounding pixels
 * (16-bit fields of Philox words, counter (y*width + x, frame,
 * 2^16 + m/8, view)), kept if inside the image and of strategy 1.
 * E-step per sample: u = M^-1(w), weight L f_r cos / p_b(source), posterior
 * gamma of the Gaussian against the BRDF under the model's pi.  M-step:
 * the batch mean/covariance merged with the state by eta = 1/(k+1) and the
 * evidence W; pi = clamp(.., pi_lo, pi_hi) unless PG_NO_CLAMP; k += 1 (at
 * most kMax).  An empty batch leaves the pixel unchanged.  The E-step sums
 * the training set in the order above, except for the online update from
 * spp 4, which sums the members drawn from sample planes below ceil(spp/2)
 * first and then the rest, each part in that order (a different rounding
 * order of the same sums; the tile never changes the result).
 * With PG_EM_BATCH in p->flags, `iterations` rounds of plain batch EM run on
 * the same training set (mu, Sigma, pi replaced; W and k kept); otherwise
 * `iterations` must be 1.  With PG_STALE_RESET (online update only), a
 * trained model (k >= 1) is first tested against its training set: with the
 * E-step densities, l_m = sum w log(pi p_g + (1 - pi) p_b) under the model
 * and l_r the same under a new model (the reset lobe and pi_init); when
 * l_m - l_r < -stale_tau sum w the model is reset before the E-step, so the
 * batch alone trains it (a reading of the stronger rejection of reprojected
 * models that Sec. 5 leaves open; the training set is the one drawn for the
 * model's k).  Reads samples->dir, pdf_brdf, strategy, radiance. */
pg_status pg_em_update(const pg_params *p, const pg_view *v, const pg_samples *in,
                       pg_gamma gamma_inout, int32_t iterations, void *stream);

/* Radiance-weighted negative log-likelihood of the mixture density D of
 * Eq. (2) over each pixel's EM training set (Sec. 3.2: the samples and
 * weights w = L f_r cos / p_src of pg_em_update's E-step), and its adjoint:
 *   NLL = -sum_j w_j log(pi N(M^-1 w_j)/(2 pi) + (1 - pi) p_b(w_j)),
 * the objective whose maximum-likelihood fit the EM update approaches, here
 * as a function a gradient method can minimise instead.  theta [8][H*pitch]
 * FP32 holds (mu_x, mu_y, l11, l21, l22, logit pi, unused, k) with
 * Sigma = L L^T; the Gaussian uses Sigma + eps I and k selects the number of
 * neighbour picks as in pg_em_update.  Writes nll [H*pitch] (nullable) and,
 * when grad_theta is not NULL, grad_theta = grad_out * dNLL/dtheta
 * ([8][H*pitch]; channels 6 and 7 are 0; grad_out NULL means 1).  theta and
 * the records are caller-owned device memory; PG_ERR_ARG when theta is NULL
 * or both outputs are NULL. */
pg_status pg_nll_backward(const pg_params *p, const pg_view *v, const pg_samples *in,
                          const float *theta, const float *grad_out, float *grad_theta,
                          float *nll, void *stream);

/* First-bounce estimate (the Monte Carlo estimator of the reflected radiance
 * of Eq. (1) with the sampling density D of Eq. (2)): estimate [H*pitch]
 * receives, per pixel, the mean over its samples of f_r(w) L(w) cos / D(w),
 * where a null sample (strategy 0, 3 or 4) or D = 0 counts zero, and 0 for a
 * pixel with omega_o below the surface.  Reads samples->dir, pdf_mix,
 * strategy and radiance and the view's normal, view_dir, roughness, albedo. */
pg_status pg_estimate(const pg_params *p, const pg_view *v, const pg_samples *in, float *estimate,
                      void *stream);

/* ---- K Gaussian lobes per pixel -------------------------------------------
 * The mixture of Eq. (2) with K Gaussian lobes instead of one (Sec. 4.1 names
 * the single lobe as the model's limit):
 *   D(w) = sum_j pi_j N_j(M^-1 w)/(2 pi) + (1 - sum_j pi_j) p_b(w).
 * Gamma is FP32 with 6K + 2 planes [6K+2][H*pitch]: lobe j at plane 6j holds
 * (mu_x, mu_y, Sigma_xx, Sigma_xy, Sigma_yy, pi_j), then W and k.  1 <= K <=
 * PG_MAX_LOBES.  Readings: a new model's lobes have Sigma = I/12, pi_init/K
 * and means (0.5 + (j - (K-1)/2) / 4, 0.5); zeta selects lobe j when it lies
 * in [c_j, c_j + pi_j) with c_j the sum of the earlier weights (the BRDF
 * otherwise); every lobe mean is carried by reprojection (a new model when
 * one falls below the horizon); each lobe is merged with its own evidence
 * like the single lobe; unless PG_NO_CLAMP, every weight is raised to
 * pi_lo/(4K) and all are scaled so that their sum lies in [pi_lo, pi_hi].
 * The random words, the training set and the BRDF strategy are those of the
 * single-lobe calls.  PG_EM_BATCH and PG_STALE_RESET are not supported
 * (PG_ERR_UNSUPPORTED); lobes outside [1, PG_MAX_LOBES] is PG_ERR_ARG, and
 * (6K + 2) * pitch * height must stay below 2^31 (PG_ERR_UNSUPPORTED). */
#define PG_MAX_LOBES 4

/* pg_reproject_sample with K lobes: out_gamma [6K+2][H*pitch] and the
 * records (dir, pdf_mix, pdf_brdf, strategy; radiance untouched).
 * prev and prev_gamma may be NULL only when frame == 0; prev must have
 * cur's width, height and pitch; out_gamma must not alias prev_gamma. */
pg_status pg_reproject_sample_lobes(const pg_params *p, int32_t lobes, const pg_view *cur,
                                    const pg_view *prev, const float *prev_gamma, float *out_gamma,
                                    const pg_samples *out, void *stream);

/* pg_em_update (online) with K lobes, in place on gamma_inout
 * [6K+2][H*pitch]: E-step posteriors gam_j = pi_j p_gj / D, per-lobe batch
 * statistics, the stepwise merge of every lobe and the weight clamp.
 * Reads samples->dir, pdf_brdf, strategy, radiance and the view's albedo. */
pg_status pg_em_update_lobes(const pg_params *p, int32_t lobes, const pg_view *v, const pg_samples *in,
                             float *gamma_inout, void *stream);

/* pg_pdf with K lobes: pdf_mix = D for n_per_px directions per pixel
 * (dir [3][n*H*pitch]); zero for pixels with omega_o below the surface and
 * directions below the horizon. */
pg_status pg_pdf_lobes(const pg_params *p, int32_t lobes, const pg_view *v, const float *gamma,
                       int32_t n_per_px, const float *dir, float *pdf_mix, void *stream);

/* ---- Positional reuse of virtual point lights -----------------------------
 * The trace stores with each sample the position y of its next surface
 * interaction (the VPL, Fig. 2 caption and Sec. 3.1); a neighbour's sample
 * then trains pixel p along the direction from p's own position x_p to y
 * rather than along the neighbour's direction, with the neighbour's radiance
 * and source density as they are (the paper reuses the VPL without a
 * change-of-measure factor).  y is given by the pixel positions and the hit
 * distance t of each sample: y = x_q + t w_q; a sample with t = +inf (no
 * interaction) trains along w_q. */

/* pg_em_update_lobes with positional reuse (K = lobes, 1 <= K <=
 * PG_MAX_LOBES; K = 1 is the single-lobe model, whose 8 planes are the FP32
 * layout of pg_gamma).  position [3][H*pitch] FP32: world position of each
 * pixel's surface point; hit_dist [spp][H*pitch] FP32 as written by
 * pg_light_ceiling (only entries of strategy-1 samples are read).  With every
 * hit distance +inf the result is that of pg_em_update_lobes. */
pg_status pg_em_update_vpl(const pg_params *p, int32_t lobes, const pg_view *v, const float *position,
                           const pg_samples *in, const float *hit_dist, float *gamma_inout, void *stream);

/* Near-field stand-in for the trace (workload of the positional reuse): an
 * emitting plane z = z above the surface whose emission is
 *   E(y) = ambient + sum over the 3x3 lamp cells around y of
 *          c exp(-|y_xy - s|^2 / (2 r^2)),
 * cell (i, j) = floor((y - origin) / period), lamp (i, j) = lamps[j][i] =
 * (sx, sy, r, c).  For each sample of strategy 1 or 2 with world direction w
 * (normalised): if w_z > 0, t = (z - x_z) / w_z and L = E(x + t w); else
 * t = +inf and L = ambient.  Other samples get L = 0 and t = 0.  Writes
 * samples->radiance and hit_dist [spp][H*pitch]. */
typedef struct pg_ceiling {
  float z, period, x0, y0, ambient;
  int32_t nx, ny;
  const float *lamps; /* [ny][nx][4] FP32 device memory, 16-byte aligned */
} pg_ceiling;
pg_status pg_light_ceiling(const pg_ceiling *c, const pg_view *v, const float *position,
                           const pg_samples *samples, float *hit_dist, void *stream);

/* ---- Batched frame: many views in a few launches -------------------------
 * One frame of n views of any size and spp (Sec. 3.1 and Sec. 3.2 for each
 * view, with the light-field stand-in between them) as an upload of a packed
 * table followed by launches over the tiles of all views: reprojection +
 * guided sampling + light field, then the online EM update (one launch per
 * spp group).
 * Per view the results are bit-identical to pg_reproject_sample,
 * pg_light_field and pg_em_update called with that view's arguments and the
 * same training tile. */
typedef struct pg_batch_view {
  pg_params params;    /* seed, frame, view, tile_w and tile_h may differ
                          between views; every other field must equal view
                          0's.  tile_w/tile_h request the training tile of
                          the view's spp group (the views of one spp are
                          trained by one launch, so they must request the
                          same tile, else PG_ERR_ARG); a built tile whose
                          LDS does not fit the spp falls back to the
                          default tile of that spp (0 = default)            */
  pg_view cur;         /* this frame's G-buffer (albedo required)             */
  pg_view prev;        /* previous frame's (read when params.frame > 0; same
                          width, height and pitch as cur)                    */
  pg_gamma gamma_in;   /* previous state (read when params.frame > 0)         */
  pg_gamma gamma_out;  /* this frame's state, cur's height and pitch; must not
                          alias gamma_in; one dtype for all views             */
  pg_samples samples;  /* records; radiance is written too                    */
  const uint8_t *vis;  /* [H*pitch] light visibility bits (device)            */
  pg_lights lights;    /* this view's light field                             */
} pg_batch_view;

/* Bytes of the packed table for n_views views (0 for n_views < 1). */
size_t pg_batch_table_bytes(int32_t n_views);

/* Checks n_views views (the same checks as the single-view calls, plus a
 * common dtype and shared parameters) and writes the packed table into
 * host_table (caller-owned host memory of at least pg_batch_table_bytes
 * bytes).  The table groups the views by spp; each group is trained by a
 * launch of its own with its tile.  Host only: no GPU work, nothing
 * retained. */
pg_status pg_batch_pack(const pg_batch_view *views, int32_t n_views, void *host_table, size_t bytes);

/* Enqueues on `stream`: a copy of `bytes` bytes from host_table to
 * device_table (caller-owned device memory), then the launches (sampling for
 * all views, then training per spp group, one block per tile), which read
 * the table there.  The launch configuration (dtype, spp groups and their tiles)
 * is read from host_table during the call.  host_table should be pinned
 * (hipHostMalloc) so that the copy is asynchronous and can be captured; it
 * must not be re-packed before the copy has run.  A captured graph replays
 * re-packed tables of other frames and views as long as the dtype and the spp
 * groups with their tiles stay those of the capture and the views have no
 * more sampling tiles, and no group more training tiles, than at the capture
 * (a launch whose part of the table differs skips it: nothing of it is
 * written).  Views must not share
 * output buffers. */
pg_status pg_frame_batched(const void *host_table, void *device_table, size_t bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * pg_frame_batched with the device copy of the table held in the library's
 * own fixed array of PG_NOALLOC_TABLE_BYTES bytes (one per GPU, kept until
 * the process ends) instead of a caller-owned device_table.  The call itself
 * allocates nothing: it copies host_table (pinned, as for pg_frame_batched)
 * into that array on `stream` and launches the same kernels, so its results
 * are those of pg_frame_batched bit for bit.  A table of more than
 * PG_NOALLOC_TABLE_BYTES bytes (pg_batch_table_bytes) returns
 * PG_ERR_UNSUPPORTED before any work.  Every call on one GPU uses the same
 * array and leaves its table there: calls that overlap on one GPU (on
 * different streams, or a replayed graph beside another call) race on it and
 * must be ordered by the caller.  The first call on a device looks the
 * array's address up (hipGetSymbolAddress) with that device current. */
#define PG_NOALLOC_TABLE_BYTES 65536
pg_status pg_frame_batched_noalloc(const void *host_table, size_t bytes, void *stream);

/* Diagnostic: Philox4x32-10 (Salmon et al., SC 2011), the generator behind
 * every random draw above, for n counters: counters [n][4] uint32 and out
 * [n][4] uint32 are device arrays, key = (seed low word, seed high word). */
pg_status pg_philox(int32_t n, const uint32_t *counters, uint64_t seed, uint32_t *out, void *stream);

/* Text of the last error on the calling thread ("" if none). */
const char *pg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
