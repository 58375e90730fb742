// C ABI of libpmmguide: argument checks on the host, then kernel launches
// on the caller's stream.  The operations are specified in pmmguide.h.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "pg_kernels.hpp"
#include "pg_lobes.hpp"
#include "pmmguide.h"

using namespace pgk;

namespace {

thread_local std::string g_last_error;

pg_status fail(pg_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
pg_status fail(pg_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

pg_status ok() {
  g_last_error.clear();
  return PG_OK;
}

pg_status check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PG_ERR_HIP, "%s: launch failed: %s", what, hipGetErrorString(e));
  return ok();
}

constexpr int kMaxDim = 16384;

pg_status check_params(const pg_params *p) {
  if (!p) return fail(PG_ERR_ARG, "params is NULL");
  if (p->k_max < 1 || p->k_max > 1000000) return fail(PG_ERR_ARG, "k_max must be >= 1");
  if (p->radius != kR) return fail(PG_ERR_UNSUPPORTED, "radius %d: only %d is built", p->radius, kR);
  if (!(p->eps_sigma > 0.0f) && p->eps_sigma != 0.0f) return fail(PG_ERR_ARG, "eps_sigma must be >= 0");
  if (!(p->pi_lo <= p->pi_hi)) return fail(PG_ERR_ARG, "pi_lo > pi_hi");
  if (!(p->s_diffuse >= 0.0f && p->s_diffuse <= 1.0f)) return fail(PG_ERR_ARG, "s_diffuse outside [0, 1]");
  if ((p->flags & PG_STALE_RESET) && p->stale_tau != p->stale_tau) return fail(PG_ERR_ARG, "stale_tau is NaN");
  return PG_OK;
}

pg_status check_view(const pg_view *v, const char *name, bool need_albedo) {
  if (!v) return fail(PG_ERR_ARG, "%s is NULL", name);
  if (v->width <= 0 || v->height <= 0) return fail(PG_ERR_ARG, "%s: width/height must be > 0", name);
  if (v->pitch < v->width) return fail(PG_ERR_ARG, "%s: pitch %d < width %d", name, v->pitch, v->width);
  if (v->width > kMaxDim || v->height > kMaxDim)
    return fail(PG_ERR_UNSUPPORTED, "%s: %dx%d exceeds %d", name, v->width, v->height, kMaxDim);
  // kernels form row offsets y * pitch with 24-bit products
  if (v->pitch >= (1 << 24)) return fail(PG_ERR_UNSUPPORTED, "%s: pitch %d is 2^24 or more", name, v->pitch);
  if ((int64_t)v->pitch * v->height * 8 * 3 >= ((int64_t)1 << 31))
    return fail(PG_ERR_UNSUPPORTED, "%s: pitch*height too large for 32-bit indexing", name);
  if (!v->normal || !v->view_dir || !v->depth || !v->roughness)
    return fail(PG_ERR_ARG, "%s: normal, view_dir, depth and roughness are required", name);
  if (need_albedo && !v->albedo) return fail(PG_ERR_ARG, "%s: albedo is required", name);
  return PG_OK;
}

// The epoch k is stored in the state's own type, so k_max must be an integer
// the type holds exactly together with every smaller one: 2^8 for BF16 (8
// significant bits), 2^11 for FP16 (11); beyond that k + 1 rounds back to k
// and the epoch would stop short of k_max.
constexpr int kMaxEpochBF16 = 256, kMaxEpochF16 = 2048;

pg_status check_gamma(const pg_params *p, pg_gamma g, const char *name) {
  if (!g.data) return fail(PG_ERR_ARG, "%s.data is NULL", name);
  if (g.dtype != PG_F32 && g.dtype != PG_F16 && g.dtype != PG_BF16)
    return fail(PG_ERR_ARG, "%s: unknown dtype %d", name, g.dtype);
  if (g.dtype == PG_BF16 && p->k_max > kMaxEpochBF16)
    return fail(PG_ERR_ARG, "%s: k_max %d exceeds %d, the largest epoch a BF16 state holds exactly", name, p->k_max,
                kMaxEpochBF16);
  if (g.dtype == PG_F16 && p->k_max > kMaxEpochF16)
    return fail(PG_ERR_ARG, "%s: k_max %d exceeds %d, the largest epoch an FP16 state holds exactly", name, p->k_max,
                kMaxEpochF16);
  return PG_OK;
}

pg_status check_samples(const pg_samples *s, bool need_pdfmix, bool need_radiance) {
  if (!s) return fail(PG_ERR_ARG, "samples is NULL");
  if (s->spp < 1 || s->spp > kMaxSpp) return fail(PG_ERR_ARG, "spp %d outside [1, %d]", s->spp, kMaxSpp);
  if (!s->dir || !s->pdf_brdf || !s->strategy) return fail(PG_ERR_ARG, "samples: dir, pdf_brdf, strategy required");
  if (need_pdfmix && !s->pdf_mix) return fail(PG_ERR_ARG, "samples: pdf_mix required");
  if (need_radiance && !s->radiance) return fail(PG_ERR_ARG, "samples: radiance required");
  return PG_OK;
}

ParamsK to_k(const pg_params *p) {
  ParamsK k;
  k.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
  k.key1 = (uint32_t)(p->seed >> 32);
  k.frame = p->frame;
  k.view = p->view;
  k.k_max = p->k_max;
  k.pi_init = p->pi_init;
  k.pi_lo = p->pi_lo;
  k.pi_hi = p->pi_hi;
  k.eps = p->eps_sigma;
  k.tau_z = p->tau_depth;
  k.tau_n = p->tau_normal;
  k.rough_min = p->rough_min;
  k.s_d = p->s_diffuse;
  k.f0 = p->f0;
  k.flags = p->flags;
  k.stale_tau = p->stale_tau;
  k.s_d_pi = p->s_diffuse * 0.318309886183790671538f;
  k.one_m_f0 = 1.0f - p->f0;
  k.one_m_sd_q = (1.0f - p->s_diffuse) * 0.0795774715459476678844f;  // / (4 pi)
  return k;
}

ViewK to_k(const pg_view *v) {
  ViewK k;
  k.W = v->width;
  k.H = v->height;
  k.pitch = v->pitch;
  k.n = v->normal;
  k.o = v->view_dir;
  k.z = v->depth;
  k.rough = v->roughness;
  k.alb = v->albedo;
  k.mv = v->motion;
  k.mask = v->disocc;
  return k;
}

SamplesK to_k(const pg_samples *s) {
  SamplesK k;
  k.spp = s->spp;
  k.dir = s->dir;
  k.pmix = s->pdf_mix;
  k.pb = s->pdf_brdf;
  k.L = s->radiance;
  k.strat = s->strategy;
  return k;
}

// 1-D grid of 64x4 tiles (the kernels map blocks to tiles in XCD bands).
dim3 stream_grid(int W, int H) { return dim3(((W + 63) / 64) * ((H + 3) / 4)); }

template <typename F>
pg_status dispatch_dtype(int dtype, F &&f) {
  switch (dtype) {
    case PG_F32: return f((float *)nullptr);
    case PG_F16: return f((_Float16 *)nullptr);
    case PG_BF16: return f((bf16s *)nullptr);
  }
  return fail(PG_ERR_ARG, "unknown dtype %d", dtype);
}

// Training tile shapes built into the library.
struct Tile {
  int w, h;
};
constexpr Tile kTiles[] = {{32, 8}, {16, 16}, {64, 4}, {32, 4}, {16, 8}, {64, 2}, {32, 16}, {64, 8}};

// Default training tile per spp (1080p pan, EM per frame).  The two-pass
// tile (online EM from spp 4) runs best at 16x16 (spp 4 230 us against 239
// at 32x8; spp 6 295 against 356; spp 8 382 against 401 and 437 at 16x8).
// The single-pass tile (up to spp 3, and batch EM or the stale test above):
// 32x8 up to spp 4; above, the staged records limit how many blocks share a
// CU's LDS, and the shape that keeps the most waves resident wins: 16x16 at
// spp 5 (266 us against 339 for 32x4), 16x8 at spp 6-8 (spp 8: 508 us
// against 726).
Tile default_tile(int spp, bool two) {
  if (two) return Tile{16, 16};
  return spp <= 4 ? Tile{32, 8} : (spp == 5 ? Tile{16, 16} : Tile{16, 8});
}

// Dynamic LDS of the single-lobe training kernels: staged records
// [spp][h+6][w+6] float4, the training lists [spp+20][w*h] uint16 and the
// pick table [48 spp] int16 (at least 8 floats per pixel, which the Gamma
// write-back reuses); the two-pass tile (online EM from spp 4, `two`)
// stages half the planes at a time plus a validity bit per record.
size_t tile_lds(Tile t, int spp, bool two) {
  return two ? em2_lds_front(t.w, t.h, spp) : em_lds_front(t.w, t.h, spp);
}

// Whether a training launch takes the two-pass tile: online EM from spp 4
// without the stale-history test (batch EM revisits the whole list every
// iteration, and the test reads it before the E-step).  At 1080p EM per
// frame: spp 8 382 us (16x16) against 503 single-pass, spp 4 230 against
// 246; at spp 2 the single-pass tile already keeps 5 blocks per CU and the
// second pass costs more than it gains (182 against 157 us).
bool em_two_pass(int spp, int batch, uint32_t flags) { return spp >= 4 && !batch && !(flags & PG_STALE_RESET); }

pg_status pick_tile(const pg_params *p, int spp, Tile &t, bool two = false) {
  if (p->tile_w == 0 && p->tile_h == 0) {
    t = default_tile(spp, two);
  } else {
    bool found = false;
    for (const Tile &c : kTiles)
      if (c.w == p->tile_w && c.h == p->tile_h) found = true;
    if (!found) return fail(PG_ERR_UNSUPPORTED, "tile %dx%d is not built", p->tile_w, p->tile_h);
    t = Tile{p->tile_w, p->tile_h};
  }
  if (tile_lds(t, spp, two) > 64 * 1024)
    return fail(PG_ERR_UNSUPPORTED, "tile %dx%d with spp %d needs %zu B of LDS (> 64 KiB)", t.w, t.h, spp,
                tile_lds(t, spp, two));
  return PG_OK;
}

template <typename TG, int TW, int TH>
pg_status launch_em_t(const ParamsK &P, const ViewK &v, const SamplesK &S, TG *g, int iters, int batch,
                      hipStream_t st) {
  const int tx = (v.W + TW - 1) / TW, ty = (v.H + TH - 1) / TH;
  const int n = tx * ty;
  const bool two = em_two_pass(S.spp, batch, P.flags);
  const size_t lds = tile_lds(Tile{TW, TH}, S.spp, two);
  if (two)
    hipLaunchKernelGGL((k_em<TG, TW, TH, false, true>), dim3(n), dim3(TW * TH), lds, st, P, v, S, g, iters, tx, n);
  else if (batch)
    hipLaunchKernelGGL((k_em<TG, TW, TH, false, false, true>), dim3(n), dim3(TW * TH), lds, st, P, v, S, g, iters,
                       tx, n);
  else if (P.flags & kStaleReset)
    hipLaunchKernelGGL((k_em<TG, TW, TH, true>), dim3(n), dim3(TW * TH), lds, st, P, v, S, g, iters, tx, n);
  else
    hipLaunchKernelGGL((k_em<TG, TW, TH, false>), dim3(n), dim3(TW * TH), lds, st, P, v, S, g, iters, tx, n);
  return PG_OK;
}

template <typename TG>
pg_status launch_em(Tile t, const ParamsK &P, const ViewK &v, const SamplesK &S, TG *g, int iters, int batch,
                    hipStream_t st) {
  if (t.w == 32 && t.h == 8) return launch_em_t<TG, 32, 8>(P, v, S, g, iters, batch, st);
  if (t.w == 16 && t.h == 16) return launch_em_t<TG, 16, 16>(P, v, S, g, iters, batch, st);
  if (t.w == 64 && t.h == 4) return launch_em_t<TG, 64, 4>(P, v, S, g, iters, batch, st);
  if (t.w == 32 && t.h == 4) return launch_em_t<TG, 32, 4>(P, v, S, g, iters, batch, st);
  if (t.w == 16 && t.h == 8) return launch_em_t<TG, 16, 8>(P, v, S, g, iters, batch, st);
  if (t.w == 32 && t.h == 16) return launch_em_t<TG, 32, 16>(P, v, S, g, iters, batch, st);
  if (t.w == 64 && t.h == 8) return launch_em_t<TG, 64, 8>(P, v, S, g, iters, batch, st);
  return launch_em_t<TG, 64, 2>(P, v, S, g, iters, batch, st);
}

template <int TW, int TH>
void launch_nll_t(const ParamsK &P, const ViewK &v, const SamplesK &S, const float *theta, const float *go,
                  float *grad, float *nll, hipStream_t st) {
  const int tx = (v.W + TW - 1) / TW, ty = (v.H + TH - 1) / TH;
  const int n = tx * ty;
  const size_t lds = (size_t)(TW + 2 * kR) * (TH + 2 * kR) * S.spp * sizeof(float4);
  hipLaunchKernelGGL((k_nll<TW, TH>), dim3(n), dim3(TW * TH), lds, st, P, v, S, theta, go, grad, nll, tx, n);
}

void launch_nll(Tile t, const ParamsK &P, const ViewK &v, const SamplesK &S, const float *theta,
                const float *go, float *grad, float *nll, hipStream_t st) {
  if (t.w == 32 && t.h == 8) launch_nll_t<32, 8>(P, v, S, theta, go, grad, nll, st);
  else if (t.w == 16 && t.h == 16) launch_nll_t<16, 16>(P, v, S, theta, go, grad, nll, st);
  else if (t.w == 64 && t.h == 4) launch_nll_t<64, 4>(P, v, S, theta, go, grad, nll, st);
  else if (t.w == 32 && t.h == 4) launch_nll_t<32, 4>(P, v, S, theta, go, grad, nll, st);
  else if (t.w == 16 && t.h == 8) launch_nll_t<16, 8>(P, v, S, theta, go, grad, nll, st);
  else if (t.w == 32 && t.h == 16) launch_nll_t<32, 16>(P, v, S, theta, go, grad, nll, st);
  else if (t.w == 64 && t.h == 8) launch_nll_t<64, 8>(P, v, S, theta, go, grad, nll, st);
  else launch_nll_t<64, 2>(P, v, S, theta, go, grad, nll, st);
}

LightsK to_k(const pg_lights *l) {
  LightsK L;
  std::memset(&L, 0, sizeof(L));
  L.count = l->count;
  L.ambient = l->ambient;
  for (int k = 0; k < l->count; ++k)
    for (int c = 0; c < 5; ++c) L.l[k][c] = l->light[k][c];
  return L;
}

pg_status check_lights(const pg_lights *l, const uint8_t *vis) {
  if (!l) return fail(PG_ERR_ARG, "lights is NULL");
  if (l->count < 0 || l->count > PG_MAX_LIGHTS) return fail(PG_ERR_ARG, "lights->count out of range");
  if (!vis && l->count > 0) return fail(PG_ERR_ARG, "vis is NULL");
  return PG_OK;
}

// ---- batched frame ----------------------------------------------------------
constexpr int kBatchMagic = 0x31424750;  // "PGB1"

size_t batch_bytes(int n) { return (size_t)kBatchViewsOffset + (size_t)n * sizeof(BatchViewK); }

// Device copy of the packed table for pg_frame_batched_noalloc: a fixed
// array in the library's own device memory (one per GPU, for the life of the
// process).  Host code never passes the array's name to a kernel or a copy:
// it holds the address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchTableBytes = PG_NOALLOC_TABLE_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchTableBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The address of `scratch` on the current device, looked up once per device.
pg_status scratch_table(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(PG_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(PG_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PG_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PG_OK;
}

// Upload of a packed table to device_table, then the batched launches.
pg_status frame_batched(const void *host_table, void *device_table, size_t bytes, hipStream_t s);

// Parameters every view of a batch must share (all but seed, frame, view).
bool shared_params_equal(const pg_params &a, const pg_params &b) {
  return a.k_max == b.k_max && a.radius == b.radius && a.pi_init == b.pi_init && a.pi_lo == b.pi_lo &&
         a.pi_hi == b.pi_hi && a.eps_sigma == b.eps_sigma && a.tau_depth == b.tau_depth &&
         a.tau_normal == b.tau_normal && a.rough_min == b.rough_min && a.s_diffuse == b.s_diffuse &&
         a.f0 == b.f0 && a.flags == b.flags;
}

pg_status in_view(pg_status st, int i) {
  if (st != PG_OK) g_last_error += " (view " + std::to_string(i) + ")";
  return st;
}

pg_status check_batch_view(const pg_batch_view &b, int dtype) {
  pg_status st;
  if ((st = check_params(&b.params)) || (st = check_view(&b.cur, "cur", true)) ||
      (st = check_gamma(&b.params, b.gamma_out, "gamma_out")) || (st = check_samples(&b.samples, true, true)) ||
      (st = check_lights(&b.lights, b.vis)))
    return st;
  if (b.params.flags & PG_EM_BATCH) return fail(PG_ERR_UNSUPPORTED, "the batched frame runs the online update only");
  if (b.params.flags & PG_STALE_RESET) return fail(PG_ERR_UNSUPPORTED, "the batched frame has no stale-history reset");
  if (b.gamma_out.dtype != dtype) return fail(PG_ERR_ARG, "views store Gamma in different dtypes");
  if (b.params.frame > 0) {
    if ((st = check_view(&b.prev, "prev", false)) || (st = check_gamma(&b.params, b.gamma_in, "gamma_in"))) return st;
    if (b.prev.width != b.cur.width || b.prev.height != b.cur.height || b.prev.pitch != b.cur.pitch)
      return fail(PG_ERR_UNSUPPORTED, "the batched frame needs prev and cur of one size and pitch");
    if (b.gamma_in.dtype != dtype) return fail(PG_ERR_ARG, "gamma_in and gamma_out dtypes differ");
    if (b.gamma_in.data == b.gamma_out.data) return fail(PG_ERR_ARG, "gamma_in aliases gamma_out");
  }
  return PG_OK;
}

BatchViewK to_batch(const pg_batch_view &b, int rs_begin, int em_begin, Tile t) {
  BatchViewK k;
  std::memset(&k, 0, sizeof(k));
  k.cur = to_k(&b.cur);
  const bool has_prev = b.params.frame > 0;
  k.prev_n = has_prev ? b.prev.normal : nullptr;
  k.prev_z = has_prev ? b.prev.depth : nullptr;
  k.gprev = has_prev ? b.gamma_in.data : nullptr;
  k.gout = b.gamma_out.data;
  k.S = to_k(&b.samples);
  k.vis = b.vis;
  k.lights = to_k(&b.lights);
  const ParamsK P = to_k(&b.params);
  k.key0 = P.key0;
  k.key1 = P.key1;
  k.frame = P.frame;
  k.view = P.view;
  k.rs_begin = rs_begin;
  k.rs_tiles_x = (b.cur.width + 63) / 64;
  k.em_begin = em_begin;
  k.em_tiles_x = (b.cur.width + t.w - 1) / t.w;
  return k;
}

template <typename TG, int TW, int TH>
pg_status launch_em_batched_t(const void *table, int dtype, int cls, int spp, int n_tiles, hipStream_t st) {
  const bool two = em_two_pass(spp, 0, 0);  // the batched frame runs online EM
  const size_t lds = tile_lds(Tile{TW, TH}, spp, two);
  if (n_tiles < 1) return PG_OK;
  // one tile per block, like k_em (the class's tile count is fixed by its views)
  if (two)
    hipLaunchKernelGGL((k_em_batched<TG, TW, TH, true>), dim3(n_tiles), dim3(TW * TH), lds, st, (const char *)table,
                       dtype, cls, spp);
  else
    hipLaunchKernelGGL((k_em_batched<TG, TW, TH, false>), dim3(n_tiles), dim3(TW * TH), lds, st, (const char *)table,
                       dtype, cls, spp);
  return PG_OK;
}

template <typename TG>
pg_status launch_em_batched(const BatchClass &c, const void *table, int dtype, int cls, hipStream_t st) {
  const int n = c.em_end - c.em_begin;
  const Tile t{c.tile_w, c.tile_h};
  if (t.w == 32 && t.h == 8) return launch_em_batched_t<TG, 32, 8>(table, dtype, cls, c.spp, n, st);
  if (t.w == 16 && t.h == 16) return launch_em_batched_t<TG, 16, 16>(table, dtype, cls, c.spp, n, st);
  if (t.w == 64 && t.h == 4) return launch_em_batched_t<TG, 64, 4>(table, dtype, cls, c.spp, n, st);
  if (t.w == 32 && t.h == 4) return launch_em_batched_t<TG, 32, 4>(table, dtype, cls, c.spp, n, st);
  if (t.w == 16 && t.h == 8) return launch_em_batched_t<TG, 16, 8>(table, dtype, cls, c.spp, n, st);
  if (t.w == 32 && t.h == 16) return launch_em_batched_t<TG, 32, 16>(table, dtype, cls, c.spp, n, st);
  if (t.w == 64 && t.h == 8) return launch_em_batched_t<TG, 64, 8>(table, dtype, cls, c.spp, n, st);
  return launch_em_batched_t<TG, 64, 2>(table, dtype, cls, c.spp, n, st);
}

// Training tile of a class of the batch: the requested one where its LDS
// fits that spp, else the default for that spp.
pg_status class_tile(const pg_params *p, int spp, Tile &t) {
  const bool two = em_two_pass(spp, 0, 0);  // the batched frame runs online EM
  if (p->tile_w == 0 && p->tile_h == 0) {
    t = default_tile(spp, two);
    return PG_OK;
  }
  pg_status st = pick_tile(p, spp, t, em_two_pass(spp, 0, 0));
  if (st == PG_OK) return st;
  bool built = false;
  for (const Tile &c : kTiles)
    if (c.w == p->tile_w && c.h == p->tile_h) built = true;
  if (!built) return st;  // an unknown shape stays an error
  t = default_tile(spp, two);
  return ok();
}

pg_status check_lobes(const pg_params *p, int32_t lobes, const pg_view *v) {
  if (lobes < 1 || lobes > kMaxLobes) return fail(PG_ERR_ARG, "lobes %d outside [1, %d]", lobes, kMaxLobes);
  if (p->flags & (PG_EM_BATCH | PG_STALE_RESET))
    return fail(PG_ERR_UNSUPPORTED, "PG_EM_BATCH and PG_STALE_RESET are not built for K lobes");
  if ((int64_t)v->pitch * v->height * (6 * lobes + 2) >= ((int64_t)1 << 31))
    return fail(PG_ERR_UNSUPPORTED, "(6K + 2) * pitch * height too large for 32-bit indexing");
  return PG_OK;
}

// Calls f with std::integral_constant<int, K> for K = lobes (checked before).
template <typename F>
pg_status dispatch_lobes(int lobes, F &&f) {
  switch (lobes) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    default: return f(std::integral_constant<int, 4>{});
  }
}

}  // namespace

extern "C" {

pg_status pg_params_default(pg_params *p) {
  if (!p) return fail(PG_ERR_ARG, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->k_max = 16;
  p->radius = 3;
  p->pi_init = 0.05f;
  p->pi_lo = 0.05f;
  p->pi_hi = 0.95f;
  p->eps_sigma = 2.5e-4f;
  p->tau_depth = 0.1f;
  p->tau_normal = 0.9f;
  p->rough_min = 0.1f;
  p->s_diffuse = 0.5f;
  p->f0 = 0.04f;
  return ok();
}

pg_status pg_reproject(const pg_params *p, const pg_view *cur, const pg_view *prev, pg_gamma prev_gamma,
                       pg_gamma out_gamma, int32_t *src_index, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(cur, "cur", false)) || (st = check_gamma(p, out_gamma, "out_gamma")))
    return st;
  const bool has_prev = p->frame > 0;
  if (has_prev) {
    if ((st = check_view(prev, "prev", false)) || (st = check_gamma(p, prev_gamma, "prev_gamma"))) return st;
    if (prev_gamma.dtype != out_gamma.dtype) return fail(PG_ERR_ARG, "prev_gamma and out_gamma dtypes differ");
    if (prev_gamma.data == out_gamma.data) return fail(PG_ERR_ARG, "prev_gamma aliases out_gamma");
  }
  const ParamsK P = to_k(p);
  const ViewK C = to_k(cur);
  const ViewK Q = has_prev ? to_k(prev) : C;
  hipStream_t s = (hipStream_t)stream;
  return dispatch_dtype(out_gamma.dtype, [&](auto *tag) {
    using TG = std::remove_pointer_t<decltype(tag)>;
    hipLaunchKernelGGL((k_reproject<TG>), stream_grid(C.W, C.H), dim3(64, 4), 0, s, P, C, Q,
                       (const TG *)(has_prev ? prev_gamma.data : out_gamma.data), (TG *)out_gamma.data,
                       src_index, has_prev ? 1 : 0);
    return check_launch("pg_reproject");
  });
}

pg_status pg_sample_mis(const pg_params *p, const pg_view *v, pg_gamma gamma, const pg_samples *out,
                        void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", false)) || (st = check_gamma(p, gamma, "gamma")) ||
      (st = check_samples(out, true, false)))
    return st;
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(out);
  hipStream_t s = (hipStream_t)stream;
  return dispatch_dtype(gamma.dtype, [&](auto *tag) {
    using TG = std::remove_pointer_t<decltype(tag)>;
    hipLaunchKernelGGL((k_sample<TG>), stream_grid(V.W, V.H), dim3(64, 4), 0, s, P, V, (const TG *)gamma.data, S);
    return check_launch("pg_sample_mis");
  });
}

pg_status pg_reproject_sample(const pg_params *p, const pg_view *cur, const pg_view *prev, pg_gamma prev_gamma,
                              pg_gamma out_gamma, const pg_samples *out, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(cur, "cur", false)) ||
      (st = check_gamma(p, out_gamma, "out_gamma")) || (st = check_samples(out, true, false)))
    return st;
  const bool has_prev = p->frame > 0;
  if (has_prev) {
    if ((st = check_view(prev, "prev", false)) || (st = check_gamma(p, prev_gamma, "prev_gamma"))) return st;
    if (prev_gamma.dtype != out_gamma.dtype) return fail(PG_ERR_ARG, "prev_gamma and out_gamma dtypes differ");
    if (prev_gamma.data == out_gamma.data) return fail(PG_ERR_ARG, "prev_gamma aliases out_gamma");
  }
  const ParamsK P = to_k(p);
  const ViewK C = to_k(cur);
  const ViewK Q = has_prev ? to_k(prev) : C;
  const SamplesK S = to_k(out);
  hipStream_t s = (hipStream_t)stream;
  return dispatch_dtype(out_gamma.dtype, [&](auto *tag) {
    using TG = std::remove_pointer_t<decltype(tag)>;
    hipLaunchKernelGGL((k_reproject_sample<TG>), stream_grid(C.W, C.H), dim3(64, 4), 0, s, P, C, Q,
                       (const TG *)(has_prev ? prev_gamma.data : out_gamma.data), (TG *)out_gamma.data, S,
                       has_prev ? 1 : 0);
    return check_launch("pg_reproject_sample");
  });
}

pg_status pg_pdf(const pg_params *p, const pg_view *v, pg_gamma gamma, int32_t n_per_px, const float *dir,
                 float *pdf_mix, float *pdf_guide, float *pdf_brdf, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", false)) || (st = check_gamma(p, gamma, "gamma")))
    return st;
  if (n_per_px < 1 || n_per_px > 64) return fail(PG_ERR_ARG, "n_per_px %d outside [1, 64]", n_per_px);
  if ((int64_t)v->pitch * v->height * n_per_px * 3 >= ((int64_t)1 << 31))
    return fail(PG_ERR_UNSUPPORTED, "n_per_px * pitch * height too large for 32-bit indexing");
  if (!dir || !pdf_mix) return fail(PG_ERR_ARG, "dir and pdf_mix are required");
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  hipStream_t s = (hipStream_t)stream;
  return dispatch_dtype(gamma.dtype, [&](auto *tag) {
    using TG = std::remove_pointer_t<decltype(tag)>;
    hipLaunchKernelGGL((k_pdf<TG>), stream_grid(V.W, V.H), dim3(64, 4), 0, s, P, V, (const TG *)gamma.data,
                       n_per_px, dir, pdf_mix, pdf_guide, pdf_brdf);
    return check_launch("pg_pdf");
  });
}

pg_status pg_light_field(const pg_lights *lights, const pg_view *v, const uint8_t *vis, const pg_samples *samples,
                         void *stream) {
  pg_status st;
  if ((st = check_lights(lights, vis)) || (st = check_view(v, "view", false)) ||
      (st = check_samples(samples, false, true)))
    return st;
  const LightsK L = to_k(lights);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(samples);
  hipLaunchKernelGGL(k_light, stream_grid(V.W, V.H), dim3(64, 4), 0, (hipStream_t)stream, L, V, vis, S);
  return check_launch("pg_light_field");
}

pg_status pg_em_update(const pg_params *p, const pg_view *v, const pg_samples *in, pg_gamma gamma_inout,
                       int32_t iterations, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", true)) || (st = check_gamma(p, gamma_inout, "gamma")) ||
      (st = check_samples(in, false, true)))
    return st;
  const int batch = (p->flags & PG_EM_BATCH) ? 1 : 0;
  if (iterations < 1 || (!batch && iterations != 1) || iterations > 1000)
    return fail(PG_ERR_ARG, "iterations %d invalid (1 without PG_EM_BATCH, 1..1000 with it)", iterations);
  Tile t;
  if ((st = pick_tile(p, in->spp, t, em_two_pass(in->spp, batch, p->flags)))) return st;
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(in);
  hipStream_t s = (hipStream_t)stream;
  return dispatch_dtype(gamma_inout.dtype, [&](auto *tag) {
    using TG = std::remove_pointer_t<decltype(tag)>;
    pg_status e = launch_em<TG>(t, P, V, S, (TG *)gamma_inout.data, iterations, batch, s);
    return e ? e : check_launch("pg_em_update");
  });
}

pg_status pg_nll_backward(const pg_params *p, const pg_view *v, const pg_samples *in, const float *theta,
                          const float *grad_out, float *grad_theta, float *nll, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", true)) || (st = check_samples(in, false, true)))
    return st;
  if (!theta) return fail(PG_ERR_ARG, "theta is NULL");
  if (!grad_theta && !nll) return fail(PG_ERR_ARG, "nothing to compute: grad_theta and nll are NULL");
  Tile t;
  if ((st = pick_tile(p, in->spp, t))) return st;
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(in);
  launch_nll(t, P, V, S, theta, grad_out, grad_theta, nll, (hipStream_t)stream);
  return check_launch("pg_nll_backward");
}

pg_status pg_estimate(const pg_params *p, const pg_view *v, const pg_samples *in, float *estimate, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", true)) || (st = check_samples(in, true, true)))
    return st;
  if (!estimate) return fail(PG_ERR_ARG, "estimate is NULL");
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(in);
  hipLaunchKernelGGL(k_estimate, stream_grid(V.W, V.H), dim3(64, 4), 0, (hipStream_t)stream, P, V, S, estimate);
  return check_launch("pg_estimate");
}

pg_status pg_reproject_sample_lobes(const pg_params *p, int32_t lobes, const pg_view *cur, const pg_view *prev,
                                    const float *prev_gamma, float *out_gamma, const pg_samples *out, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(cur, "cur", false)) || (st = check_lobes(p, lobes, cur)) ||
      (st = check_samples(out, true, false)))
    return st;
  if (!out_gamma) return fail(PG_ERR_ARG, "out_gamma is NULL");
  const bool has_prev = p->frame > 0;
  if (has_prev) {
    if ((st = check_view(prev, "prev", false))) return st;
    if (!prev_gamma) return fail(PG_ERR_ARG, "prev_gamma is NULL");
    if (prev_gamma == out_gamma) return fail(PG_ERR_ARG, "prev_gamma aliases out_gamma");
    if (prev->width != cur->width || prev->height != cur->height || prev->pitch != cur->pitch)
      return fail(PG_ERR_UNSUPPORTED, "prev must have cur's width, height and pitch");
  }
  const ParamsK P = to_k(p);
  const ViewK C = to_k(cur);
  const ViewK Q = has_prev ? to_k(prev) : C;
  const SamplesK S = to_k(out);
  hipStream_t s = (hipStream_t)stream;
  return dispatch_lobes(lobes, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL((k_lobes_reproject_sample<K>), stream_grid(C.W, C.H), dim3(64, 4), 0, s, P, C, Q,
                       has_prev ? prev_gamma : out_gamma, out_gamma, S, has_prev ? 1 : 0);
    return check_launch("pg_reproject_sample_lobes");
  });
}

pg_status pg_em_update_lobes(const pg_params *p, int32_t lobes, const pg_view *v, const pg_samples *in,
                             float *gamma_inout, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", true)) || (st = check_lobes(p, lobes, v)) ||
      (st = check_samples(in, false, true)))
    return st;
  if (!gamma_inout) return fail(PG_ERR_ARG, "gamma is NULL");
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(in);
  hipStream_t s = (hipStream_t)stream;
  // 32x8 tiles, 32x4 above 4 spp (the records of 8 planes with the halo and
  // the lists fit 64 KiB)
  const int TH = in->spp > 4 ? 4 : 8;
  const int tx = (V.W + 31) / 32, ty = (V.H + TH - 1) / TH;
  const size_t lds_tile = (size_t)in->spp * (32 + 2 * kR) * (TH + 2 * kR) * sizeof(float4) +
                          (size_t)(in->spp + 20) * 32 * TH * sizeof(uint16_t) + (size_t)pick_table_bytes(in->spp);
  const size_t lds_wb = (size_t)(6 * lobes + 2) * 32 * TH * sizeof(float);  // write-back area
  const size_t lds = lds_tile > lds_wb ? lds_tile : lds_wb;
  return dispatch_lobes(lobes, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    if (TH == 8)
      hipLaunchKernelGGL((k_lobes_em<K, 32, 8>), dim3(tx * ty), dim3(256), lds, s, P, V, S, gamma_inout, tx,
                         tx * ty, nullptr, nullptr);
    else
      hipLaunchKernelGGL((k_lobes_em<K, 32, 4>), dim3(tx * ty), dim3(128), lds, s, P, V, S, gamma_inout, tx,
                         tx * ty, nullptr, nullptr);
    return check_launch("pg_em_update_lobes");
  });
}

pg_status pg_em_update_vpl(const pg_params *p, int32_t lobes, const pg_view *v, const float *position,
                           const pg_samples *in, const float *hit_dist, float *gamma_inout, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", true)) || (st = check_lobes(p, lobes, v)) ||
      (st = check_samples(in, false, true)))
    return st;
  if (!gamma_inout) return fail(PG_ERR_ARG, "gamma is NULL");
  if (!position || !hit_dist) return fail(PG_ERR_ARG, "position and hit_dist are required");
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  const SamplesK S = to_k(in);
  hipStream_t s = (hipStream_t)stream;
  const int TH = in->spp > 4 ? 4 : 8;
  const int tx = (V.W + 31) / 32, ty = (V.H + TH - 1) / TH;
  const size_t lds_tile = (size_t)in->spp * (32 + 2 * kR) * (TH + 2 * kR) * sizeof(float4) +
                          (size_t)(in->spp + 20) * 32 * TH * sizeof(uint16_t) + (size_t)pick_table_bytes(in->spp);
  const size_t lds_wb = (size_t)(6 * lobes + 2) * 32 * TH * sizeof(float);
  const size_t lds = lds_tile > lds_wb ? lds_tile : lds_wb;
  return dispatch_lobes(lobes, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    if (TH == 8)
      hipLaunchKernelGGL((k_lobes_em<K, 32, 8, true>), dim3(tx * ty), dim3(256), lds, s, P, V, S, gamma_inout,
                         tx, tx * ty, position, hit_dist);
    else
      hipLaunchKernelGGL((k_lobes_em<K, 32, 4, true>), dim3(tx * ty), dim3(128), lds, s, P, V, S, gamma_inout,
                         tx, tx * ty, position, hit_dist);
    return check_launch("pg_em_update_vpl");
  });
}

pg_status pg_light_ceiling(const pg_ceiling *c, const pg_view *v, const float *position, const pg_samples *samples,
                           float *hit_dist, void *stream) {
  pg_status st;
  if ((st = check_view(v, "view", false)) || (st = check_samples(samples, false, true))) return st;
  if (!c || !c->lamps) return fail(PG_ERR_ARG, "ceiling and its lamps are required");
  if (c->nx < 1 || c->ny < 1 || (int64_t)c->nx * c->ny > (1 << 24))
    return fail(PG_ERR_ARG, "lamp lattice %d x %d invalid", c->nx, c->ny);
  if (!(c->period > 0.0f)) return fail(PG_ERR_ARG, "period must be > 0");
  if (!position || !hit_dist) return fail(PG_ERR_ARG, "position and hit_dist are required");
  if (((uintptr_t)c->lamps & 15u) != 0) return fail(PG_ERR_ARG, "lamps must be 16-byte aligned");
  CeilingK C;
  C.z = c->z;
  C.period = c->period;
  C.x0 = c->x0;
  C.y0 = c->y0;
  C.ambient = c->ambient;
  C.nx = c->nx;
  C.ny = c->ny;
  C.lamps = c->lamps;
  const ViewK V = to_k(v);
  const SamplesK S = to_k(samples);
  hipLaunchKernelGGL(k_light_ceiling, stream_grid(V.W, V.H), dim3(64, 4), 0, (hipStream_t)stream, C, V, position, S,
                     hit_dist);
  return check_launch("pg_light_ceiling");
}

pg_status pg_pdf_lobes(const pg_params *p, int32_t lobes, const pg_view *v, const float *gamma, int32_t n_per_px,
                       const float *dir, float *pdf_mix, void *stream) {
  pg_status st;
  if ((st = check_params(p)) || (st = check_view(v, "view", false)) || (st = check_lobes(p, lobes, v))) return st;
  if (!gamma) return fail(PG_ERR_ARG, "gamma is NULL");
  if (n_per_px < 1 || n_per_px > 64) return fail(PG_ERR_ARG, "n_per_px %d outside [1, 64]", n_per_px);
  if ((int64_t)v->pitch * v->height * n_per_px * 3 >= ((int64_t)1 << 31))
    return fail(PG_ERR_UNSUPPORTED, "n_per_px * pitch * height too large for 32-bit indexing");
  if (!dir || !pdf_mix) return fail(PG_ERR_ARG, "dir and pdf_mix are required");
  const ParamsK P = to_k(p);
  const ViewK V = to_k(v);
  hipStream_t s = (hipStream_t)stream;
  return dispatch_lobes(lobes, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    hipLaunchKernelGGL((k_lobes_pdf<K>), stream_grid(V.W, V.H), dim3(64, 4), 0, s, P, V, gamma, n_per_px, dir,
                       pdf_mix);
    return check_launch("pg_pdf_lobes");
  });
}

size_t pg_batch_table_bytes(int32_t n_views) { return n_views < 1 ? 0 : batch_bytes(n_views); }

pg_status pg_batch_pack(const pg_batch_view *views, int32_t n_views, void *host_table, size_t bytes) {
  if (!views || n_views < 1) return fail(PG_ERR_ARG, "pg_batch_pack: no views");
  if (n_views > (1 << 20)) return fail(PG_ERR_UNSUPPORTED, "pg_batch_pack: %d views", n_views);
  if (!host_table || bytes < batch_bytes(n_views))
    return fail(PG_ERR_ARG, "pg_batch_pack: table of %zu bytes, %zu needed", bytes, batch_bytes(n_views));
  const int dtype = views[0].gamma_out.dtype;
  pg_status st;
  int per_spp[kMaxSpp + 1] = {0}, first_of[kMaxSpp + 1] = {0};
  for (int i = 0; i < n_views; ++i) {
    if ((st = in_view(check_batch_view(views[i], dtype), i))) return st;
    if (!shared_params_equal(views[i].params, views[0].params))
      return in_view(fail(PG_ERR_ARG, "parameters other than seed, frame, view and tile differ from view 0's"), i);
    for (int j = 0; j < i; ++j)
      if (views[j].gamma_out.data == views[i].gamma_out.data || views[j].samples.dir == views[i].samples.dir)
        return in_view(fail(PG_ERR_ARG, "output buffers shared with view %d", j), i);
    // the views of one spp share a training launch, so they request one tile
    const int spp = views[i].samples.spp;
    if (per_spp[spp] && (views[i].params.tile_w != views[first_of[spp]].params.tile_w ||
                         views[i].params.tile_h != views[first_of[spp]].params.tile_h))
      return in_view(fail(PG_ERR_ARG, "views of spp %d request different training tiles (view %d asks for %dx%d)",
                          spp, first_of[spp], views[first_of[spp]].params.tile_w,
                          views[first_of[spp]].params.tile_h), i);
    if (!per_spp[spp]) first_of[spp] = i;
    ++per_spp[spp];
  }
  // classes by spp, each with the tile its views request
  BatchClass cls[kMaxSpp];
  Tile ctile[kMaxSpp];
  int n_classes = 0, class_of[kMaxSpp + 1];
  for (int spp = 1; spp <= kMaxSpp; ++spp) {
    class_of[spp] = -1;
    if (!per_spp[spp]) continue;
    if ((st = class_tile(&views[first_of[spp]].params, spp, ctile[n_classes]))) return in_view(st, first_of[spp]);
    std::memset(&cls[n_classes], 0, sizeof(BatchClass));
    cls[n_classes].spp = spp;
    cls[n_classes].tile_w = ctile[n_classes].w;
    cls[n_classes].tile_h = ctile[n_classes].h;
    class_of[spp] = n_classes++;
  }
  std::memset(host_table, 0, batch_bytes(n_views));
  BatchViewK *out = reinterpret_cast<BatchViewK *>((char *)host_table + kBatchViewsOffset);
  int64_t rs = 0, em = 0;
  int k = 0;
  for (int c = 0; c < n_classes; ++c) {
    cls[c].em_begin = (int)em;
    for (int i = 0; i < n_views; ++i) {  // the views of this class in the caller's order
      if (class_of[views[i].samples.spp] != c) continue;
      const pg_view &cv = views[i].cur;
      const Tile t = ctile[c];
      out[k++] = to_batch(views[i], (int)rs, (int)em, t);
      rs += (int64_t)((cv.width + 63) / 64) * ((cv.height + 3) / 4);
      em += (int64_t)((cv.width + t.w - 1) / t.w) * ((cv.height + t.h - 1) / t.h);
      if (rs >= ((int64_t)1 << 31) || em >= ((int64_t)1 << 31))
        return fail(PG_ERR_UNSUPPORTED, "pg_batch_pack: too many tiles for 32-bit indexing");
    }
    cls[c].em_end = (int)em;
  }
  BatchHeader *hd = reinterpret_cast<BatchHeader *>(host_table);
  hd->n_views = n_views;
  hd->rs_tiles = (int)rs;
  hd->em_tiles = (int)em;
  hd->dtype = dtype;
  hd->n_classes = n_classes;
  hd->magic = kBatchMagic;
  hd->base = to_k(&views[0].params);
  for (int c = 0; c < n_classes; ++c) hd->cls[c] = cls[c];
  return ok();
}

pg_status pg_frame_batched(const void *host_table, void *device_table, size_t bytes, void *stream) {
  if (!host_table || !device_table) return fail(PG_ERR_ARG, "pg_frame_batched: NULL table");
  return frame_batched(host_table, device_table, bytes, (hipStream_t)stream);
}

pg_status pg_frame_batched_noalloc(const void *host_table, size_t bytes, void *stream) {
  if (!host_table) return fail(PG_ERR_ARG, "pg_frame_batched_noalloc: NULL table");
  if (bytes >= (size_t)kBatchViewsOffset) {
    const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(host_table);
    if (hd->magic == kBatchMagic && hd->n_views >= 1 && batch_bytes(hd->n_views) > kScratchTableBytes)
      return fail(PG_ERR_UNSUPPORTED, "pg_frame_batched_noalloc: a table of %d views needs %zu bytes, more than the %zu "
                  "of the library's table", hd->n_views, batch_bytes(hd->n_views), kScratchTableBytes);
  }
  void *table = nullptr;
  pg_status st = scratch_table(&table);
  if (st) return st;
  return frame_batched(host_table, table, bytes, (hipStream_t)stream);
}

}  // extern "C"

namespace {

pg_status frame_batched(const void *host_table, void *device_table, size_t bytes, hipStream_t s) {
  if (bytes < (size_t)kBatchViewsOffset) return fail(PG_ERR_ARG, "pg_frame_batched: table too small");
  const BatchHeader hd = *reinterpret_cast<const BatchHeader *>(host_table);
  if (hd.magic != kBatchMagic || hd.n_views < 1 || bytes < batch_bytes(hd.n_views) || hd.n_classes < 1 ||
      hd.n_classes > kMaxSpp)
    return fail(PG_ERR_ARG, "pg_frame_batched: host_table was not packed by pg_batch_pack for %zu bytes", bytes);
  if (hipMemcpyAsync(device_table, host_table, batch_bytes(hd.n_views), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(PG_ERR_HIP, "pg_frame_batched: table upload failed: %s", hipGetErrorString(hipGetLastError()));
  return dispatch_dtype(hd.dtype, [&](auto *tag) {
    using TG = std::remove_pointer_t<decltype(tag)>;
    pg_status e;
    if (hd.rs_tiles > 0)
      hipLaunchKernelGGL((k_rs_batched<TG>), dim3(hd.rs_tiles), dim3(256), 0, s, (const char *)device_table,
                         hd.dtype);
    if ((e = check_launch("pg_frame_batched (sampling)"))) return e;
    for (int c = 0; c < hd.n_classes; ++c)
      if ((e = launch_em_batched<TG>(hd.cls[c], device_table, hd.dtype, c, s))) return e;
    return check_launch("pg_frame_batched (training)");
  });
}

}  // namespace

extern "C" {

/* Diagnostic: Philox4x32-10 words for n counters (device arrays [n][4]). */
pg_status pg_philox(int32_t n, const uint32_t *counters, uint64_t seed, uint32_t *out, void *stream) {
  if (n < 0 || (n > 0 && (!counters || !out))) return fail(PG_ERR_ARG, "pg_philox: bad arguments");
  if (n == 0) return ok();
  hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, counters,
                     (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32), out);
  return check_launch("pg_philox");
}

const char *pg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
