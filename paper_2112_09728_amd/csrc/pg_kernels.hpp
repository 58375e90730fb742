// Kernels of the path-guiding hot path for gfx950.
//
// One lane per pixel.  Streaming passes (reprojection, sampling, densities,
// light field) use 64x4 blocks so that each wave reads one 256-byte row
// segment of every plane.  The training pass stages the sample records of a
// tile plus a 3-pixel halo in LDS as float4 (direction, L/p_src or 0), so the
// neighbour picks of Sec. 4.2 are LDS reads, and maps block ids to tiles so
// that each XCD works on one contiguous band of the image (its L2 then holds
// the halo rows its neighbours share).
#pragma once
#include "pg_device.hpp"

namespace pgk {

struct ViewK {
  int W, H, pitch;
  const float *n, *o, *z, *rough, *alb, *mv;
  const uint8_t *mask;
};

struct ParamsK {
  uint32_t key0, key1, frame, view;
  int k_max;
  float pi_init, pi_lo, pi_hi, eps, tau_z, tau_n, rough_min, s_d, f0;
  uint32_t flags;
  float stale_tau;
  // material constants derived on the host (FP32, as the device would round
  // them), so that kernels take them as uniform operands
  float s_d_pi, one_m_f0, one_m_sd_q;  // s_d / pi, 1 - f0, (1 - s_d) / (4 pi)
};

struct SamplesK {
  int spp;
  float *dir, *pmix, *pb, *L;
  uint8_t *strat;
};

constexpr uint32_t kNoClamp = 1u;
constexpr uint32_t kStaleReset = 4u;
constexpr int kR = 3;                       // pick radius: 7x7 window
constexpr int kSide = 2 * kR + 1;
constexpr int kCand = kSide * kSide - 1;    // 48 neighbours

// Blocks are dealt to the 8 XCDs round robin; xcd_tile gives XCD j the j-th
// contiguous run of the n tiles, so that neighbouring tiles (which share
// cache lines and halos) are fetched into the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
  // blocks are dealt to the 8 XCDs round robin; give XCD j the j-th
  // contiguous run of tiles
  const int xcd = bid & 7, local = bid >> 3;
  const int base = n >> 3, rem = n & 7;
  return xcd * base + min(xcd, rem) + local;
}

// Streaming kernels: one 64x4 pixel tile per block of a 1-D grid, tiles in
// XCD bands.
__device__ __forceinline__ void stream_xy(int W, int H, int &x, int &y) {
  const int tx = (W + 63) >> 6, n = tx * ((H + 3) >> 2);
  const int t = xcd_tile((int)blockIdx.x, n);
  x = (t % tx) * 64 + (int)threadIdx.x;
  y = (t / tx) * 4 + (int)threadIdx.y;
}

__device__ __forceinline__ V3 load3(const float *p, int plane, int idx) {
  return V3{at(p, idx), at(p + plane, idx), at(p + 2 * plane, idx)};
}

__device__ __forceinline__ void gamma_reset(const ParamsK &P, float g[8]) {
  g[0] = 0.5f;
  g[1] = 0.5f;
  g[2] = 1.0f / 12.0f;
  g[3] = 0.0f;
  g[4] = 1.0f / 12.0f;
  g[5] = P.pi_init;
  g[6] = 0.0f;
  g[7] = 0.0f;
}

// Per-pixel material constants in the local frame.
__device__ __forceinline__ Pixel make_pixel(const ParamsK &P, V3 n, V3 o, float rough, float albedo) {
  Pixel px;
  px.f = make_frame(n);
  px.wo = to_local(px.f, normalized(o));
  const float alpha = rough * rough;
  px.alpha2 = alpha * alpha;
  px.albedo_pi = albedo * kInvPi;
  const float g1 = smith_g1(px.wo, px.alpha2) * frcp(2.0f * kPi * px.wo.z);
  px.f0_g1 = P.f0 * g1;
  px.omf0_g1 = P.one_m_f0 * g1;
  px.s_d = P.s_d;
  px.s_d_pi = P.s_d_pi;
  px.one_m_sd_q = P.one_m_sd_q;
  return px;
}

// ---------------------------------------------------------------------------
// Reprojection of one pixel (Sec. 3.1).  The decisions that turn FP32 inputs
// into a source address or a reset flag use explicit operation orders:
// validity and the normal test are fma(z, z', fma(y, y', x * x')), the
// address is (x + 1/2) - mv, the depth test |z - z'| > tau z.
// The G-buffer values of one pixel that both reprojection and sampling read.
struct PixelIn {
  V3 n, o;
  float rough;
};

__device__ __forceinline__ PixelIn load_pixel(const ViewK &v, int idx) {
  const int plane = v.H * v.pitch;
  return PixelIn{load3(v.n, plane, idx), load3(v.o, plane, idx), v.rough[idx]};
}

template <typename TG>
__device__ __forceinline__ int reproject_pixel(const ParamsK &P, const ViewK &cur, const ViewK &prev,
                                               const TG *__restrict__ gprev, bool has_prev, int x,
                                               int y, const PixelIn &pi, float g[8]) {
  const int plane = cur.H * cur.pitch;
  const int idx = y * cur.pitch + x;
  const V3 n = pi.n;
  const bool guided = dot3(n, pi.o) > 0.0f && pi.rough >= P.rough_min;
  // everything read at p, then everything read at the source q: two rounds
  // of loads whatever the tests decide
  float zp = 0.0f, mx = 0.0f, my = 0.0f;
  bool keep = has_prev && guided;
  if (keep) {
    zp = cur.z[idx];
    if (cur.mv) {
      mx = cur.mv[idx];
      my = cur.mv[plane + idx];
    }
    if (cur.mask != nullptr && cur.mask[idx] != 0) keep = false;
  }
  int qx = 0, qy = 0;
  if (keep) {
    const float fx = ((float)x + 0.5f) - mx;
    const float fy = ((float)y + 0.5f) - my;
    if (fx >= 0.0f && fy >= 0.0f && fx < (float)prev.W && fy < (float)prev.H) {
      qx = (int)floorf(fx);
      qy = (int)floorf(fy);
    } else {
      keep = false;
    }
  }
  if (keep) {
    const int pplane = prev.H * prev.pitch;
    const int qidx = qy * prev.pitch + qx;
    const float zq = prev.z[qidx];
    const V3 nq = load3(prev.n, pplane, qidx);
    gamma_load(gprev, pplane, qidx, g);
    if (fabsf(zp - zq) > P.tau_z * zp) keep = false;
    if (dot3(n, nq) < P.tau_n) keep = false;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (!isfinite(g[c])) keep = false;
    if (keep && !(n.x == nq.x && n.y == nq.y && n.z == nq.z)) {
      // change of hemisphere: keep the world direction of M(mu)
      const Frame fq = make_frame(nq);
      const Frame fp = make_frame(n);
      const V3 lq = sq2hemi(fminf(fmaxf(g[0], 0.0f), 1.0f), fminf(fmaxf(g[1], 0.0f), 1.0f));
      const V3 lp = to_local(fp, to_world(fq, lq));
      if (lp.z <= 0.0f) {
        keep = false;
      } else {
        hemi2sq(normalized(lp), g[0], g[1]);
      }
    }
  }
  if (!keep) {
    gamma_reset(P, g);
    return -1;
  }
  return qy * prev.W + qx;
}

// First-bounce estimate of one pixel: the mean over its samples of
// f_r L cos / D (null samples count zero), the Monte Carlo estimator of the
// reflected radiance with the mixture density of the samples.
__global__ __launch_bounds__(256) void k_estimate(ParamsK P, ViewK v, SamplesK S, float *__restrict__ out) {
  int x, y;
  stream_xy(v.W, v.H, x, y);
  if (x >= v.W || y >= v.H) return;
  const int plane = v.H * v.pitch;
  const int idx = y * v.pitch + x;
  const int splane = S.spp * plane;
  const V3 n = load3(v.n, plane, idx), o = load3(v.o, plane, idx);
  float acc = 0.0f;
  if (dot3(n, o) > 0.0f) {
    const Pixel px = make_pixel(P, n, o, v.rough[idx], v.alb[idx]);
    for (int s = 0; s < S.spp; ++s) {
      const int r = (s * v.H + y) * v.pitch + x;
      const uint8_t code = S.strat[r];
      const float D = S.pmix[r];
      if (!(code == 1 || code == 2) || !(D > 0.0f)) continue;
      const V3 l = to_local(px.f, normalized(V3{S.dir[r], S.dir[splane + r], S.dir[2 * splane + r]}));
      if (l.z <= 0.0f) continue;
      float f, pb;
      brdf_eval(px, l, f, pb);
      acc += f * S.L[r] * l.z / D;
    }
    acc /= (float)S.spp;
  }
  out[idx] = acc;
}

// Analytic incident radiance (stand-in for the trace).  For unit w and xi,
// w . xi - 1 = -|w - xi|^2 / 2, which has no cancellation near the axis.
struct LightsK {
  int count;
  float ambient;
  float l[8][5];
};

__device__ __forceinline__ float light_radiance(const LightsK &Lt, uint32_t bits, V3 wdir) {
  const V3 w = normalized(wdir);
  float L = Lt.ambient;
  for (int k = 0; k < Lt.count; ++k) {
    if (!((bits >> k) & 1u)) continue;
    const V3 a = V3{w.x - Lt.l[k][0], w.y - Lt.l[k][1], w.z - Lt.l[k][2]};
    L = fmaf(Lt.l[k][4], expf(-0.5f * Lt.l[k][3] * dot3(a, a)), L);
  }
  return L;
}

// ---------------------------------------------------------------------------
// Sampling of one pixel (Sec. 3.1, Eq. (2)).  Each strategy's own density is
// taken in its sample space (Gaussian from z, GGX from xi_1), the other
// component from the direction.
// With Lt given, the radiance of each sample is evaluated as well (the
// batched frame fuses the trace stand-in into this pass).
__device__ __forceinline__ void sample_pixel(const ParamsK &P, const ViewK &v, const SamplesK &S,
                                             int x, int y, const PixelIn &pi, const float g[8],
                                             const LightsK *Lt = nullptr, uint32_t visbits = 0) {
  const int plane = v.H * v.pitch;
  const int splane = S.spp * plane;
  const V3 n = pi.n;
  const V3 o = pi.o;
  const float rough = pi.rough;
  const bool valid = dot3(n, o) > 0.0f;
  const bool guided = valid && rough >= P.rough_min;
  const float pe = (guided && g[7] >= 1.0f) ? g[5] : 0.0f;
  const Pixel px = make_pixel(P, n, o, rough, 0.0f);
  const Gauss G = gauss_setup(g[0], g[1], g[2], g[3], g[4], P.eps);
  const uint32_t pix = (uint32_t)(y * v.W + x);
  for (int s = 0; s < S.spp; ++s) {
    const int rec = (s * v.H + y) * v.pitch + x;
    uint8_t code = 0;
    V3 l = V3{0.0f, 0.0f, 0.0f};
    float D = 0.0f, pb = 0.0f;
    if (valid) {
      const uint4 w4 = philox4x32_10(pix, P.frame, (uint32_t)s, P.view, P.key0, P.key1);
      const float zeta = u24(w4.x), xl = u24(w4.y), x1 = u24(w4.z), x2 = u24(w4.w);
      float sn, cs;
      sincospi_small(2.0f * x2, &sn, &cs);
      // the guided and the cosine draws take p_b from the direction, after
      // the branches, so that a wave whose lanes took both evaluates it once
      bool pb_dir = false;
      float pgz = 0.0f;  // the Gaussian density of a guided draw, from z
      if (zeta < pe) {
        // -2 ln(1 - x1) = -2 ln2 log2(1 - x1); 1 - x1 >= 2^-24 is normal
        const float rho = fsqrt(-1.38629436f * __builtin_amdgcn_logf(1.0f - x1));
        const float z1 = rho * cs, z2 = rho * sn;
        const float ux = fmaf(G.l11, z1, G.mx);
        const float uy = fmaf(G.l22, z2, fmaf(G.l21, z1, G.my));
        if (ux >= 0.0f && ux <= 1.0f && uy >= 0.0f && uy <= 1.0f) {
          l = sq2hemi(ux, uy);
          pgz = G.norm * __builtin_amdgcn_exp2f(-0.72134752f * fmaf(z1, z1, z2 * z2));
          pb_dir = l.z > 0.0f;
          code = 2;
        } else {
          code = 3;
        }
      } else if (xl < P.s_d) {
        const float r = fsqrt(x1);
        l = V3{r * cs, r * sn, fsqrt(1.0f - x1)};
        pb_dir = l.z > 0.0f;
        code = pb_dir ? 1 : 4;
      }
      if (pb_dir) pb = brdf_pdf_only(px, l);
      if (code == 2) {
        D = fmaf(pe, pgz, (1.0f - pe) * pb);
      } else if (code == 0) {
        // the GGX draw (the only strategy left without a code)
        // x1 <= 1 - 2^-24, so 1 - x1 and t2 (0 or >= alpha^2 2^-24) are normal
        const float t2 = px.alpha2 * x1 * frcp(1.0f - x1);
        const float ch = __builtin_amdgcn_rsqf(1.0f + t2);
        const float sh = fsqrt(t2) * ch;
        const V3 h = V3{sh * cs, sh * sn, ch};
        const float woh = dot3(px.wo, h);
        l = V3{2.0f * woh * h.x - px.wo.x, 2.0f * woh * h.y - px.wo.y, 2.0f * woh * h.z - px.wo.z};
        const bool ok = l.z > 0.0f && woh > 0.0f;
        if (ok) {
          // GGX density of the drawn normal in closed form of xi_1:
          // D(h) = (1 - xi_1 (1 - alpha^2))^2 / (pi alpha^2)
          const float q = fmaf(-x1, 1.0f - px.alpha2, 1.0f);
          const float pggx = 0.25f * kInvPi * q * q * ch * frcp(px.alpha2 * woh);
          pb = fmaf(px.s_d * kInvPi, l.z, (1.0f - px.s_d) * pggx);
        }
        code = ok ? 1 : 4;
      }
      if (code == 1) {  // a BRDF draw: the Gaussian's density from the direction
        float pg = 0.0f;
        if (pe > 0.0f) {
          float ux, uy;
          hemi2sq(l, ux, uy);
          pg = gauss_pdf_fast(G, ux, uy);
        }
        D = fmaf(pe, pg, (1.0f - pe) * pb);
      }
    }
    V3 w = V3{0.0f, 0.0f, 0.0f};
    if (code == 1 || code == 2) {
      w = to_world(px.f, l);
    } else {
      D = 0.0f;
      pb = 0.0f;
    }
    S.dir[rec] = w.x;
    S.dir[splane + rec] = w.y;
    S.dir[2 * splane + rec] = w.z;
    S.pmix[rec] = D;
    S.pb[rec] = pb;
    S.strat[rec] = code;
    if (Lt) S.L[rec] = (code == 1 || code == 2) ? light_radiance(*Lt, visbits, w) : 0.0f;
  }
}

template <typename TG>
__global__ __launch_bounds__(256) void k_reproject(ParamsK P, ViewK cur, ViewK prev,
                                                   const TG *__restrict__ gprev, TG *__restrict__ gout,
                                                   int32_t *__restrict__ src_index, int has_prev) {
  int x, y;
  stream_xy(cur.W, cur.H, x, y);
  if (x >= cur.W || y >= cur.H) return;
  float g[8];
  const int idx = y * cur.pitch + x;
  const int src = reproject_pixel(P, cur, prev, gprev, has_prev != 0, x, y, load_pixel(cur, idx), g);
  gamma_store(gout, cur.H * cur.pitch, idx, g);
  if (src_index) src_index[idx] = src;
}

template <typename TG>
__global__ __launch_bounds__(256) void k_sample(ParamsK P, ViewK v, const TG *__restrict__ gamma,
                                                SamplesK S) {
  int x, y;
  stream_xy(v.W, v.H, x, y);
  if (x >= v.W || y >= v.H) return;
  float g[8];
  const int idx = y * v.pitch + x;
  gamma_load(gamma, v.H * v.pitch, idx, g);
  sample_pixel(P, v, S, x, y, load_pixel(v, idx), g);
}

// Reprojection and sampling of one pixel: the reprojected model stays in
// registers, the sample pass sees it exactly as stored (rounded to TG), and
// the state is stored last (after the G-buffer has been read once).
template <typename TG>
__device__ __forceinline__ void reproject_sample_pixel(const ParamsK &P, const ViewK &cur, const ViewK &prev,
                                                       const TG *__restrict__ gprev, TG *__restrict__ gout,
                                                       const SamplesK &S, bool has_prev, int x, int y,
                                                       const LightsK *Lt = nullptr,
                                                       const uint8_t *vis = nullptr) {
  const int idx = y * cur.pitch + x;
  const PixelIn pi = load_pixel(cur, idx);
  const uint32_t visbits = vis ? vis[idx] : 0u;
  float g[8];
  reproject_pixel(P, cur, prev, gprev, has_prev, x, y, pi, g);
  float gs[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    TG t;
    gamma_put(&t, c, g[c]);
    gs[c] = gamma_get(&t, c);
  }
  sample_pixel(P, cur, S, x, y, pi, gs, Lt, visbits);
  gamma_store(gout, cur.H * cur.pitch, idx, g);
}

template <typename TG>
__global__ __launch_bounds__(256) void k_reproject_sample(ParamsK P, ViewK cur, ViewK prev,
                                                          const TG *__restrict__ gprev,
                                                          TG *__restrict__ gout, SamplesK S,
                                                          int has_prev) {
  int x, y;
  stream_xy(cur.W, cur.H, x, y);
  if (x >= cur.W || y >= cur.H) return;
  reproject_sample_pixel(P, cur, prev, gprev, gout, S, has_prev != 0, x, y);
}

// Densities of given directions.
template <typename TG>
__global__ __launch_bounds__(256) void k_pdf(ParamsK P, ViewK v, const TG *__restrict__ gamma, int n_per_px,
                                             const float *__restrict__ dir, float *__restrict__ pmix,
                                             float *__restrict__ pguide, float *__restrict__ pbrdf) {
  int x, y;
  stream_xy(v.W, v.H, x, y);
  if (x >= v.W || y >= v.H) return;
  const int plane = v.H * v.pitch;
  const int idx = y * v.pitch + x;
  const int dplane = n_per_px * plane;
  float g[8];
  gamma_load(gamma, plane, idx, g);
  const V3 n = load3(v.n, plane, idx);
  const V3 o = load3(v.o, plane, idx);
  const float rough = v.rough[idx];
  const bool valid = dot3(n, o) > 0.0f;
  const bool guided = valid && rough >= P.rough_min;
  const float pe = (guided && g[7] >= 1.0f) ? g[5] : 0.0f;
  const Pixel px = make_pixel(P, n, o, rough, 0.0f);
  const Gauss G = gauss_setup(g[0], g[1], g[2], g[3], g[4], P.eps);
  for (int j = 0; j < n_per_px; ++j) {
    const int r = (j * v.H + y) * v.pitch + x;
    const V3 w = V3{dir[r], dir[dplane + r], dir[2 * dplane + r]};
    float pg = 0.0f, pb = 0.0f;
    const float ww = dot3(w, w);
    if (valid && ww > 0.0f) {
      const V3 l = to_local(px.f, normalized(w));
      if (l.z > 0.0f) {
        float ux, uy;
        hemi2sq(l, ux, uy);
        pg = gauss_pdf_acc(G, ux, uy);
        pb = brdf_pdf_only(px, l);
      }
    }
    pmix[r] = fmaf(pe, pg, (1.0f - pe) * pb);
    if (pguide) pguide[r] = pg;
    if (pbrdf) pbrdf[r] = pb;
  }
}


__global__ __launch_bounds__(256) void k_light(LightsK Lt, ViewK v, const uint8_t *__restrict__ vis,
                                               SamplesK S) {
  int x, y;
  stream_xy(v.W, v.H, x, y);
  if (x >= v.W || y >= v.H) return;
  const int plane = v.H * v.pitch;
  const int idx = y * v.pitch + x;
  const int splane = S.spp * plane;
  const uint32_t bits = vis[idx];
  for (int s = 0; s < S.spp; ++s) {
    const int r = (s * v.H + y) * v.pitch + x;
    const uint8_t code = S.strat[r];
    S.L[r] = (code == 1 || code == 2)
                 ? light_radiance(Lt, bits, V3{S.dir[r], S.dir[splane + r], S.dir[2 * splane + r]})
                 : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// Training pass (Sec. 3.2, Sec. 4.2).
//
// Block = one TW x TH tile; LDS holds the records of the tile and a
// 3-pixel halo for every sample index: float4 (direction, L / p_src) with 0
// in the last slot for records that are not BRDF-strategy samples or lie
// outside the image (such records add nothing to any sum, which is the same
// as leaving them out of the training set).

template <int TW, int TH>
__device__ __forceinline__ void stage_records(const ViewK &v, const SamplesK &S, float4 *lds, int tx0,
                                              int ty0, int s0 = 0) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH;
  constexpr int IT = (SA + NT - 1) / NT;  // records of one sample plane per thread
  const int plane = v.H * v.pitch;
  const int splane = S.spp * plane;
  int gi[IT];
  bool in[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = threadIdx.x + i * NT;
    // e < 2^13, so the float quotient floors exactly
    const int sy = (int)(((float)e + 0.5f) * (1.0f / SW));
    const int sx = e - (int)__umul24((uint32_t)sy, (uint32_t)SW);
    const int gx = tx0 - kR + sx, gy = ty0 - kR + sy;
    in[i] = e < SA && gx >= 0 && gy >= 0 && gx < v.W && gy < v.H;
    gi[i] = row_off(gy, v.pitch) + gx;  // used only inside the image
  }
  for (int s = s0; s < S.spp; ++s) {
    // every load of this sample plane is issued before the first use
    uint8_t st[IT];
    float px[IT], py[IT], pz[IT], pl[IT], pp[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      st[i] = 0;
      px[i] = py[i] = pz[i] = pl[i] = pp[i] = 0.0f;
      if (in[i]) {
        const int o = s * plane + gi[i];
        st[i] = at(S.strat, o);
        pp[i] = at(S.pb, o);
        px[i] = at(S.dir, o);
        py[i] = at(S.dir + splane, o);
        pz[i] = at(S.dir + 2 * splane, o);
        pl[i] = at(S.L, o);
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = threadIdx.x + i * NT;
      if (IT * NT == SA || e < SA) {
        // a BRDF sample's density is a normal number (at least s_d cos/pi of
        // a valid draw, or the GGX density of the drawn normal)
        const bool ok = st[i] == 1 && pp[i] > 0.0f;
        lds[s * SA + e] = ok ? make_float4(px[i], py[i], pz[i], pl[i] * frcp(fmaxf(pp[i], 1.17549435e-38f)))
                             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
  }
}

// Running sums of one E-step: B0 = sum w, B1 = sum w gamma, and the
// weighted mean (mx, my) and normalised scatter (sxx, sxy, syy) of the
// samples' points under the weights v = w gamma, updated per sample in the
// pairwise form
//   m += (v / B1') d,   S = (B1 / B1') (S + (v / B1') d d^T),   d = r - m,
// which has no cancellation when a heavy sample follows light ones.  The
// points are r = u - mu, relative to the lobe's mean before the step (the
// value the Gaussian term needs anyway, exact near the mean); accum_to_unit
// adds the mean back once, after the last sample.  A Gaussian weight below
// FP32's normal range counts as no evidence, so the reciprocal of B1' is
// always of a normal number.
struct Accum {
  float B0, B1, mx, my, sxx, sxy, syy;
};

// The mean of the points r = u - mu back to u (the scatter is the same).
__device__ __forceinline__ void accum_to_unit(Accum &a, const LobeTerm &t) {
  a.mx += 0.5f - t.hx;
  a.my += 0.5f - t.hy;
}

// Stepwise merge of one frame's E-step sums into the state (Sec. 3.2):
// eta = 1/(k+1) and the evidence W; only ratios of evidences appear, so a
// subnormal B1 is harmless.
__device__ __forceinline__ void em_merge_online(const ParamsK &P, float g[8], const Accum &a) {
  const float eta = frcp(g[7] + 1.0f);  // k + 1 in [1, kMax + 1]
  const float sw = fmaf(1.0f - eta, g[6], eta * a.B0);
  const float so = (1.0f - eta) * g[5] * g[6];
  const float sn = eta * a.B1;
  const float sg = so + sn;
  if (sg > 0.0f && a.B1 > 0.0f) {
    float al, be;
    div2_pos(so, sn, sg, al, be);
    const float dx = g[0] - a.mx, dy = g[1] - a.my;
    const float ab = al * be;
    g[0] = fmaf(al, g[0], be * a.mx);
    g[1] = fmaf(al, g[1], be * a.my);
    g[2] = fmaf(ab * dx, dx, fmaf(al, g[2], be * a.sxx));
    g[3] = fmaf(ab * dx, dy, fmaf(al, g[3], be * a.sxy));
    g[4] = fmaf(ab * dy, dy, fmaf(al, g[4], be * a.syy));
  }
  float pn = div_pos(sg, sw);  // sg <= sw: B1 <= B0 and pi <= 1
  if (!(P.flags & kNoClamp)) pn = fminf(fmaxf(pn, P.pi_lo), P.pi_hi);
  g[5] = pn;
  g[6] = sw;
  g[7] = fminf(g[7] + 1.0f, (float)P.k_max);
}

struct EmCtx {
  Pixel px;
  LobeTerm T;  // the lobe's Gaussian term
  float pi;
};

// One training sample of a list (its staged record is never zero: lists
// hold only BRDF-strategy records inside the image).  Mean and scatter
// accumulate relative to the lobe's centre (see Accum).
__device__ __forceinline__ void em_visit(const EmCtx &c, float4 r, Accum &a) {
  const V3 l = to_local(c.px.f, V3{r.x, r.y, r.z});
  if (l.z <= 0.0f) return;
  float ox, oy, f, pb;
  hemi2sq_c(l, ox, oy);
  const float rx = fmaf(0.5f, ox, c.T.hx), ry = fmaf(0.5f, oy, c.T.hy);
  brdf_eval(c.px, l, f, pb);
  const float w = r.w * f * l.z;
  const float ga = lobe_eval(c.T, rx, ry);
  const float gb = fmaf(-c.pi, pb, pb);  // (1 - pi) p_b, one rounding
  const float gam = ga * __builtin_amdgcn_rcpf(fmaxf(ga + gb, 1.17549435e-38f));
  a.B0 += w;
  const float vw = w * gam;
  if (vw >= 1.17549435e-38f) {
    const float bn = a.B1 + vw;
    const float rb = __builtin_amdgcn_rcpf(bn);
    const float fr = vw * rb, keep = a.B1 * rb;
    a.B1 = bn;
    const float dx = rx - a.mx, dy = ry - a.my;
    a.mx = fmaf(dx, fr, a.mx);
    a.my = fmaf(dy, fr, a.my);
    const float fx = fr * dx, fy = fr * dy;
    a.sxx = keep * fmaf(fx, dx, a.sxx);
    a.sxy = keep * fmaf(fx, dy, a.sxy);
    a.syy = keep * fmaf(fy, dy, a.syy);
  }
}

// Pick m of a pixel: the 16-bit field m of the stream-1 Philox words gives a
// code c uniform over (48 neighbours) x spp; returns the LDS index of that
// candidate.  All products fit 24 bits (full-rate v_mul_u32_u24); the code is
// split as c = o spp + s by (c ceil(2^16/spp)) >> 16, exact for c < 48 spp,
// and the neighbour o (centre skipped) of the 7x7 window sits at row o / 7 =
// (37 o) >> 8 (exact for o < 49), column o mod 7.
template <int SA, int SW>
__device__ __forceinline__ int pick_entry(uint4 w4, int m, uint32_t cs, uint32_t inv_spp, uint32_t spp,
                                          int own) {
  const int wsel = (m >> 1) & 3;
  const uint32_t word = wsel == 0 ? w4.x : wsel == 1 ? w4.y : wsel == 2 ? w4.z : w4.w;
  const uint32_t h = (m & 1) ? (word >> 16) : (word & 0xFFFFu);
  const uint32_t c = __umul24(h, cs) >> 16;
  const uint32_t o0 = __umul24(c, inv_spp) >> 16;
  const uint32_t s = c - __umul24(o0, spp);
  const uint32_t o = o0 + (o0 >= (uint32_t)(kCand / 2) ? 1u : 0u);
  const uint32_t row = __umul24(o, 37u) >> 8;
  return (int)__umul24(s, (uint32_t)SA) + own + (int)(o + __umul24(row, (uint32_t)(SW - kSide))) -
         (kR * SW + kR);
}

// Bytes of the pick table in dynamic LDS (after the records and the lists).
__host__ __device__ constexpr int pick_table_bytes(int spp) { return (kCand * spp * 2 + 15) & ~15; }

// Pick table of a tile shape: code c in [0, 48 spp) of a pick -> offset of
// its candidate's staged record from the pixel's own: s SA + dy SW + dx with
// (o, s) = (c div spp, c mod spp), the centre of the window skipped, and
// (dx, dy) = (o mod 7 - 3, o div 7 - 3).  Built once per block, so that a
// pick costs one LDS read instead of the integer arithmetic of pick_entry.
template <int SA, int SW>
__device__ __forceinline__ void build_pick_table(int16_t *tab, int spp) {
  // c div spp = (c ceil(2^16 / spp)) >> 16, exact for c < 48 spp
  const uint32_t inv_spp = (65536u + (uint32_t)spp - 1u) / (uint32_t)spp;
  for (int c = (int)threadIdx.x; c < kCand * spp; c += (int)blockDim.x) {
    const int o0 = (int)(__umul24((uint32_t)c, inv_spp) >> 16), s = c - o0 * spp;
    const int o = o0 + (o0 >= kCand / 2 ? 1 : 0);
    const int row = o / kSide;
    tab[c] = (int16_t)(s * SA + (row - kR) * SW + (o - row * kSide - kR));
  }
}

// The two-pass training tile (online EM from spp 4) holds the records of
// the first ceil(spp/2) sample planes at a time; its dynamic LDS: those
// records [PG][SA] float4, a validity bit for every candidate record of all
// planes [spp SA] (bytes rounded up to 16), the lists [spp+20][w h] uint16,
// the pick table and, per pixel, the list's entries in the first pass
// [w h] uint8.
__host__ __device__ constexpr int em2_planes(int spp) { return (spp + 1) >> 1; }
__host__ __device__ constexpr size_t em2_bits_bytes(int tw, int th, int spp) {
  return (((size_t)spp * (tw + 2 * kR) * (th + 2 * kR) + 31) / 32 * 4 + 15) & ~(size_t)15;
}
__host__ __device__ constexpr size_t em2_lds_front(int tw, int th, int spp) {
  return (size_t)(tw + 2 * kR) * (th + 2 * kR) * em2_planes(spp) * 16 + em2_bits_bytes(tw, th, spp) +
         (size_t)(spp + 20) * tw * th * 2 + (size_t)pick_table_bytes(spp) + (size_t)tw * th;
}

// Where a training tile's lists start in dynamic LDS (after the records, and
// in the two-pass tile after the validity bits); the pick table follows the
// lists.
template <int TW, int TH, bool TWO>
__device__ __forceinline__ uint16_t *em_lists(float4 *lds, int spp) {
  constexpr int SA = (TW + 2 * kR) * (TH + 2 * kR);
  if (TWO)
    return reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(lds + em2_planes(spp) * SA) +
                                        em2_bits_bytes(TW, TH, spp));
  return reinterpret_cast<uint16_t *>(lds + spp * SA);
}

// The pick table of a training tile, at its place in dynamic LDS (called by
// every thread before em_tile; em_tile's first barrier publishes it).
template <int TW, int TH, bool TWO = false>
__device__ __forceinline__ void build_em_pick_table(float4 *lds, int spp) {
  constexpr int SW = TW + 2 * kR, SA = SW * (TH + 2 * kR), NT = TW * TH;
  build_pick_table<SA, SW>(reinterpret_cast<int16_t *>(em_lists<TW, TH, TWO>(lds, spp) + (spp + 20) * NT), spp);
}

// Number of neighbour picks N(k) = 5 + floor(15 (kMax - k) / kMax) (Sec. 4.2).
__device__ __forceinline__ int n_picks(const ParamsK &P, int k) {
  k = k < 0 ? 0 : (k > P.k_max ? P.k_max : k);
  return 5 + (15 * (P.k_max - k)) / P.k_max;
}

// A list entry is the byte offset of its staged record from the start of the
// records area (below 64 KiB: the area is part of one block's LDS), so that
// the record's LDS address is the entry plus a constant.
__device__ __forceinline__ float4 list_record(const float4 *lds, uint32_t off) {
  return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(lds) + off);
}

// Calls f on the staged records of n list entries of one pixel, at rows
// j0, j0 + step, ... of its column (column `me` of the [rows][nt] list
// area).  AHEAD = 0: one record at a time (its entry's and its own LDS
// reads wait in turn); AHEAD = 1: the next record is read from LDS before
// f runs on the current one (its entry's read still waits); AHEAD = 2: the
// next record and the entry after it, so both dependent LDS reads of a
// visit pass during the previous visits' arithmetic (four more registers).
// Reads past the last entry repeat the last entry (always a staged record).
template <int AHEAD, typename F>
__device__ __forceinline__ void for_each_record(const float4 *rec, const uint16_t *list, int nt, int me, int j0,
                                                int step, int n, F &&f) {
  static_assert(AHEAD >= 0 && AHEAD <= 2, "look-ahead of at most two records");
  if (n <= 0) return;
  const uint16_t *col = list + me;
  if (AHEAD == 0) {
    for (int i = 0; i < n; ++i) f(list_record(rec, col[(j0 + step * i) * nt]));
    return;
  }
  const int last = n - 1;
  auto entry = [&](int i) { return (uint32_t)col[(j0 + step * min(i, last)) * nt]; };
  float4 r0 = list_record(rec, entry(0));
  if (AHEAD == 1) {
    for (int i = 0; i < n; ++i) {
      const float4 r1 = list_record(rec, entry(i + 1));
      f(r0);
      r0 = r1;
    }
  } else {
    uint32_t off1 = entry(1);
    for (int i = 0; i < n; ++i) {
      const uint32_t off2 = entry(i + 2);
      const float4 r1 = list_record(rec, off1);
      f(r0);
      r0 = r1;
      off1 = off2;
    }
  }
}

// Training list of one pixel: the LDS byte offsets of its kept candidates, in the
// order of the training set (own samples by sample index, then picks by pick
// index), stored in column `col` of the list area.  A candidate is kept when
// its staged record is a BRDF-strategy sample inside the image.  Candidates
// are examined eight at a time (one Philox call): their addresses are formed
// in registers and their records read together, then appended without
// branches (a rejected candidate's slot is overwritten by the next one; the
// area has room for every candidate).  Returns the list length.
template <int TW, int TH>
__device__ __forceinline__ int build_list(const ParamsK &P, const float4 *lds, const int16_t *ptab, uint16_t *list,
                                          int col, int lx, int ly, int npick, int spp, uint32_t pix) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH;
  const uint32_t cs = (uint32_t)(kCand * spp);
  const int own = (ly + kR) * SW + (lx + kR);
  int n = 0;
  {
    float wv[kMaxSpp];
#pragma unroll
    for (int s = 0; s < kMaxSpp; ++s) wv[s] = s < spp ? lds[s * SA + own].w : 0.0f;
#pragma unroll
    for (int s = 0; s < kMaxSpp; ++s)
      if (s < spp) {
        list[n * NT + col] = (uint16_t)((s * SA + own) << 4);
        n += wv[s] != 0.0f ? 1 : 0;
      }
  }
  for (int m0 = 0; m0 < npick; m0 += 8) {
    const uint4 w4 = philox4x32_10(pix, P.frame, (1u << 16) | (uint32_t)(m0 >> 3), P.view, P.key0, P.key1);
    int e[8];
    float wv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      // the 16-bit field j of the four words, scaled to a code in [0, 48 spp)
      const uint32_t word = (j >> 1) == 0 ? w4.x : (j >> 1) == 1 ? w4.y : (j >> 1) == 2 ? w4.z : w4.w;
      const uint32_t h = (j & 1) ? (word >> 16) : (word & 0xFFFFu);
      e[j] = own + ptab[__umul24(h, cs) >> 16];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) wv[j] = lds[e[j]].w;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (m0 + j < npick) {
        list[n * NT + col] = (uint16_t)(e[j] << 4);
        n += wv[j] != 0.0f ? 1 : 0;
      }
  }
  return n;
}

// Rejection of a stale history (the stronger rejection of reprojected models
// that Sec. 5 leaves open, as read here): the weighted log-likelihood of the
// pixel's training set under the model, l_m = sum w log(pi p_g + (1 - pi)
// p_b), against the one under a new model (reset lobe, pi_init), l_r; the
// history is stale when l_m - l_r < -stale_tau sum w.  A pass of its own
// over the list, so that the E-step is untouched when the test is off.
__device__ __forceinline__ bool stale_history(const ParamsK &P, const Pixel &px, const float g[8],
                                              const float4 *lds, const uint16_t *list, int me, int len, int nt) {
  const Gauss G = gauss_setup(g[0], g[1], g[2], g[3], g[4], P.eps);
  const Gauss G0 = gauss_setup(0.5f, 0.5f, 1.0f / 12.0f, 0.0f, 1.0f / 12.0f, P.eps);
  const float pi = g[5], pi0 = P.pi_init;
  float lm = 0.0f, lr = 0.0f, ws = 0.0f;
  for (int j = 0; j < len; ++j) {
    const float4 r = list_record(lds, list[j * nt + me]);
    const V3 l = to_local(px.f, V3{r.x, r.y, r.z});
    if (l.z <= 0.0f) continue;
    float ux, uy, f, pb;
    hemi2sq(l, ux, uy);
    brdf_eval(px, l, f, pb);
    const float w = r.w * f * l.z;
    const float dm = fmaf(pi, gauss_pdf_acc(G, ux, uy), (1.0f - pi) * pb);
    const float dr = fmaf(pi0, gauss_pdf_acc(G0, ux, uy), (1.0f - pi0) * pb);
    if (!(w > 0.0f) || !(dm > 0.0f) || !(dr > 0.0f)) continue;
    lm = fmaf(w, __logf(dm), lm);
    lr = fmaf(w, __logf(dr), lr);
    ws += w;
  }
  return ws > 0.0f && (lm - lr) < -P.stale_tau * ws;
}

// Counting sort of the tile's items by decreasing work `len` (0 .. kMaxLen -
// 1) so that the lanes of a wave carry nearly equal work (the order inside a
// class is irrelevant: a pixel's arithmetic does not depend on the lane that
// runs it).  The k-th heaviest group of 64 items goes to wave (k + rot) mod
// waves, so that the heavy waves of the blocks resident on a CU do not all
// land on the same SIMD.  cnt[0 .. kMaxLen) must be zero and visible to the
// block on entry.  Each thread offers `item`; returns the item this lane
// takes.
constexpr int kMaxLen = kMaxSpp + 21;

template <int NT>
__device__ __forceinline__ int balance(int len, int item, int *cnt, uint16_t *perm, int rot) {
  static_assert(kMaxLen <= 32, "one half-wave scans the classes");
  const int rank = atomicAdd(&cnt[len], 1);
  __syncthreads();
  if (threadIdx.x < 64) {
    // wave 0: cnt[b] <- items in the classes heavier than b (suffix scan)
    const int l = threadIdx.x;
    const int c = l < kMaxLen ? cnt[l] : 0;
    int x = c;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
      const int y = __shfl_down(x, d, 64);
      if (l + d < 32) x += y;
    }
    if (l < kMaxLen) cnt[l] = x - c;
  }
  __syncthreads();
  constexpr int NW = NT / 64;
  const int pos = cnt[len] + rank;                                // rank in the sorted order
  const int wave = NW > 1 ? ((pos >> 6) + rot) % NW : 0;
  perm[wave * 64 + (pos & 63)] = (uint16_t)item;
  __syncthreads();
  return perm[threadIdx.x];
}

// LDS of one training tile besides the dynamic records/state/lists area.
template <int NT>
struct EmShared {
  int cnt[2][kMaxLen];
  uint16_t perm[NT];
  uint8_t work[NT];  // per pixel: candidate count, then list length
};

// Dynamic LDS of the single-lobe training kernels: the records
// [spp][h+6][w+6] float4, the lists [spp+20][w h] uint16 and the pick table
// (the block's EmShared is static).  Keeping EmShared static measured 2% faster
// than placing it after the dynamic area, where the records would start at
// LDS address 0 and the list entries could serve as addresses directly.
__host__ __device__ constexpr size_t em_lds_front(int tw, int th, int spp) {
  return (size_t)(tw + 2 * kR) * (th + 2 * kR) * spp * 16 + (size_t)(spp + 20) * tw * th * 2 +
         (size_t)pick_table_bytes(spp);
}

// One thread's share of a training tile's inputs, held in registers while
// the loads are in flight: what decides its pixel's candidate count (epoch,
// normal, view direction, roughness; natural order) and its records of
// sample plane 0.
template <int TW, int TH>
struct EmInput {
  static constexpr int SW = TW + 2 * kR, SA = SW * (TH + 2 * kR), NT = TW * TH, IT = (SA + NT - 1) / NT;
  float k, rough;
  V3 n, o;
  uint32_t st[IT];
  float px[IT], py[IT], pz[IT], pl[IT], pp[IT];
};

// Issue the loads of a tile's inputs (no use of the results here).
template <typename TG, int TW, int TH>
__device__ __forceinline__ void em_load(const ViewK &v, const SamplesK &S, const TG *gamma, int tx0, int ty0,
                                        EmInput<TW, TH> &R) {
  using In = EmInput<TW, TH>;
  const int plane = v.H * v.pitch;
  const int t = threadIdx.x;
  const int x0 = tx0 + t % TW, y0 = ty0 + t / TW;
  R.k = R.rough = 0.0f;
  R.n = R.o = V3{0, 0, 0};
  if (x0 < v.W && y0 < v.H) {
    const int idx0 = row_off(y0, v.pitch) + x0;
    R.k = gamma_get(&at(gamma + 7 * plane, idx0), 7);
    R.rough = at(v.rough, idx0);
    R.n = load3(v.n, plane, idx0);
    R.o = load3(v.o, plane, idx0);
  }
  const int splane = S.spp * plane;
#pragma unroll
  for (int i = 0; i < In::IT; ++i) {
    const int e = t + i * In::NT;
    // e < 2^13, so the float quotient floors exactly
    const int sy = (int)(((float)e + 0.5f) * (1.0f / In::SW));
    const int sx = e - (int)__umul24((uint32_t)sy, (uint32_t)In::SW);
    const int gx = tx0 - kR + sx, gy = ty0 - kR + sy;
    R.st[i] = 0;
    R.px[i] = R.py[i] = R.pz[i] = R.pl[i] = R.pp[i] = 0.0f;
    if (e < In::SA && gx >= 0 && gy >= 0 && gx < v.W && gy < v.H) {
      const int o = row_off(gy, v.pitch) + gx;
      R.st[i] = at(S.strat, o);
      R.pp[i] = at(S.pb, o);
      R.px[i] = at(S.dir, o);
      R.py[i] = at(S.dir + splane, o);
      R.pz[i] = at(S.dir + 2 * splane, o);
      R.pl[i] = at(S.L, o);
    }
  }
}

// One training tile.  Its inputs arrive in R (what decides each pixel's
// candidate count, natural order; records of plane 0; further planes are
// staged here): stage the records in LDS; sort the pixels by candidate count
// and build each pixel's training list; sort them again by list length, load
// each pixel's state and material in that order and run the E- and M-steps;
// write the tile's Gamma back in natural order through LDS (full cache
// lines).  Every thread of the block calls it and
// none leaves early; a block that runs several tiles synchronises between
// them (the write-back area overlaps the records).
// Dynamic LDS: records [spp][SH][SW] float4, then lists [spp + 20][NT]
// uint16, then the pick table [48 spp] int16; the write-back reuses the area
// ([8][NT] float).
template <typename TG, int TW, int TH, bool STALE = false, bool BATCH = false>
__device__ __forceinline__ void em_tile(const ParamsK &P, const ViewK &v, const SamplesK &S, TG *gamma,
                                        int iterations, int tx0, int ty0, int rot, float4 *lds,
                                        EmShared<TW * TH> &sh, const EmInput<TW, TH> &R) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH, IT = EmInput<TW, TH>::IT;
  uint16_t *list = reinterpret_cast<uint16_t *>(lds + S.spp * SA);
  float *wb = reinterpret_cast<float *>(lds);  // write-back area, once the records are no longer read
  const int plane = v.H * v.pitch;
  const int t = threadIdx.x;
  const int x0 = tx0 + t % TW, y0 = ty0 + t / TW;
  const bool in_image = x0 < v.W && y0 < v.H;
  int16_t *ptab = reinterpret_cast<int16_t *>(list + (S.spp + 20) * NT);
  if (t < 2 * kMaxLen) (&sh.cnt[0][0])[t] = 0;
  // plane-0 records to LDS
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = t + i * NT;
    if (IT * NT == SA || e < SA) {
      // a BRDF sample's density is a normal number (at least s_d cos/pi of a
      // valid draw, or the GGX density of the drawn normal)
      const bool ok = R.st[i] == 1 && R.pp[i] > 0.0f;
      lds[e] = ok ? make_float4(R.px[i], R.py[i], R.pz[i], R.pl[i] * frcp(fmaxf(R.pp[i], 1.17549435e-38f)))
                  : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  if (S.spp > 1) stage_records<TW, TH>(v, S, lds, tx0, ty0, 1);
  // the number of candidates of this lane's pixel (0 when it is not trained)
  int ncand = 0;
  if (in_image && dot3(R.n, R.o) > 0.0f && R.rough >= P.rough_min) ncand = S.spp + n_picks(P, (int)R.k);
  sh.work[t] = (uint8_t)ncand;
  __syncthreads();
  // lists: pixels by decreasing candidate count
  int me;
  {
    const int pa = balance<NT>(ncand, t, sh.cnt[0], sh.perm, rot);
    const int nc = sh.work[pa];
    int len = 0;
    if (nc > 0) {
      const int lx = pa % TW, ly = pa / TW;
      len = build_list<TW, TH>(P, lds, ptab, list, pa, lx, ly, nc - S.spp, S.spp,
                               (uint32_t)(row_off(ty0 + ly, v.W) + tx0 + lx));
    }
    sh.work[pa] = (uint8_t)len;
    // E- and M-steps: pixels by decreasing list length
    me = balance<NT>(len, pa, sh.cnt[1], sh.perm, rot + 1);
  }
  const int len = sh.work[me];
  EmCtx c;
  float g[8];
  // every pixel of the tile, trained or not, passes its state to the
  // natural-order write-back through LDS (the loads run for the trained
  // lanes of the wave anyway)
  const int mex = tx0 + me % TW, mey = ty0 + me / TW;
  const bool me_in = mex < v.W && mey < v.H;
  const int idx = row_off(mey, v.pitch) + mex;
  if (me_in) gamma_load(gamma, plane, idx, g);
  if (len > 0) {
    c.px = make_pixel(P, load3(v.n, plane, idx), load3(v.o, plane, idx), at(v.rough, idx), at(v.alb, idx));
    if (STALE && !BATCH && g[7] >= 1.0f && stale_history(P, c.px, g, lds, list, me, len, NT)) gamma_reset(P, g);
  }
  if (len > 0) {  // otherwise no training sample (or no pixel): the model stays as it is
    const int iters = BATCH ? iterations : 1;
    for (int it = 0; it < iters; ++it) {
      c.T = lobe_term(gauss_setup(g[0], g[1], g[2], g[3], g[4], P.eps), g[5]);
      c.pi = g[5];
      Accum a = {0, 0, 0, 0, 0, 0, 0};
      // at spp 1 one record at a time: 8 waves per SIMD cover the LDS
      // latency, and a look-ahead's index arithmetic measured 3% slower;
      // above, the staged records leave 4-5 waves and the reads go ahead
      // (batch EM, with more state live, keeps one record at a time)
      if (!BATCH && S.spp > 1)
        for_each_record<2>(lds, list, NT, me, 0, 1, len, [&](float4 r) { em_visit(c, r, a); });
      else
        for_each_record<0>(lds, list, NT, me, 0, 1, len, [&](float4 r) { em_visit(c, r, a); });
      if (!(a.B0 > 0.0f)) break;
      accum_to_unit(a, c.T);
      if (!BATCH) {
        em_merge_online(P, g, a);
      } else {
        if (a.B1 > 0.0f) {
          g[0] = a.mx;
          g[1] = a.my;
          g[2] = a.sxx;
          g[3] = a.sxy;
          g[4] = a.syy;
        }
        float pn = div_pos(a.B1, a.B0);
        if (!(P.flags & kNoClamp)) pn = fminf(fmaxf(pn, P.pi_lo), P.pi_hi);
        g[5] = pn;
      }
    }
  }
  __syncthreads();  // records and lists are no longer read
  if (me_in) {
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) wb[ch * NT + me] = g[ch];
  }
  __syncthreads();
  if (in_image) {
    float go[8];
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) go[ch] = wb[ch * NT + t];
    gamma_store(gamma, plane, row_off(y0, v.pitch) + x0, go);
  }
}

// Two-pass training tile (online EM from spp 4).  Above spp 1 the staged
// records of every sample plane fill the LDS and few blocks share a CU (at
// spp 4 and 32x8, 3 blocks: VALU 53% busy; at spp 8, 18% occupancy).  Here
// the records of the first PG = ceil(spp/2) planes are staged, with one
// validity bit per candidate record of all planes; each pixel's list is built
// once, as in em_tile, storing its entries of the first planes from the
// front of its column and those of the last planes from the back; the E-step
// runs over the first planes, the records area is restaged with the last
// planes, and the same sums continue over them.  Each pass keeps the
// training set's order, so the result does not depend on the tile shape.

// Validity bits and (for planes below `pg`) records of sample planes
// [s0, s1) of a tile; with `bits` false only records, placed at plane
// s - s0.  Each thread's halo positions are computed once for all planes.
template <int TW, int TH>
__device__ __forceinline__ void stage2(const ViewK &v, const SamplesK &S, float4 *rec, uint32_t *vb, int tx0,
                                       int ty0, int s0, int s1, int pg, bool bits) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH;
  constexpr int IT = (SA + NT - 1) / NT;
  const int plane = v.H * v.pitch;
  const int splane = S.spp * plane;
  int gi[IT];
  bool in[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = threadIdx.x + i * NT;
    // e < 2^13, so the float quotient floors exactly
    const int sy = (int)(((float)e + 0.5f) * (1.0f / SW));
    const int sx = e - (int)__umul24((uint32_t)sy, (uint32_t)SW);
    const int gx = tx0 - kR + sx, gy = ty0 - kR + sy;
    in[i] = e < SA && gx >= 0 && gy >= 0 && gx < v.W && gy < v.H;
    gi[i] = row_off(gy, v.pitch) + gx;  // used only inside the image
  }
  for (int s = s0; s < s1; ++s) {
    const bool keep_rec = !bits || s < pg;
    const int rs = bits ? s : s - s0;  // plane index in the records area
    // every load of this sample plane is issued before the first use
    uint8_t st[IT];
    float px[IT], py[IT], pz[IT], pl[IT], pp[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      st[i] = 0;
      px[i] = py[i] = pz[i] = pl[i] = pp[i] = 0.0f;
      if (in[i]) {
        const int o = s * plane + gi[i];
        st[i] = at(S.strat, o);
        pp[i] = at(S.pb, o);
        if (keep_rec) {
          px[i] = at(S.dir, o);
          py[i] = at(S.dir + splane, o);
          pz[i] = at(S.dir + 2 * splane, o);
          pl[i] = at(S.L, o);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = threadIdx.x + i * NT;
      if (IT * NT == SA || e < SA) {
        // a BRDF sample's density is a normal number (at least s_d cos/pi of
        // a valid draw, or the GGX density of the drawn normal)
        const bool ok = st[i] == 1 && pp[i] > 0.0f;
        if (keep_rec)
          rec[rs * SA + e] = ok ? make_float4(px[i], py[i], pz[i], pl[i] * frcp(fmaxf(pp[i], 1.17549435e-38f)))
                                : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (bits && ok) {
          const int b = s * SA + e;
          atomicOr(&vb[b >> 5], 1u << (b & 31));
        }
      }
    }
  }
}

// Training list of one pixel for the two-pass tile: the same candidates in
// the same order as build_list, kept by their validity bit; an entry is the
// record's byte offset in its pass's records area, the first pass's entries
// from the front of column `col`, the last pass's from the back.  Returns
// the list length and the first pass's count in n0.
template <int TW, int TH>
__device__ __forceinline__ int build_list2(const ParamsK &P, const uint32_t *vb, const int16_t *ptab,
                                           uint16_t *list, int col, int lx, int ly, int npick, int spp,
                                           uint32_t pix, int &n0) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH;
  const int cap = spp + 20;
  const int split = em2_planes(spp) * SA;  // first record of the last pass
  const uint32_t cs = (uint32_t)(kCand * spp);
  const int own = (ly + kR) * SW + (lx + kR);
  int a = 0, b = 0;  // entries of the first and of the last pass
  auto put = [&](int e, bool ok) {
    const bool last = e >= split;
    const int slot = last ? cap - 1 - b : a;  // a rejected entry is overwritten by the next
    list[slot * NT + col] = (uint16_t)((last ? e - split : e) << 4);
    a += (ok && !last) ? 1 : 0;
    b += (ok && last) ? 1 : 0;
  };
#pragma unroll
  for (int s = 0; s < kMaxSpp; ++s)
    if (s < spp) {
      const int e = s * SA + own;
      put(e, (vb[e >> 5] >> (e & 31)) & 1u);
    }
  for (int m0 = 0; m0 < npick; m0 += 8) {
    const uint4 w4 = philox4x32_10(pix, P.frame, (1u << 16) | (uint32_t)(m0 >> 3), P.view, P.key0, P.key1);
    int e[8];
    uint32_t wv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      // the 16-bit field j of the four words, scaled to a code in [0, 48 spp)
      const uint32_t word = (j >> 1) == 0 ? w4.x : (j >> 1) == 1 ? w4.y : (j >> 1) == 2 ? w4.z : w4.w;
      const uint32_t h = (j & 1) ? (word >> 16) : (word & 0xFFFFu);
      e[j] = own + ptab[__umul24(h, cs) >> 16];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) wv[j] = vb[e[j] >> 5];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (m0 + j < npick) put(e[j], (wv[j] >> (e[j] & 31)) & 1u);
  }
  n0 = a;
  return a + b;
}

template <typename TG, int TW, int TH>
__device__ __forceinline__ void em_tile2(const ParamsK &P, const ViewK &v, const SamplesK &S, TG *gamma, int tx0,
                                         int ty0, int rot, float4 *lds, EmShared<TW * TH> &sh,
                                         const EmInput<TW, TH> &R) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH, IT = EmInput<TW, TH>::IT;
  const int spp = S.spp, pg = em2_planes(spp), cap = spp + 20;
  float4 *rec = lds;
  uint32_t *vb = reinterpret_cast<uint32_t *>(lds + pg * SA);
  const int nvb = (int)(em2_bits_bytes(TW, TH, spp) / 4);
  uint16_t *list = em_lists<TW, TH, true>(lds, spp);
  const int16_t *ptab = reinterpret_cast<const int16_t *>(list + cap * NT);
  uint8_t *work0 = reinterpret_cast<uint8_t *>(list + cap * NT) + pick_table_bytes(spp);
  float *wb = reinterpret_cast<float *>(lds);  // write-back area (records, bits, lists: all dead by then)
  const int plane = v.H * v.pitch;
  const int t = threadIdx.x;
  const int x0 = tx0 + t % TW, y0 = ty0 + t / TW;
  const bool in_image = x0 < v.W && y0 < v.H;
  if (t < 2 * kMaxLen) (&sh.cnt[0][0])[t] = 0;
  for (int w = t; w < nvb; w += NT) vb[w] = 0u;
  __syncthreads();  // the bits are zero before they are set
  // plane 0 from the registers, then the other planes
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = t + i * NT;
    if (IT * NT == SA || e < SA) {
      const bool ok = R.st[i] == 1 && R.pp[i] > 0.0f;
      rec[e] = ok ? make_float4(R.px[i], R.py[i], R.pz[i], R.pl[i] * frcp(fmaxf(R.pp[i], 1.17549435e-38f)))
                  : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (ok) atomicOr(&vb[e >> 5], 1u << (e & 31));
    }
  }
  stage2<TW, TH>(v, S, rec, vb, tx0, ty0, 1, spp, pg, true);
  int ncand = 0;
  if (in_image && dot3(R.n, R.o) > 0.0f && R.rough >= P.rough_min) ncand = spp + n_picks(P, (int)R.k);
  sh.work[t] = (uint8_t)ncand;
  __syncthreads();
  int me;
  {
    const int pa = balance<NT>(ncand, t, sh.cnt[0], sh.perm, rot);
    const int nc = sh.work[pa];
    int len = 0, n0 = 0;
    if (nc > 0) {
      const int lx = pa % TW, ly = pa / TW;
      len = build_list2<TW, TH>(P, vb, ptab, list, pa, lx, ly, nc - spp, spp,
                                (uint32_t)(row_off(ty0 + ly, v.W) + tx0 + lx), n0);
    }
    sh.work[pa] = (uint8_t)len;
    work0[pa] = (uint8_t)n0;
    // each pass lasts as long as its longest list in the wave, so the lanes
    // are grouped by the longer of their two parts (max(n0) + max(n1) per
    // wave), not by the whole list
    me = balance<NT>(max(n0, len - n0), pa, sh.cnt[1], sh.perm, rot + 1);
  }
  const int len = sh.work[me], n0 = work0[me];
  float g[8];
  const int mex = tx0 + me % TW, mey = ty0 + me / TW;
  const bool me_in = mex < v.W && mey < v.H;
  const int idx = row_off(mey, v.pitch) + mex;
  if (me_in) gamma_load(gamma, plane, idx, g);
  Accum a = {0, 0, 0, 0, 0, 0, 0};
  // the pixel's context is built for each pass (its loads hit the caches):
  // across the restaging only the sums and the state stay in registers
  if (len > 0) {
    EmCtx c;
    c.px = make_pixel(P, load3(v.n, plane, idx), load3(v.o, plane, idx), at(v.rough, idx), at(v.alb, idx));
    c.T = lobe_term(gauss_setup(g[0], g[1], g[2], g[3], g[4], P.eps), g[5]);
    c.pi = g[5];
    for_each_record<2>(rec, list, NT, me, 0, 1, n0, [&](float4 r) { em_visit(c, r, a); });
  }
  __syncthreads();  // the first planes' records are no longer read
  stage2<TW, TH>(v, S, rec, vb, tx0, ty0, pg, spp, 0, false);
  __syncthreads();
  if (len > 0) {
    EmCtx c;
    c.px = make_pixel(P, load3(v.n, plane, idx), load3(v.o, plane, idx), at(v.rough, idx), at(v.alb, idx));
    c.T = lobe_term(gauss_setup(g[0], g[1], g[2], g[3], g[4], P.eps), g[5]);
    c.pi = g[5];
    for_each_record<2>(rec, list, NT, me, cap - 1, -1, len - n0, [&](float4 r) { em_visit(c, r, a); });
    if (a.B0 > 0.0f) {  // otherwise no weight: the model stays as it is
      accum_to_unit(a, c.T);
      em_merge_online(P, g, a);
    }
  }
  __syncthreads();  // records and lists are no longer read
  if (me_in) {
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) wb[ch * NT + me] = g[ch];
  }
  __syncthreads();
  if (in_image) {
    float go[8];
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) go[ch] = wb[ch * NT + t];
    gamma_store(gamma, plane, row_off(y0, v.pitch) + x0, go);
  }
}

// One tile per block (blocks are mapped to XCD bands by xcd_tile); with the
// LDS and registers of a tile, several blocks share each CU, which hides the
// loads of one block behind the arithmetic of the others better than a
// persistent loop with register prefetch.
// TWO: the two-pass tile (online EM above spp 1; em2_lds_front).
template <typename TG, int TW, int TH, bool STALE, bool TWO = false, bool BATCH = false>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(TWO ? 5 : 8))) void k_em(ParamsK P, ViewK v, SamplesK S, TG *__restrict__ gamma,
                                               int iterations, int tiles_x, int n_tiles) {
  extern __shared__ float4 lds[];  // records, lists and the pick table (em_lds_front, em2_lds_front)
  __shared__ EmShared<TW * TH> sh;
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  const int tx0 = (tile % tiles_x) * TW, ty0 = (tile / tiles_x) * TH;
  build_em_pick_table<TW, TH, TWO>(lds, S.spp);  // before the loads: fewer live registers
  EmInput<TW, TH> R;
  em_load(v, S, gamma, tx0, ty0, R);
  if (TWO)
    em_tile2<TG, TW, TH>(P, v, S, gamma, tx0, ty0, (int)blockIdx.x, lds, sh, R);
  else
    em_tile<TG, TW, TH, STALE, BATCH>(P, v, S, gamma, iterations, tx0, ty0, (int)blockIdx.x, lds, sh, R);
}

// ---------------------------------------------------------------------------
// Weighted NLL of the mixture over the training set and its adjoint.
struct NllAccum {
  float loss, gmx, gmy, gxx, gxy, gyy, gl;
};

struct NllCtx {
  Pixel px;
  Gauss G;
  float pi, one_m_pi, mux, muy, ia, ib, ic;
};

__device__ __forceinline__ void nll_visit(const NllCtx &c, float4 r, NllAccum &a) {
  if (r.w == 0.0f) return;
  const V3 l = to_local(c.px.f, V3{r.x, r.y, r.z});
  if (l.z <= 0.0f) return;
  float ux, uy, f, pb;
  hemi2sq(l, ux, uy);
  brdf_eval(c.px, l, f, pb);
  const float w = r.w * f * l.z;
  const float pg = gauss_pdf_acc(c.G, ux, uy);
  const float ga = c.pi * pg;
  const float D = fmaf(c.one_m_pi, pb, ga);
  a.loss = fmaf(-w, logf(D), a.loss);
  const float gam = D > 0.0f ? ga / D : 0.0f;
  const float dx = ux - c.mux, dy = uy - c.muy;
  const float vx = fmaf(c.ia, dx, c.ib * dy), vy = fmaf(c.ib, dx, c.ic * dy);
  const float wg = w * gam;
  a.gmx = fmaf(-wg, vx, a.gmx);
  a.gmy = fmaf(-wg, vy, a.gmy);
  a.gxx = fmaf(-0.5f * wg, fmaf(vx, vx, -c.ia), a.gxx);
  a.gxy = fmaf(-0.5f * wg, fmaf(vx, vy, -c.ib), a.gxy);
  a.gyy = fmaf(-0.5f * wg, fmaf(vy, vy, -c.ic), a.gyy);
  a.gl = fmaf(-w, gam - c.pi, a.gl);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void k_nll(ParamsK P, ViewK v, SamplesK S, const float *__restrict__ theta,
                                                const float *__restrict__ grad_out, float *__restrict__ grad,
                                                float *__restrict__ nll, int tiles_x, int n_tiles) {
  extern __shared__ float4 lds[];
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH;
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  const int tx0 = (tile % tiles_x) * TW, ty0 = (tile / tiles_x) * TH;
  stage_records<TW, TH>(v, S, lds, tx0, ty0);
  __syncthreads();
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int x = tx0 + lx, y = ty0 + ly;
  if (x >= v.W || y >= v.H) return;
  const int plane = v.H * v.pitch;
  const int idx = y * v.pitch + x;
  const V3 n = load3(v.n, plane, idx);
  const V3 o = load3(v.o, plane, idx);
  const float rough = v.rough[idx];
  float th[8];
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) th[ch] = theta[ch * plane + idx];
  NllAccum a = {0, 0, 0, 0, 0, 0, 0};
  float gr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (dot3(n, o) > 0.0f && rough >= P.rough_min) {
    NllCtx c;
    c.px = make_pixel(P, n, o, rough, v.alb[idx]);
    const float l11 = th[2], l21 = th[3], l22 = th[4];
    const float sxx = l11 * l11, sxy = l11 * l21, syy = fmaf(l21, l21, l22 * l22);
    c.G = gauss_setup(th[0], th[1], sxx, sxy, syy, P.eps);
    c.pi = 1.0f / (1.0f + expf(-th[5]));
    c.one_m_pi = 1.0f - c.pi;
    c.mux = th[0];
    c.muy = th[1];
    const float A = sxx + P.eps, B = sxy, Cc = syy + P.eps;
    const float idet = 1.0f / fmaf(A, Cc, -B * B);
    c.ia = Cc * idet;
    c.ib = -B * idet;
    c.ic = A * idet;
    int k = (int)th[7];
    k = k < 0 ? 0 : (k > P.k_max ? P.k_max : k);
    const int npick = n_picks(P, k);
    const uint32_t pix = (uint32_t)(y * v.W + x);
    const uint32_t cs = (uint32_t)(kCand * S.spp);
    const uint32_t inv_spp = (65536u + (uint32_t)S.spp - 1u) / (uint32_t)S.spp;
    const int own = (ly + kR) * SW + (lx + kR);
    for (int s = 0; s < S.spp; ++s) nll_visit(c, lds[s * SA + own], a);
    uint4 w4 = make_uint4(0, 0, 0, 0);
    for (int m = 0; m < npick; ++m) {
      if ((m & 7) == 0) w4 = philox4x32_10(pix, P.frame, (1u << 16) | (uint32_t)(m >> 3), P.view, P.key0, P.key1);
      nll_visit(c, lds[pick_entry<SA, SW>(w4, m, cs, inv_spp, (uint32_t)S.spp, own)], a);
    }
    const float sc = grad_out ? grad_out[idx] : 1.0f;
    gr[0] = sc * a.gmx;
    gr[1] = sc * a.gmy;
    gr[2] = sc * 2.0f * fmaf(a.gxx, l11, a.gxy * l21);
    gr[3] = sc * 2.0f * fmaf(a.gxy, l11, a.gyy * l21);
    gr[4] = sc * 2.0f * (a.gyy * l22);
    gr[5] = sc * a.gl;
  }
  if (grad) {
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) grad[ch * plane + idx] = gr[ch];
  }
  if (nll) nll[idx] = a.loss;
}

// ---------------------------------------------------------------------------
// Batched frame: many views of any size and spp in two persistent launches
// (reprojection + sampling + light, then training) that read everything from
// a table in device memory, so that one captured graph (table upload + two
// kernels) replays later frames of all views once the table is re-packed.
struct BatchViewK {
  ViewK cur;
  const float *prev_n, *prev_z;
  const void *gprev;
  void *gout;
  SamplesK S;
  const uint8_t *vis;
  LightsK lights;
  uint32_t key0, key1, frame, view;
  int rs_begin, rs_tiles_x, em_begin, em_tiles_x;
};

// The views of a table are ordered by spp; the views of one spp form a class
// whose training tiles are contiguous in the tile list and run in a launch of
// their own, with the tile shape and LDS of that spp.
struct BatchClass {
  int spp, tile_w, tile_h, em_begin, em_end, pad[3];
};

struct BatchHeader {
  int n_views, rs_tiles, em_tiles, dtype, n_classes, magic, pad[2];
  ParamsK base;  // fields shared by every view (key, frame, view come per view)
  BatchClass cls[kMaxSpp];
};

constexpr int kBatchViewsOffset = (int)((sizeof(BatchHeader) + 63) / 64 * 64);

__device__ __forceinline__ const BatchViewK *batch_views(const char *table) {
  return reinterpret_cast<const BatchViewK *>(table + kBatchViewsOffset);
}

// The view owning tile t: the last one whose first tile is <= t (the tiles of
// consecutive views are contiguous).  Uniform across the block.
template <bool EM>
__device__ __forceinline__ int batch_find(const BatchViewK *vs, int n, int t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int b = EM ? vs[mid].em_begin : vs[mid].rs_begin;
    if (b <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ ParamsK batch_params(const ParamsK &base, const BatchViewK &bv) {
  ParamsK P = base;
  P.key0 = bv.key0;
  P.key1 = bv.key1;
  P.frame = bv.frame;
  P.view = bv.view;
  return P;
}

// Reprojection + sampling + light field over the 64x4 pixel tiles of all
// views, one block per tile (a persistent grid-stride loop held 72-80 VGPRs,
// this 60-62).  `dtype` is the launch's Gamma type: a table of another type,
// or with more tiles than the grid, is not processed.
template <typename TG>
__global__ __launch_bounds__(256) void k_rs_batched(const char *__restrict__ table, int dtype) {
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(table);
  if (hd->dtype != dtype) return;
  const int n_views = hd->n_views, n_tiles = hd->rs_tiles;
  const BatchViewK *vs = batch_views(table);
  // one block per tile, in tile order: blocks are dealt to the XCDs round
  // robin, so the views (ordered by spp) are interleaved over the XCDs
  const int t = (int)blockIdx.x;
  if (n_tiles > (int)gridDim.x || t >= n_tiles) return;  // more tiles than the grid: a different table
  const BatchViewK &bv = vs[batch_find<false>(vs, n_views, t)];
  const int local = t - bv.rs_begin;
  const int x = (local % bv.rs_tiles_x) * 64 + (int)(threadIdx.x & 63);
  const int y = (local / bv.rs_tiles_x) * 4 + (int)(threadIdx.x >> 6);
  const ViewK cur = bv.cur;
  if (x >= cur.W || y >= cur.H) return;
  const ParamsK P = batch_params(hd->base, bv);
  ViewK prev = cur;
  prev.n = bv.prev_n;
  prev.z = bv.prev_z;
  reproject_sample_pixel(P, cur, prev, (const TG *)bv.gprev, (TG *)bv.gout, bv.S, bv.frame > 0, x, y,
                         &bv.lights, bv.vis);
}

// Training over the TW x TH tiles of the views of class `cls`, one block per
// tile in XCD bands (like k_em: with no state carried from tile to tile the
// kernel fits 8 waves/SIMD; a persistent loop over tiles needed ~30 more
// VGPRs).  `spp_cap` is the spp the dynamic LDS was sized for; a table whose
// class differs from the launch (tile, spp, dtype, or more tiles than the
// grid) is not processed.
template <typename TG, int TW, int TH, bool TWO>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(TH == 2 ? 1 : (TWO ? 5 : 8)))) void k_em_batched(const char *__restrict__ table, int dtype, int cls,
                                                       int spp_cap) {
  extern __shared__ float4 lds[];  // sized for spp_cap (em_lds_front, em2_lds_front)
  __shared__ EmShared<TW * TH> sh;
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(table);
  if (hd->dtype != dtype || cls >= hd->n_classes) return;
  const BatchClass c = hd->cls[cls];
  if (c.spp > spp_cap || c.tile_w != TW || c.tile_h != TH) return;
  const int n_views = hd->n_views;
  const BatchViewK *vs = batch_views(table);
  const int n = c.em_end - c.em_begin;
  // a class with more tiles than the grid (a replayed launch for other views)
  // differs from the launch: not processed
  if (n > (int)gridDim.x || (int)blockIdx.x >= n) return;
  const int t = c.em_begin + xcd_tile((int)blockIdx.x, n);
  const BatchViewK &bv = vs[batch_find<true>(vs, n_views, t)];
  const int l = t - bv.em_begin;
  const int tx0 = (l % bv.em_tiles_x) * TW, ty0 = (l / bv.em_tiles_x) * TH;
  const ParamsK P = batch_params(hd->base, bv);
  build_em_pick_table<TW, TH, TWO>(lds, bv.S.spp);
  EmInput<TW, TH> R;
  em_load(bv.cur, bv.S, (const TG *)bv.gout, tx0, ty0, R);
  if (TWO)
    em_tile2<TG, TW, TH>(P, bv.cur, bv.S, (TG *)bv.gout, tx0, ty0, (int)blockIdx.x, lds, sh, R);
  else
    em_tile<TG, TW, TH>(P, bv.cur, bv.S, (TG *)bv.gout, 1, tx0, ty0, (int)blockIdx.x, lds, sh, R);
}

// Philox words for given counters (diagnostic entry).
__global__ void k_philox(int n, const uint32_t *__restrict__ ctr, uint32_t key0, uint32_t key1,
                         uint32_t *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key0, key1);
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

}  // namespace pgk
