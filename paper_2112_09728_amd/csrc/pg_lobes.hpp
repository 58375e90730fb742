// K Gaussian lobes per pixel: the single lobe of the mixture of Eq. (2)
// generalised to
//   D(w) = sum_j pi_j N_j(M^-1 w) / (2 pi) + (1 - sum_j pi_j) p_b(w),
// the limit of one Gaussian per pixel that Sec. 4.1 names lifted.  FP32
// state of 6K + 2 planes: lobe j at plane 6j holds (mu_x, mu_y, S_xx, S_xy,
// S_yy, pi_j), then W and k.
//
// Readings of the extension: a new model's lobes share Sigma = I/12 and
// pi_init/K at the distinct means (0.5 + (j - (K-1)/2) / 4, 0.5); zeta selects
// lobe j when it falls in [c_j, c_j + pi_j), c_j the sum of the earlier
// weights, else the BRDF; each lobe is merged with its own evidence like the
// single lobe; the clamp raises every weight to pi_lo/(4K) and scales them so
// that their sum lies in [pi_lo, pi_hi]; reprojection carries every lobe mean
// to the new hemisphere and starts a new model when any falls below it.
//
// Kernels: one lane per pixel.  The streaming pass (reprojection + sampling)
// and the densities use the 64x4 XCD-banded tiles of the single-lobe path;
// the training pass uses the single-lobe pass's LDS staging of a tile's
// records, its compacted training lists and its lane balancing, with the
// E-step and merge of K lobes.
#pragma once
#include "pg_kernels.hpp"

namespace pgk {

constexpr int kMaxLobes = 4;

template <int K>
__device__ __forceinline__ void lobes_reset(const ParamsK &P, float g[6 * K + 2]) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    g[6 * j + 0] = 0.5f + 0.25f * ((float)j - 0.5f * (float)(K - 1));
    g[6 * j + 1] = 0.5f;
    g[6 * j + 2] = 1.0f / 12.0f;
    g[6 * j + 3] = 0.0f;
    g[6 * j + 4] = 1.0f / 12.0f;
    g[6 * j + 5] = P.pi_init / (float)K;
  }
  g[6 * K] = 0.0f;
  g[6 * K + 1] = 0.0f;
}

template <int K>
__device__ __forceinline__ void lobes_load(const float *__restrict__ g, int plane, int idx, float out[6 * K + 2]) {
#pragma unroll
  for (int c = 0; c < 6 * K + 2; ++c) out[c] = g[c * plane + idx];
}

template <int K>
__device__ __forceinline__ void lobes_store(float *__restrict__ g, int plane, int idx, const float in[6 * K + 2]) {
#pragma unroll
  for (int c = 0; c < 6 * K + 2; ++c) g[c * plane + idx] = in[c];
}

// Reprojection of one pixel (Sec. 3.1 with K lobes): the tests and the
// source address of the single-lobe pass; every lobe mean keeps its world
// direction across a change of normal.
template <int K>
__device__ __forceinline__ void lobes_reproject(const ParamsK &P, const ViewK &cur, const ViewK &prev,
                                                const float *__restrict__ gprev, bool has_prev, int x, int y,
                                                const PixelIn &pi, float g[6 * K + 2]) {
  const int plane = cur.H * cur.pitch;
  const int idx = y * cur.pitch + x;
  const V3 n = pi.n;
  const bool guided = dot3(n, pi.o) > 0.0f && pi.rough >= P.rough_min;
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
    lobes_load<K>(gprev, pplane, qidx, g);
    if (fabsf(zp - zq) > P.tau_z * zp) keep = false;
    if (dot3(n, nq) < P.tau_n) keep = false;
#pragma unroll
    for (int c = 0; c < 6 * K + 2; ++c)
      if (!isfinite(g[c])) keep = false;
    if (keep && !(n.x == nq.x && n.y == nq.y && n.z == nq.z)) {
      const Frame fq = make_frame(nq);
      const Frame fp = make_frame(n);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const V3 lq = sq2hemi(fminf(fmaxf(g[6 * j], 0.0f), 1.0f), fminf(fmaxf(g[6 * j + 1], 0.0f), 1.0f));
        const V3 lp = to_local(fp, to_world(fq, lq));
        if (lp.z <= 0.0f)
          keep = false;
        else
          hemi2sq(normalized(lp), g[6 * j], g[6 * j + 1]);
      }
    }
  }
  if (!keep) lobes_reset<K>(P, g);
}

// Sampling of one pixel with the K-lobe mixture: the random words and the
// BRDF strategy of the single-lobe pass; a guided draw takes the lobe that
// zeta selects.  Every density is taken at the drawn direction.
template <int K>
__device__ __forceinline__ void lobes_sample(const ParamsK &P, const ViewK &v, const SamplesK &S, int x, int y,
                                             const PixelIn &pi, const float g[6 * K + 2]) {
  const int plane = v.H * v.pitch;
  const int splane = S.spp * plane;
  const bool valid = dot3(pi.n, pi.o) > 0.0f;
  const bool guided = valid && pi.rough >= P.rough_min && g[6 * K + 1] >= 1.0f;
  const Pixel px = make_pixel(P, pi.n, pi.o, pi.rough, 0.0f);
  Gauss G[K];
  float w[K], tot = 0.0f;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    G[j] = gauss_setup(g[6 * j], g[6 * j + 1], g[6 * j + 2], g[6 * j + 3], g[6 * j + 4], P.eps);
    w[j] = guided ? g[6 * j + 5] : 0.0f;
    tot += w[j];
  }
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
      // the lobe zeta selects (-1: the BRDF)
      int lobe = -1;
      float c = 0.0f;
      float gmx = 0.0f, gmy = 0.0f, gl11 = 0.0f, gl21 = 0.0f, gl22 = 0.0f;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float cn = c + w[j];
        if (lobe < 0 && zeta >= c && zeta < cn) {
          lobe = j;
          gmx = G[j].mx;
          gmy = G[j].my;
          gl11 = G[j].l11;
          gl21 = G[j].l21;
          gl22 = G[j].l22;
        }
        c = cn;
      }
      bool ok;
      if (lobe >= 0) {
        const float rho = fsqrt(-1.38629436f * __builtin_amdgcn_logf(1.0f - x1));
        const float z1 = rho * cs, z2 = rho * sn;
        const float ux = fmaf(gl11, z1, gmx);
        const float uy = fmaf(gl22, z2, fmaf(gl21, z1, gmy));
        ok = ux >= 0.0f && ux <= 1.0f && uy >= 0.0f && uy <= 1.0f;
        if (ok) l = sq2hemi(ux, uy);
        code = ok ? 2 : 3;
      } else {
        if (xl < P.s_d) {
          const float r = fsqrt(x1);
          l = V3{r * cs, r * sn, fsqrt(1.0f - x1)};
          ok = l.z > 0.0f;
        } else {
          const float t2 = px.alpha2 * x1 * frcp(1.0f - x1);
          const float ch = __builtin_amdgcn_rsqf(1.0f + t2);
          const float sh = fsqrt(t2) * ch;
          const V3 h = V3{sh * cs, sh * sn, ch};
          const float woh = dot3(px.wo, h);
          l = V3{2.0f * woh * h.x - px.wo.x, 2.0f * woh * h.y - px.wo.y, 2.0f * woh * h.z - px.wo.z};
          ok = l.z > 0.0f && woh > 0.0f;
        }
        code = ok ? 1 : 4;
      }
      if (ok && l.z > 0.0f) {  // a guided draw on the rim has no density
        pb = brdf_pdf_only(px, l);
        D = (1.0f - tot) * pb;
        if (guided) {
          float ux, uy;
          hemi2sq(l, ux, uy);
#pragma unroll
          for (int j = 0; j < K; ++j) D = fmaf(w[j], gauss_pdf_fast(G[j], ux, uy), D);
        }
      }
    }
    V3 wd = V3{0.0f, 0.0f, 0.0f};
    if (code == 1 || code == 2) {
      wd = to_world(px.f, l);
    } else {
      D = 0.0f;
      pb = 0.0f;
    }
    S.dir[rec] = wd.x;
    S.dir[splane + rec] = wd.y;
    S.dir[2 * splane + rec] = wd.z;
    S.pmix[rec] = D;
    S.pb[rec] = pb;
    S.strat[rec] = code;
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_lobes_reproject_sample(ParamsK P, ViewK cur, ViewK prev,
                                                                const float *__restrict__ gprev,
                                                                float *__restrict__ gout, SamplesK S, int has_prev) {
  int x, y;
  stream_xy(cur.W, cur.H, x, y);
  if (x >= cur.W || y >= cur.H) return;
  const int idx = y * cur.pitch + x;
  const PixelIn pi = load_pixel(cur, idx);
  float g[6 * K + 2];
  lobes_reproject<K>(P, cur, prev, gprev, has_prev != 0, x, y, pi, g);
  lobes_sample<K>(P, cur, S, x, y, pi, g);
  lobes_store<K>(gout, cur.H * cur.pitch, idx, g);
}

template <int K>
__global__ __launch_bounds__(256) void k_lobes_pdf(ParamsK P, ViewK v, const float *__restrict__ gamma, int n_per_px,
                                                   const float *__restrict__ dir, float *__restrict__ pmix) {
  int x, y;
  stream_xy(v.W, v.H, x, y);
  if (x >= v.W || y >= v.H) return;
  const int plane = v.H * v.pitch;
  const int idx = y * v.pitch + x;
  const int dplane = n_per_px * plane;
  float g[6 * K + 2];
  lobes_load<K>(gamma, plane, idx, g);
  const PixelIn pi = load_pixel(v, idx);
  const bool valid = dot3(pi.n, pi.o) > 0.0f;
  const bool guided = valid && pi.rough >= P.rough_min && g[6 * K + 1] >= 1.0f;
  const Pixel px = make_pixel(P, pi.n, pi.o, pi.rough, 0.0f);
  float tot = 0.0f;
#pragma unroll
  for (int j = 0; j < K; ++j) tot += guided ? g[6 * j + 5] : 0.0f;
  for (int s = 0; s < n_per_px; ++s) {
    const int r = (s * v.H + y) * v.pitch + x;
    const V3 w = V3{dir[r], dir[dplane + r], dir[2 * dplane + r]};
    float D = 0.0f;
    if (valid && dot3(w, w) > 0.0f) {
      const V3 l = to_local(px.f, normalized(w));
      if (l.z > 0.0f) {
        D = (1.0f - tot) * brdf_pdf_only(px, l);
        if (guided) {
          float ux, uy;
          hemi2sq(l, ux, uy);
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const Gauss G = gauss_setup(g[6 * j], g[6 * j + 1], g[6 * j + 2], g[6 * j + 3], g[6 * j + 4], P.eps);
            D = fmaf(g[6 * j + 5], gauss_pdf_acc(G, ux, uy), D);
          }
        }
      }
    }
    pmix[r] = D;
  }
}

// E-step of one training record for K lobes: posterior gam_j = pi_j p_gj / D
// under the model's weights, and the per-lobe running sums of em_visit.
template <int K>
struct LobesCtx {
  Pixel px;
  LobeTerm T[K];  // each lobe's Gaussian term in the centred square
  float one_m_tot;
  V3 xp;  // positional reuse: the pixel's position relative to the tile's reference point
};

// With VPL, a record with r.w > 0 holds its virtual point light y (relative
// to the tile's reference point) and trains along y - x_p; r.w < 0 marks a
// sample without an interaction, trained along its own direction with weight
// -r.w.
template <int K, bool VPL = false>
__device__ __forceinline__ void lobes_visit(const LobesCtx<K> &c, float4 r, float &B0, Accum a[K]) {
  if (r.w == 0.0f) return;
  V3 wd = V3{r.x, r.y, r.z};
  if (VPL) {
    if (r.w > 0.0f) {
      wd = V3{r.x - c.xp.x, r.y - c.xp.y, r.z - c.xp.z};
      if (!(dot3(wd, wd) > 0.0f)) return;
      wd = normalized(wd);
    } else {
      r.w = -r.w;
    }
  }
  const V3 l = to_local(c.px.f, wd);
  if (l.z <= 0.0f) return;
  float ox, oy, f, pb;
  hemi2sq_c(l, ox, oy);
  brdf_eval(c.px, l, f, pb);
  const float w = r.w * f * l.z;
  float ga[K], rx[K], ry[K], D = c.one_m_tot * pb;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    rx[j] = fmaf(0.5f, ox, c.T[j].hx);  // relative to lobe j's mean (see Accum)
    ry[j] = fmaf(0.5f, oy, c.T[j].hy);
    ga[j] = lobe_eval(c.T[j], rx[j], ry[j]);
    D += ga[j];
  }
  const float rD = __builtin_amdgcn_rcpf(fmaxf(D, 1.17549435e-38f));
  B0 += w;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float vw = w * (ga[j] * rD);
    if (vw >= 1.17549435e-38f) {
      const float bn = a[j].B1 + vw;
      const float rb = __builtin_amdgcn_rcpf(bn);
      const float fr = vw * rb, keep = a[j].B1 * rb;
      a[j].B1 = bn;
      const float dx = rx[j] - a[j].mx, dy = ry[j] - a[j].my;
      a[j].mx = fmaf(dx, fr, a[j].mx);
      a[j].my = fmaf(dy, fr, a[j].my);
      const float fx = fr * dx, fy = fr * dy;
      a[j].sxx = keep * fmaf(fx, dx, a[j].sxx);
      a[j].sxy = keep * fmaf(fx, dy, a[j].sxy);
      a[j].syy = keep * fmaf(fy, dy, a[j].syy);
    }
  }
}

// Staging of a tile's records for positional reuse: like stage_records, but
// a BRDF record with a finite hit distance t holds its virtual point light
// y = x_q + t w relative to the tile's reference point c (positions of the
// image are large; differences of nearby ones are small and exact), and one
// without an interaction holds its direction with the weight negated.
template <int TW, int TH>
__device__ __forceinline__ void stage_records_vpl(const ViewK &v, const SamplesK &S, const float *__restrict__ pos,
                                                  const float *__restrict__ hit, V3 cref, float4 *lds, int tx0,
                                                  int ty0) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH;
  constexpr int IT = (SA + NT - 1) / NT;
  const int plane = v.H * v.pitch;
  const int splane = S.spp * plane;
  int gi[IT];
  bool in[IT];
  V3 xq[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = threadIdx.x + i * NT;
    const int sy = (int)(((float)e + 0.5f) * (1.0f / SW));
    const int sx = e - sy * SW;
    const int gx = tx0 - kR + sx, gy = ty0 - kR + sy;
    in[i] = e < SA && gx >= 0 && gy >= 0 && gx < v.W && gy < v.H;
    gi[i] = gy * v.pitch + gx;
    xq[i] = V3{0.0f, 0.0f, 0.0f};
    if (in[i]) xq[i] = V3{pos[gi[i]] - cref.x, pos[plane + gi[i]] - cref.y, pos[2 * plane + gi[i]] - cref.z};
  }
  for (int s = 0; s < S.spp; ++s) {
    uint8_t st[IT];
    float px[IT], py[IT], pz[IT], pl[IT], pp[IT], th[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      st[i] = 0;
      px[i] = py[i] = pz[i] = pl[i] = pp[i] = th[i] = 0.0f;
      if (in[i]) {
        const int o = s * plane + gi[i];
        st[i] = at(S.strat, o);
        pp[i] = at(S.pb, o);
        px[i] = at(S.dir, o);
        py[i] = at(S.dir + splane, o);
        pz[i] = at(S.dir + 2 * splane, o);
        pl[i] = at(S.L, o);
        th[i] = at(hit, o);
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = threadIdx.x + i * NT;
      if (IT * NT == SA || e < SA) {
        const bool ok = st[i] == 1 && pp[i] > 0.0f;
        const float w = pl[i] * frcp(fmaxf(pp[i], 1.17549435e-38f));
        float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (ok) {
          if (isfinite(th[i])) {
            const V3 d = normalized(V3{px[i], py[i], pz[i]});
            r = make_float4(fmaf(th[i], d.x, xq[i].x), fmaf(th[i], d.y, xq[i].y), fmaf(th[i], d.z, xq[i].z), w);
          } else {
            r = make_float4(px[i], py[i], pz[i], -w);
          }
        }
        lds[s * SA + e] = r;
      }
    }
  }
}

// E-step of one pixel over its training list (LDS byte offsets list[j * stride])
// and the stepwise merge of every lobe, in place on g.  A list whose samples
// carry no weight leaves g as it is.
template <int K, bool VPL = false>
__device__ __forceinline__ void lobes_update(const ParamsK &P, const ViewK &v, int idx, const float4 *lds,
                                             const uint16_t *list, int stride, int len, float g[6 * K + 2],
                                             V3 xp = V3{0.0f, 0.0f, 0.0f}) {
  const int plane = v.H * v.pitch;
  LobesCtx<K> c;
  c.xp = xp;
  c.px = make_pixel(P, load3(v.n, plane, idx), load3(v.o, plane, idx), at(v.rough, idx), at(v.alb, idx));
  float tot = 0.0f;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    c.T[j] = lobe_term(gauss_setup(g[6 * j], g[6 * j + 1], g[6 * j + 2], g[6 * j + 3], g[6 * j + 4], P.eps),
                       g[6 * j + 5]);
    tot += g[6 * j + 5];
  }
  c.one_m_tot = 1.0f - tot;
  float B0 = 0.0f;
  Accum a[K];
#pragma unroll
  for (int j = 0; j < K; ++j) a[j] = Accum{0, 0, 0, 0, 0, 0, 0};
  // records read ahead of the visits only where that costs no wave: at 4
  // lobes (4 waves per SIMD either way; EM -1%); at 2 and 3 lobes the six
  // registers it takes drop a wave (2 lobes: +3%)
  if constexpr (K >= 4)
    for_each_record<2>(lds, list, stride, 0, 0, 1, len, [&](float4 r) { lobes_visit<K, VPL>(c, r, B0, a); });
  else
    for (int j = 0; j < len; ++j) lobes_visit<K, VPL>(c, list_record(lds, list[j * stride]), B0, a);
  if (!(B0 > 0.0f)) return;
#pragma unroll
  for (int j = 0; j < K; ++j) accum_to_unit(a[j], c.T[j]);  // mean and scatter back to u
  const float Wv = g[6 * K], kk = g[6 * K + 1];
  const float eta = frcp(kk + 1.0f);
  const float sw = fmaf(1.0f - eta, Wv, eta * B0);
  const float isw = 1.0f / sw;
  float pn[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    float *l = g + 6 * j;
    const float so = (1.0f - eta) * l[5] * Wv;
    const float sn = eta * a[j].B1;
    const float sg = so + sn;
    if (sg > 0.0f && a[j].B1 > 0.0f) {
      const float al = so / sg, be = sn / sg;
      const float dx = l[0] - a[j].mx, dy = l[1] - a[j].my;
      const float ab = al * be;
      l[0] = fmaf(al, l[0], be * a[j].mx);
      l[1] = fmaf(al, l[1], be * a[j].my);
      l[2] = fmaf(ab * dx, dx, fmaf(al, l[2], be * a[j].sxx));
      l[3] = fmaf(ab * dx, dy, fmaf(al, l[3], be * a[j].sxy));
      l[4] = fmaf(ab * dy, dy, fmaf(al, l[4], be * a[j].syy));
    }
    pn[j] = sg * isw;
  }
  if (!(P.flags & kNoClamp)) {
    const float fl = P.pi_lo * (0.25f / (float)K);
    float tt = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      pn[j] = fmaxf(pn[j], fl);
      tt += pn[j];
    }
    const float scale = tt > 0.0f ? fminf(fmaxf(tt, P.pi_lo), P.pi_hi) / tt : 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) pn[j] *= scale;
  }
#pragma unroll
  for (int j = 0; j < K; ++j) g[6 * j + 5] = pn[j];
  g[6 * K] = sw;
  g[6 * K + 1] = fminf(kk + 1.0f, (float)P.k_max);
}

// Training pass with K lobes (Sec. 3.2, Sec. 4.2), on the tile machinery of
// the single-lobe pass: the records of a TW x TH tile and its halo staged in
// LDS, the pixels sorted by candidate count to build their training lists
// (own samples, then the N(k) picks of stream 1, rejected candidates
// compacted away), sorted again by list length so that the lanes of a wave
// carry nearly equal work, then the E-step of each lane's pixel over its list
// and the stepwise merge of every lobe.
// Dynamic LDS: records [spp][SH][SW] float4, then lists [spp + 20][NT]
// uint16; the write-back reuses it ([6K + 2][NT] float).
// With VPL, positions [3][H*pitch] and hit distances [spp][H*pitch] give the
// positional reuse of virtual point lights (the training directions of every
// pixel are re-derived from the staged y).
// Two lobes (directional) fit 72 VGPRs without spilling, 7 waves per SIMD
// instead of the 6 that the compiler's own choice (75) leaves: EM -4%; at
// 8 waves, or with VPL at 7, it spills.
template <int K, int TW, int TH, bool VPL = false>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(K == 2 && !VPL ? 7 : 1))) void k_lobes_em(ParamsK P, ViewK v, SamplesK S, float *__restrict__ gamma,
                                                     int tiles_x, int n_tiles, const float *__restrict__ pos,
                                                     const float *__restrict__ hit) {
  constexpr int SW = TW + 2 * kR, SH = TH + 2 * kR, SA = SW * SH, NT = TW * TH;
  extern __shared__ float4 lds[];
  __shared__ EmShared<NT> sh;
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  const int tx0 = (tile % tiles_x) * TW, ty0 = (tile / tiles_x) * TH;
  const int t = threadIdx.x;
  const int spp = S.spp;
  const int plane = v.H * v.pitch;
  uint16_t *list = reinterpret_cast<uint16_t *>(lds + spp * SA);
  if (t < 2 * kMaxLen) (&sh.cnt[0][0])[t] = 0;
  int16_t *ptab = reinterpret_cast<int16_t *>(list + (spp + 20) * NT);
  build_pick_table<SA, SW>(ptab, spp);
  // the candidate count of this lane's pixel (0 when it is not trained)
  int ncand = 0;
  {
    const int x0 = tx0 + t % TW, y0 = ty0 + t / TW;
    if (x0 < v.W && y0 < v.H) {
      const int idx0 = y0 * v.pitch + x0;
      const PixelIn pin = load_pixel(v, idx0);
      if (dot3(pin.n, pin.o) > 0.0f && pin.rough >= P.rough_min)
        ncand = spp + n_picks(P, (int)gamma[(6 * K + 1) * plane + idx0]);
    }
  }
  V3 cref = V3{0.0f, 0.0f, 0.0f};
  if (VPL) {
    const int ci = min(ty0, v.H - 1) * v.pitch + min(tx0, v.W - 1);
    cref = load3(pos, plane, ci);
    stage_records_vpl<TW, TH>(v, S, pos, hit, cref, lds, tx0, ty0);
  } else {
    stage_records<TW, TH>(v, S, lds, tx0, ty0, 0);
  }
  sh.work[t] = (uint8_t)ncand;
  __syncthreads();
  int me;
  {
    const int pa = balance<NT>(ncand, t, sh.cnt[0], sh.perm, (int)blockIdx.x);
    const int nc = sh.work[pa];
    int len = 0;
    if (nc > 0) {
      const int lx = pa % TW, ly = pa / TW;
      len = build_list<TW, TH>(P, lds, ptab, list, pa, lx, ly, nc - spp, spp,
                               (uint32_t)((ty0 + ly) * v.W + tx0 + lx));
    }
    sh.work[pa] = (uint8_t)len;
    me = balance<NT>(len, pa, sh.cnt[1], sh.perm, (int)blockIdx.x + 1);
  }
  const int len = sh.work[me];
  float g[6 * K + 2];
  if (len > 0) {  // otherwise no training sample (or no pixel): the model stays as it is
    const int idx = (ty0 + me / TW) * v.pitch + tx0 + me % TW;
    lobes_load<K>(gamma, plane, idx, g);
    V3 xp = V3{0.0f, 0.0f, 0.0f};
    if (VPL) xp = V3{pos[idx] - cref.x, pos[plane + idx] - cref.y, pos[2 * plane + idx] - cref.z};
    lobes_update<K, VPL>(P, v, idx, lds, list + me, NT, len, g, xp);
  }
  // write-back in natural order through LDS (full cache lines), over the
  // records and lists once no lane reads them
  float *wb = reinterpret_cast<float *>(lds);
  __syncthreads();
  if (len > 0) {
#pragma unroll
    for (int c = 0; c < 6 * K + 2; ++c) wb[c * NT + me] = g[c];
  }
  __syncthreads();
  const int x0 = tx0 + t % TW, y0 = ty0 + t / TW;
  if (sh.work[t] > 0 && x0 < v.W && y0 < v.H) {
    const int idx0 = y0 * v.pitch + x0;
#pragma unroll
    for (int c = 0; c < 6 * K + 2; ++c) gamma[c * plane + idx0] = wb[c * NT + t];
  }
}

// ---------------------------------------------------------------------------
// Near-field stand-in for the trace: an emitting plane z = z_c whose emission
// is a lattice of Gaussian lamps (sx, sy, r, c) summed over the 3x3 cells
// around the hit point; writes the radiance and the hit distance of every
// live sample (+inf and the ambient term for a ray that does not rise).
struct CeilingK {
  float z, period, x0, y0, ambient;
  int nx, ny;
  const float *lamps;
};

__device__ __forceinline__ float ceiling_emission(const CeilingK &C, float yx, float yy) {
  const float fx = (yx - C.x0) / C.period, fy = (yy - C.y0) / C.period;
  float E = C.ambient;
  if (!(fx >= -1.0f && fx < (float)C.nx + 1.0f && fy >= -1.0f && fy < (float)C.ny + 1.0f)) return E;
  const int ci = (int)floorf(fx), cj = (int)floorf(fy);
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      const int i = ci + di, j = cj + dj;
      if (i < 0 || j < 0 || i >= C.nx || j >= C.ny) continue;
      const float4 l = reinterpret_cast<const float4 *>(C.lamps)[j * C.nx + i];
      const float dx = yx - l.x, dy = yy - l.y;
      E = fmaf(l.w, expf(-(dx * dx + dy * dy) / (2.0f * l.z * l.z)), E);
    }
  return E;
}

__global__ __launch_bounds__(256) void k_light_ceiling(CeilingK C, ViewK v, const float *__restrict__ pos,
                                                       SamplesK S, float *__restrict__ hit) {
  int x, y;
  stream_xy(v.W, v.H, x, y);
  if (x >= v.W || y >= v.H) return;
  const int plane = v.H * v.pitch;
  const int idx = y * v.pitch + x;
  const int splane = S.spp * plane;
  const V3 xp = load3(pos, plane, idx);
  for (int s = 0; s < S.spp; ++s) {
    const int r = (s * v.H + y) * v.pitch + x;
    const uint8_t code = S.strat[r];
    float L = 0.0f, t = 0.0f;
    if (code == 1 || code == 2) {
      const V3 w = normalized(V3{S.dir[r], S.dir[splane + r], S.dir[2 * splane + r]});
      if (w.z > 0.0f) {
        t = (C.z - xp.z) / w.z;
        L = ceiling_emission(C, fmaf(t, w.x, xp.x), fmaf(t, w.y, xp.y));
      } else {
        t = __builtin_inff();
        L = C.ambient;
      }
    }
    S.L[r] = L;
    hit[r] = t;
  }
}

}  // namespace pgk
