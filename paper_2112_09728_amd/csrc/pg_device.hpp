// Device math for the path-guiding kernels (gfx950, FP32 arithmetic).
//
// Everything a kernel needs per pixel or per sample: the counter-based RNG,
// the shading frame, the Shirley-Chiu map M and its inverse, the synthetic
// Lambert + GGX material, the Gaussian on the unit square and the storage
// conversions of the model planes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgk {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float k4OverPi = 1.27323954473516268615f;
constexpr float kInv4Pi2 = 0.0253302959105844428f;  // 1 / (4 pi^2)
constexpr int kMaxSpp = 8;

struct V3 {
  float x, y, z;
};

__device__ __forceinline__ float dot3(V3 a, V3 b) { return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)); }

// Hardware square root and reciprocal (at most 1 ulp, normal inputs).  The
// default HIP sqrtf and '/' are correctly rounded and several times longer;
// the per-sample paths use these instead wherever the argument is known to
// be a normal number.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// x / d and y / d for d > 0 (and x, y at most a few times d) with one hardware
// reciprocal, about 1.5 ulp each instead of a correctly rounded division's
// ten instructions: d, and x and y with it, which leaves the quotients as
// they are, is scaled by a power of two when it lies outside [2^-62, 2^62],
// since the reciprocal flushes subnormal inputs and outputs.
__device__ __forceinline__ void div2_pos(float x, float y, float d, float &qx, float &qy) {
  const float s = d < 0x1p-62f ? 0x1p64f : (d > 0x1p62f ? 0x1p-64f : 1.0f);
  const float r = __builtin_amdgcn_rcpf(d * s);
  qx = (x * s) * r;
  qy = (y * s) * r;
}
__device__ __forceinline__ float div_pos(float x, float d) {
  float q, unused;
  div2_pos(x, 0.0f, d, q, unused);
  return q;
}
// Row offset y * pitch of a pixel: both below 2^24 (the library bounds the
// sides and the pitch), so the full-rate 24-bit multiply gives it.
__device__ __forceinline__ int row_off(int y, int pitch) { return (int)__umul24((uint32_t)y, (uint32_t)pitch); }
// Element i of an array whose base is uniform across the wave, with i taken
// as an unsigned 32-bit offset: the access then uses the scalar-base plus
// vector-offset form instead of 64-bit address arithmetic in every lane.
template <typename T>
__device__ __forceinline__ T &at(T *p, int i) {
  return p[(uint32_t)i];
}
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011): ten rounds, two 32x32 -> 64-bit
// multiplications per round, key bumped by the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32 -> 64-bit multiply (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input XOR in one instruction (v_bitop3_b32, truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
  }
  return make_uint4(c0, c1, c2, c3);
}

// 24-bit uniform in [0, 1), exact in FP32.
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// Shading frame: Duff et al., "Building an Orthonormal Basis, Revisited"
// (JCGT 2017), around the normalised shading normal.
struct Frame {
  V3 t, b, n;
};

__device__ __forceinline__ Frame make_frame(V3 n) {
  const float inv = __builtin_amdgcn_rsqf(dot3(n, n));
  n = V3{n.x * inv, n.y * inv, n.z * inv};
  const float sign = copysignf(1.0f, n.z);
  const float a = -frcp(sign + n.z);  // sign + n.z lies in [1, 2]
  const float c = n.x * n.y * a;
  Frame f;
  f.t = V3{1.0f + sign * n.x * n.x * a, sign * c, -sign * n.x};
  f.b = V3{c, sign + n.y * n.y * a, -n.y};
  f.n = n;
  return f;
}
__device__ __forceinline__ V3 to_local(const Frame &f, V3 w) { return V3{dot3(w, f.t), dot3(w, f.b), dot3(w, f.n)}; }
__device__ __forceinline__ V3 to_world(const Frame &f, V3 l) {
  return V3{fmaf(l.z, f.n.x, fmaf(l.y, f.b.x, l.x * f.t.x)),
            fmaf(l.z, f.n.y, fmaf(l.y, f.b.y, l.x * f.t.y)),
            fmaf(l.z, f.n.z, fmaf(l.y, f.b.z, l.x * f.t.z))};
}
__device__ __forceinline__ V3 normalized(V3 v) {
  const float inv = __builtin_amdgcn_rsqf(dot3(v, v));
  return V3{v.x * inv, v.y * inv, v.z * inv};
}

// sin(pi t) and cos(pi t) for |t| <= 2: t = r + j/2 with |r| <= 1/4, Taylor
// series of sin and cos at pi r (|pi r| <= pi/4: truncation below 2e-9, about
// 1 ulp in FP32), then the quarter turn j.
__device__ __forceinline__ void sincospi_small(float t, float *s, float *c) {
  const float j = rintf(2.0f * t);
  const float r = fmaf(-0.5f, j, t);
  const float r2 = r * r;
  // sin(pi r) = r (pi - pi^3 r^2/3! + pi^5 r^4/5! - pi^7 r^6/7! + pi^9 r^8/9!)
  float ps = 8.21458866e-02f;
  ps = fmaf(ps, r2, -5.99264529e-01f);
  ps = fmaf(ps, r2, 2.55016404e+00f);
  ps = fmaf(ps, r2, -5.16771278e+00f);
  ps = fmaf(ps, r2, 3.14159265e+00f);
  const float sr = r * ps;
  // cos(pi r) = 1 - pi^2 r^2/2! + pi^4 r^4/4! - pi^6 r^6/6! + pi^8 r^8/8! - pi^10 r^10/10!
  float pc = -2.58068914e-02f;
  pc = fmaf(pc, r2, 2.35330630e-01f);
  pc = fmaf(pc, r2, -1.33526277e+00f);
  pc = fmaf(pc, r2, 4.05871213e+00f);
  pc = fmaf(pc, r2, -4.93480220e+00f);
  const float cr = fmaf(pc, r2, 1.0f);
  const int q = ((int)j) & 3;
  const float ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// ---------------------------------------------------------------------------
// M: unit square -> upper hemisphere.  Concentric square-to-disk map of
// Shirley and Chiu (JGT 1997) followed by the equal-area lift
// (x, y) -> (x sqrt(2 - r^2), y sqrt(2 - r^2), 1 - r^2).  The sector angle is
// kept in units of pi so that sincospi needs no multiplication by pi.
__device__ __forceinline__ V3 sq2hemi(float ux, float uy) {
  const float a = 2.0f * ux - 1.0f, b = 2.0f * uy - 1.0f;
  float r, q;
  // a nonzero a or b is at least 2^-23 in magnitude, so the reciprocals
  // below are of normal numbers
  if (fabsf(a) > fabsf(b)) {
    r = a;
    q = 0.25f * b * frcp(a);
  } else if (b != 0.0f) {
    r = b;
    q = 0.5f - 0.25f * a * frcp(b);
  } else {
    return V3{0.0f, 0.0f, 1.0f};
  }
  float s, c;
  sincospi_small(q, &s, &c);
  const float r2 = r * r;
  const float k = r * fsqrt(2.0f - r2);
  return V3{k * c, k * s, 1.0f - r2};
}

// (4/pi) atan(t) on [-1, 1]: odd polynomial t * P(t^2) of degree 17, the
// coefficients of a fit of atan made for this library (max error 5.8e-9 in
// exact arithmetic) multiplied by 4/pi and rounded to FP32 (max error
// 4.3e-8 of the scaled function, below half an ulp of its values near 1).
__device__ __forceinline__ float atan_4pi_unit(float t) {
  const float s = t * t;
  float p = 3.127998672e-03f;
  p = fmaf(p, s, -1.833637990e-02f);
  p = fmaf(p, s, 5.065103248e-02f);
  p = fmaf(p, s, -9.211707115e-02f);
  p = fmaf(p, s, 1.336767375e-01f);
  p = fmaf(p, s, -1.803063750e-01f);
  p = fmaf(p, s, 2.544684708e-01f);
  p = fmaf(p, s, -4.244038165e-01f);
  p = fmaf(p, s, 1.273239374e+00f);
  return t * p;
}

// M^-1 for a direction in the local frame with w.z >= 0 (|w| = 1 up to
// rounding).  The disk radius is rho = sqrt((w_x^2 + w_y^2)/(1 + w_z)), which
// avoids the cancellation of 1 - w_z; inside each of the four concentric
// sectors the disk angle is atan of the ratio of the smaller to the larger of
// w_x, w_y (the disk scaling cancels in that ratio).  Branch free.
// hemi2sq_c gives the point o = 2u - 1 of the centred square, hemi2sq the
// point u of the unit square.
__device__ __forceinline__ void hemi2sq_c(V3 w, float &ox, float &oy) {
  const float s2 = fmaf(w.x, w.x, w.y * w.y);
  const float rho = s2 > 0.0f ? s2 * __builtin_amdgcn_rsqf(s2 * (1.0f + w.z)) : 0.0f;
  const bool bigx = fabsf(w.x) > fabsf(w.y);
  const float num = bigx ? w.y : w.x;
  const float den = bigx ? w.x : w.y;
  const float t = den != 0.0f ? num * __builtin_amdgcn_rcpf(den) : 0.0f;
  const float r = copysignf(rho, den);
  const float o = r * atan_4pi_unit(t);
  ox = bigx ? r : o;
  oy = bigx ? o : r;
}
__device__ __forceinline__ void hemi2sq(V3 w, float &ux, float &uy) {
  float ox, oy;
  hemi2sq_c(w, ox, oy);
  ux = fmaf(0.5f, ox, 0.5f);
  uy = fmaf(0.5f, oy, 0.5f);
}
// ---------------------------------------------------------------------------
// Synthetic material: Lambert + GGX (Walter et al., EGSR 2007) with Smith G1
// and Schlick F, alpha = roughness^2.  Sampling density
// p_b = s_d wi_z/pi + (1 - s_d) D(h) h_z / (4 wo.h).
struct Pixel {
  Frame f;
  V3 wo;            // local view direction
  float alpha2;     // alpha^2
  float albedo_pi;  // albedo / pi
  float f0_g1, omf0_g1;  // f0 and 1 - f0 times G1(wo) / (2 pi wo_z)
  float s_d, s_d_pi;
  float one_m_sd_q;  // (1 - s_d) / (4 pi)
};

__device__ __forceinline__ float smith_g1(V3 v, float alpha2) {
  return 2.0f * v.z * frcp(v.z + fsqrt(fmaf(alpha2, fmaf(v.x, v.x, v.y * v.y), v.z * v.z)));
}

// f_r and p_b of a local direction wi with wi.z > 0, one reciprocal in all.
// With the unnormalised half vector h = wo + wi, den = h_x^2 + h_y^2 +
// alpha^2 h_z^2 and q = sqrt(alpha^2 (wi_x^2 + wi_y^2) + wi_z^2):
//   D(h/|h|)              = alpha^2 |h|^4 / (pi den^2)
//   p_ggx = D h_z/(4 wo.h) = alpha^2 |h|^4 h_z / (4 pi den^2 (wo.h))
//   G1(wi) / wi_z          = 2 / (wi_z + q)
//   f_spec = F D G1(wi) G1(wo) / (4 wi_z wo_z) = F D (G1(wo)/(2 wo_z)) / (wi_z + q)
// and R = 1 / (den^2 (wo.h) (wi_z + q)) serves both denominators; the 1/pi of
// D rides on the pixel's G1(wo) / (2 pi wo_z), which also carries Schlick's
// f0 and 1 - f0, and, with the 1/4 of p_ggx, on the constant
// (1 - s_d) / (4 pi).
__device__ __forceinline__ void brdf_eval(const Pixel &px, V3 wi, float &f, float &pdf) {
  const V3 h = V3{px.wo.x + wi.x, px.wo.y + wi.y, px.wo.z + wi.z};
  const float hh = dot3(h, h);
  const float den = fmaf(px.alpha2, h.z * h.z, fmaf(h.x, h.x, h.y * h.y));
  const float q = fsqrt(fmaf(px.alpha2, fmaf(wi.x, wi.x, wi.y * wi.y), wi.z * wi.z));
  const float wq = wi.z + q;
  const float woh_u = dot3(px.wo, h);  // |h| (wo . h_hat)
  const float R = __builtin_amdgcn_rcpf(den * den * woh_u * wq);
  const float A = px.alpha2 * hh * hh;  // pi D den^2
  const float pggx4 = A * h.z * wq * R;  // 4 pi p_ggx
  pdf = fmaf(px.s_d_pi, wi.z, px.one_m_sd_q * pggx4);
  const float woh = woh_u * __builtin_amdgcn_rsqf(hh);
  const float m = 1.0f - woh;
  const float m2 = m * m;
  const float Fg = fmaf(px.omf0_g1, m2 * m2 * m, px.f0_g1);  // F G1(wo) / (2 pi wo_z)
  f = fmaf(Fg * A, woh_u * R, px.albedo_pi);
}

__device__ __forceinline__ float brdf_pdf_only(const Pixel &px, V3 wi) {
  const V3 h = V3{px.wo.x + wi.x, px.wo.y + wi.y, px.wo.z + wi.z};
  const float hh = dot3(h, h);
  const float den = fmaf(px.alpha2, h.z * h.z, fmaf(h.x, h.x, h.y * h.y));
  const float R = frcp(den * den * dot3(px.wo, h));
  const float pggx4 = px.alpha2 * hh * hh * h.z * R;  // 4 pi p_ggx
  return fmaf(px.s_d_pi, wi.z, px.one_m_sd_q * pggx4);
}

// ---------------------------------------------------------------------------
// Gaussian N(mu, Sigma + eps I) on the unit square via its lower Cholesky
// factor; the Schur complement is floored at eps against rounding.
struct Gauss {
  float mx, my, l11, l21, l22, i11, i22, norm;  // norm = 1/(4 pi^2 l11 l22)
};

__device__ __forceinline__ Gauss gauss_setup(float mx, float my, float sxx, float sxy, float syy,
                                             float eps) {
  Gauss g;
  g.mx = mx;
  g.my = my;
  // the floors keep every argument a normal number when eps > 0
  const float f = fmaxf(eps, 1.17549435e-38f);
  g.l11 = fsqrt(fmaxf(sxx + eps, f));
  g.i11 = frcp(g.l11);
  g.l21 = sxy * g.i11;
  g.l22 = fsqrt(fmaxf((syy + eps) - g.l21 * g.l21, f));
  g.i22 = frcp(g.l22);
  g.norm = kInv4Pi2 * g.i11 * g.i22;
  return g;
}

// Squared Mahalanobis distance |L^-1 (u - mu)|^2.
__device__ __forceinline__ float gauss_q(const Gauss &g, float ux, float uy) {
  const float z1 = (ux - g.mx) * g.i11;
  const float z2 = (uy - g.my - g.l21 * z1) * g.i22;
  return fmaf(z1, z1, z2 * z2);
}

// The weighted Gaussian term pi N(u) / (2 pi) of a lobe as the E-step
// evaluates it, at a point given relative to the lobe's mean, r = u - mu =
// o/2 + h with h = 1/2 - mu, formed from the centred point o in one rounding
// (h is exact for mu >= 1/4, within half an ulp of 1/2 below; the mean is
// added back as 1/2 - h, exactly the centre the points were measured from):
//   pi_norm exp2(-log2(e)/2 (z1^2 + z2^2)),  z1 = i11 rx,  z2 = i22 ry + c21 z1,
// the whitening L^-1 (u - mu) with c21 = -l21 i22, and pi_norm =
// pi / (4 pi^2 l11 l22).  (Folding sqrt(log2(e)/2) into i11 and i22 saves one
// multiplication but rounds the scale twice and squares it, which the far
// tail of a lobe carries into the weights: kept separate.)
struct LobeTerm {
  float hx, hy, i11, i22, c21, pi_norm;  // h = 1/2 - mu
};
__device__ __forceinline__ LobeTerm lobe_term(const Gauss &g, float pi) {
  LobeTerm t;
  t.hx = 0.5f - g.mx;
  t.hy = 0.5f - g.my;
  t.i11 = g.i11;
  t.i22 = g.i22;
  t.c21 = -g.l21 * g.i22;
  t.pi_norm = pi * g.norm;
  return t;
}
__device__ __forceinline__ float lobe_eval(const LobeTerm &t, float rx, float ry) {
  const float z1 = rx * t.i11;
  const float z2 = fmaf(ry, t.i22, z1 * t.c21);
  return t.pi_norm * __builtin_amdgcn_exp2f(-0.72134752044448170368f * fmaf(z1, z1, z2 * z2));
}
// Solid-angle density N(u)/(2 pi), accurate exponential.
__device__ __forceinline__ float gauss_pdf_acc(const Gauss &g, float ux, float uy) {
  return g.norm * expf(-0.5f * gauss_q(g, ux, uy));
}
// Same with the hardware exp2 (about 1e-6 relative for the arguments met here).
__device__ __forceinline__ float gauss_pdf_fast(const Gauss &g, float ux, float uy) {
  return g.norm * __builtin_amdgcn_exp2f(-0.72134752044448170368f * gauss_q(g, ux, uy));
}

// ---------------------------------------------------------------------------
// Storage of the model planes: FP32, FP16 or BF16, round-to-nearest-even.
struct bf16s {
  uint16_t bits;
};

template <typename T> struct GammaIO;
template <> struct GammaIO<float> {
  static __device__ __forceinline__ float load(const float *p) { return *p; }
  static __device__ __forceinline__ void store(float *p, float v) { *p = v; }
  static constexpr float kMax = 3.40282347e38f;
};
template <> struct GammaIO<_Float16> {
  static __device__ __forceinline__ float load(const _Float16 *p) { return (float)*p; }
  static __device__ __forceinline__ void store(_Float16 *p, float v) { *p = (_Float16)v; }
  static constexpr float kMax = 65504.0f;
};
template <> struct GammaIO<bf16s> {
  static __device__ __forceinline__ float load(const bf16s *p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
  }
  static __device__ __forceinline__ void store(bf16s *p, float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
      p->bits = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
      return;
    }
    u += 0x7FFFu + ((u >> 16) & 1u);
    p->bits = (uint16_t)(u >> 16);
  }
  static constexpr float kMax = 3.38953139e38f;
};

// FP16 and BF16 states hold mu - 1/2 in planes 0 and 1: the lobe means lie in
// [0, 1], mostly near the centre of the square (the normal direction), where
// a value near zero keeps more significant bits than one near 1/2; FP32
// states hold mu itself.
template <typename T> struct MuOffset { static constexpr float v = 0.5f; };
template <> struct MuOffset<float> { static constexpr float v = 0.0f; };

// Channel c of a state as stored (the offset taken off mu, W saturated).
template <typename T>
__device__ __forceinline__ void gamma_put(T *p, int c, float v) {
  if constexpr (MuOffset<T>::v != 0.0f)
    if (c < 2) v -= MuOffset<T>::v;
  if (c == 6) v = fminf(v, GammaIO<T>::kMax);
  GammaIO<T>::store(p, v);
}
template <typename T>
__device__ __forceinline__ float gamma_get(const T *p, int c) {
  // (x + 0 is no identity for x = -0, so FP32 states skip the add)
  if constexpr (MuOffset<T>::v != 0.0f) return GammaIO<T>::load(p) + (c < 2 ? MuOffset<T>::v : 0.0f);
  return GammaIO<T>::load(p);
}

template <typename T>
__device__ __forceinline__ void gamma_load(const T *g, int plane, int idx, float out[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) out[c] = gamma_get(&at(g + c * plane, idx), c);
}
template <typename T>
__device__ __forceinline__ void gamma_store(T *g, int plane, int idx, const float in[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) gamma_put(&at(g + c * plane, idx), c, in[c]);
}

}  // namespace pgk
