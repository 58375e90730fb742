"""Pins of the oracle's material model and of the E-step importance weight.

The BRDF's specular term is checked factor by factor against definitions
that the oracle does not use:
  * Smith's masking G1 = 1/(1 + Lambda), Lambda taken from its integral over
    the GGX slope distribution (Smith 1967; Heitz, "Understanding the
    Masking-Shadowing Function in Microfacet-Based BRDFs", JCGT 2014), not
    from its closed form;
  * Schlick's Fresnel factor through its cosine-weighted hemispherical
    average F0 + (1 - F0)/21, and its dependence on wo.h alone;
  * the Lambert term and the energy bound of the specular lobe.
The weight w = L f_r cos / p_src of every training sample (Sec. 3.2, the
luminance of L_i f_r cos of the Fig. 2 caption over the density the sample
was drawn with) is pinned by its expectation: on a flat scene lit by the
analytic field, the mean weight of a pixel's training set equals the
hemisphere quadrature of L f_r cos over the probability that a BRDF draw is
valid.  A last test plants each of the mistakes these pins are meant to
catch in a copy of the oracle and checks that a pin fails.  CPU only.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest
from scipy import integrate

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _upper_dirs(rng, n, max_theta_deg=85.0):
    ct = rng.uniform(np.cos(np.radians(max_theta_deg)), 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(1.0 - ct * ct)
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1)


def g1_from_slopes(v, alpha):
    """Smith masking of direction v (unit, v_z > 0) for GGX roughness alpha:
    G1 = 1 / (1 + Lambda) with Lambda = (1/mu) int_mu^inf (q - mu) P2(q) dq,
    mu = cot(theta_v), where P2(q) = 1 / (2 alpha (1 + q^2/alpha^2)^(3/2)) is
    the one-dimensional marginal of the GGX slope distribution
    P22 = 1 / (pi alpha^2 (1 + |slope|^2/alpha^2)^2), integrated numerically."""
    out = np.empty(len(v))
    for i, d in enumerate(v):
        s = np.hypot(d[0], d[1])
        if s == 0.0:
            out[i] = 1.0
            continue
        mu = d[2] / s
        # q = alpha t: (q - mu) P2(q) dq = (alpha t - mu) / (2 (1 + t^2)^(3/2)) dt
        val, _ = integrate.quad(lambda t: (alpha * t - mu) / (2.0 * (1.0 + t * t) ** 1.5), mu / alpha, np.inf,
                                epsabs=0.0, epsrel=1e-13, limit=200)
        out[i] = 1.0 / (1.0 + val / mu)
    return out


# ----------------------------------------------------------------- G1 and 4 cos cos
def check_specular_masking(alpha):
    """With albedo 0 and F0 = 1 the BRDF is the specular term alone; divided by
    the GGX-sampling density (s_d = 0, which carries D(h) h_z / (4 wo.h)) the
    normal distribution cancels and
        f / p_ggx * wi_z wo_z h_z / (wo.h) = G1(wi) G1(wo)."""
    rng = np.random.default_rng(int(alpha * 1000) + 3)
    n = 60
    wo = _upper_dirs(rng, n)
    wi = _upper_dirs(rng, n)
    f = O.brdf_f(wo, wi, alpha, 0.0, f0=1.0)
    p = O.brdf_pdf(wo, wi, alpha, s_diffuse=0.0)
    h = _unit(wo + wi)
    r = f / p * wi[:, 2] * wo[:, 2] * h[:, 2] / np.einsum("ij,ij->i", wo, h)
    want = g1_from_slopes(wi, alpha) * g1_from_slopes(wo, alpha)
    np.testing.assert_allclose(r, want, rtol=1e-9)
    # at normal incidence and exit nothing is masked: G1(n)^2 = 1
    nrm = np.array([[0.0, 0.0, 1.0]])
    f0 = O.brdf_f(nrm, nrm, alpha, 0.0, f0=1.0)
    p0 = O.brdf_pdf(nrm, nrm, alpha, s_diffuse=0.0)
    assert abs(f0[0] / p0[0] - 1.0) < 1e-12


@pytest.mark.parametrize("alpha", [0.01, 0.1, 0.4, 0.8, 1.0])
def test_specular_masking_from_slope_integral(alpha):
    check_specular_masking(alpha)


# ------------------------------------------------------------------ Fresnel
def schlick_factor(c):
    """The Fresnel part of the oracle's BRDF at wo.h = c, as the ratio of the
    specular term at F0 = 0 to that at F0 = 1 (both with albedo 0): with
    F = F0 + (1 - F0) S(c) the ratio is S(c).  Geometry: wo and wi mirror
    each other about the normal, so h = n and wo.h = cos(theta_o) = c."""
    s = np.sqrt(1.0 - c * c)
    wo = np.stack([s, 0 * c, c], -1)
    wi = np.stack([-s, 0 * c, c], -1)
    return O.brdf_f(wo, wi, 0.5, 0.0, f0=0.0) / O.brdf_f(wo, wi, 0.5, 0.0, f0=1.0)


def check_schlick_fresnel():
    # cosine-weighted hemispherical average of Schlick's factor:
    # 2 int_0^1 (1 - c)^5 c dc = 2 B(2, 6) = 1/21 (a degree-6 polynomial: exact
    # for a Gauss-Legendre rule of 8 nodes)
    c, wc = _gl(8, 0.0, 1.0)
    avg = 2.0 * (schlick_factor(c) * c * wc).sum()
    assert abs(avg - 1.0 / 21.0) < 1e-13, avg
    # the factor depends on wo.h only: tilted half vectors, same wo.h
    rng = np.random.default_rng(17)
    for _ in range(20):
        hv = _unit(np.array([*rng.normal(size=2) * 0.3, 1.0]))
        cc = rng.uniform(0.3, 0.95)
        # wo at angle acos(cc) from h in a random plane through h; keep only
        # geometries whose wo and mirrored wi stay above the surface
        t = _unit(np.cross(hv, rng.normal(size=3)))
        wo = cc * hv + np.sqrt(1 - cc * cc) * t
        wi = 2 * cc * hv - wo
        if wo[2] <= 0.05 or wi[2] <= 0.05:
            continue
        r = O.brdf_f(wo, wi[None], 0.3, 0.0, f0=0.0)[0] / O.brdf_f(wo, wi[None], 0.3, 0.0, f0=1.0)[0]
        assert abs(r - schlick_factor(np.array([cc]))[0]) < 1e-12
    # F is affine in F0 (Schlick's form): F0 = 0.04 sits 4% of the way to F0 = 1
    wo, wi = _upper_dirs(rng, 30), _upper_dirs(rng, 30)
    f04 = O.brdf_f(wo, wi, 0.3, 0.0, f0=0.04)
    np.testing.assert_allclose(f04, 0.04 * O.brdf_f(wo, wi, 0.3, 0.0, f0=1.0)
                               + 0.96 * O.brdf_f(wo, wi, 0.3, 0.0, f0=0.0), rtol=1e-13)


def test_schlick_fresnel_hemispherical_average():
    check_schlick_fresnel()


def test_lambert_term_and_normal_incidence_fresnel():
    """At wo = wi = n the Fresnel factor is F0 (wo.h = 1): with F0 = 0 only the
    Lambert term albedo/pi remains, and its cosine-weighted integral over the
    hemisphere is the albedo (textbook)."""
    n = np.array([[0.0, 0.0, 1.0]])
    for albedo in (0.2, 0.7):
        assert abs(O.brdf_f(n, n, 0.4, albedo, f0=0.0)[0] - albedo / np.pi) < 1e-15
        f1 = O.brdf_f(n, n, 0.4, 0.0, f0=1.0)[0]
        assert abs(O.brdf_f(n, n, 0.4, 0.0, f0=0.25)[0] - 0.25 * f1) < 1e-14 * f1


@pytest.mark.parametrize("alpha", [0.02, 0.3, 1.0])
def test_specular_lobe_conserves_energy(alpha):
    """White furnace: with F0 = 1 and albedo 0, int f_r cos dw <= 1 (masking
    and the directions reflected below the surface take energy away), tending
    to 1 as alpha -> 0.  Monte Carlo over the GGX sampler (s_d = 0), whose
    density the sampler pins fix; null draws count 0."""
    rng = np.random.default_rng(23)
    n = 200000
    wo = _unit(np.array([0.2, 0.1, 1.0]))
    wi, ok = O.brdf_sample(wo, alpha, rng.uniform(0, 1 - 2**-24, (n, 3)), 0.0)
    f = O.brdf_f(wo, wi[ok], alpha, 0.0, f0=1.0)
    p = O.brdf_pdf(wo, wi[ok], alpha, 0.0)
    est = np.zeros(n)
    est[ok] = f * wi[ok, 2] / p
    m, se = est.mean(), est.std() / np.sqrt(n)
    assert m <= 1.0 + 5 * se, (m, se)
    if alpha <= 0.02:
        assert m > 0.995, m


# -------------------------------------------------------- E-step weight
def _sg_radiance(dirs, lights, ambient):
    L = np.full(dirs.shape[0], ambient)
    for ax, ay, az, lam, c in lights:
        L += c * np.exp(lam * (dirs @ np.array([ax, ay, az]) - 1.0))
    return L


def check_estep_weight(seed=5):
    """Flat scene (normal +z everywhere, one view direction, roughness 0.6,
    albedo 0.6) at frame 0, so every sample is a BRDF draw (pi_eff = 0) and
    every record of the 7x7 windows is drawn from the same density.  The mean
    weight of a pixel's training set, B0 / |J_p| with B0 from the oracle's
    E-step, is then an unbiased estimate of
        int L f_r cos dw / P(valid BRDF draw),
    both integrals by hemisphere quadrature.  Pixels 8 apart have disjoint
    windows, so their estimates are independent."""
    H = W = 160
    vdir = _unit(np.array([0.3, -0.2, 1.0]))
    scene = dict(normal=np.broadcast_to(np.array([0, 0, 1.0])[:, None, None], (3, H, W)),
                 view_dir=np.broadcast_to(vdir[:, None, None], (3, H, W)),
                 depth=np.full((H, W), 1000.0), roughness=np.full((H, W), 0.6),
                 albedo=np.full((H, W), 0.6))
    v = O.OView(scene)
    P = O.params(seed, frame=0)
    spp = 2
    g0 = np.zeros((8, H, W))
    g0[0] = g0[1] = 0.5
    g0[2] = g0[4] = 1.0 / 12.0
    g0[5] = 0.05
    rec = O.sample(P, v, g0, spp)
    lights = np.array([[*_unit([0.4, 0.2, 0.9]), 20.0, 8.0],
                       [*_unit([-0.5, 0.3, 0.6]), 5.0, 3.0],
                       [*_unit([0.1, -0.7, 0.7]), 40.0, 12.0]], np.float32)
    ambient = 0.05
    vis = np.full((H, W), 7, np.uint8)
    rec["radiance"] = O.light(lights, ambient, vis, rec["dir"], rec["strategy"])
    _, stats = O.em(P, v, rec, g0, with_stats=True)
    z = []
    for y in range(8, H - 8, 8):
        for x in range(8, W - 8, 8):
            _, _, keep = O.training_set(P, v, spp, rec["strategy"], x, y, 0)
            if keep.sum():
                z.append(stats[0, y, x] / keep.sum())
    z = np.array(z)
    # quadrature in the local frame (the frame of +z is the identity)
    c, wc = _gl(400, 0.0, 1.0)
    p, wp = _gl(400, 0.0, 2.0 * np.pi)
    C_, P_ = np.meshgrid(c, p, indexing="ij")
    s = np.sqrt(1 - C_ * C_)
    dirs = np.stack([s * np.cos(P_), s * np.sin(P_), C_], -1).reshape(-1, 3)
    wts = np.outer(wc, wp).reshape(-1)
    alpha = 0.6 ** 2
    f = O.brdf_f(vdir, dirs, alpha, 0.6, f0=0.04)
    lf = _sg_radiance(dirs, lights.astype(np.float64), ambient)
    integral = (lf * f * dirs[:, 2] * wts).sum()
    p_valid = (O.brdf_pdf(vdir, dirs, alpha, 0.5) * wts).sum()
    want = integral / p_valid
    se = z.std() / np.sqrt(len(z))
    assert len(z) >= 300
    assert abs(z.mean() - want) < 5 * se, (z.mean(), want, se)
    assert se < 0.05 * want  # the check is sharp enough to see a missing cos or density


def test_estep_weight_expectation():
    check_estep_weight()


# ------------------------------------------------------------ planted mistakes
MUTATIONS = [
    # (name, original text in oracle.c, mutated text, pin that must fail)
    ("G1 with alpha instead of alpha^2", "alpha * alpha * (v[0] * v[0] + v[1] * v[1])",
     "alpha * (v[0] * v[0] + v[1] * v[1])", "check_specular_masking(0.4)"),
    ("Schlick exponent 4", "pow(1.0 - woh, 5.0)", "pow(1.0 - woh, 4.0)", "check_schlick_fresnel()"),
    ("specular without 1/(4 wi_z wo_z)", " / (4.0 * wi[2] * wo[2])", "", "check_specular_masking(0.4)"),
    ("weight without 1/p_src", "*w = L * f * l[2] / p_src;", "*w = L * f * l[2];", "check_estep_weight()"),
    ("weight without cos", "*w = L * f * l[2] / p_src;", "*w = L * f / p_src;", "check_estep_weight()"),
]


@pytest.mark.parametrize("name,orig,mut,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistakes(name, orig, mut, pin):
    """Each mistake planted in a copy of the oracle makes its pin fail (and the
    unmodified oracle passes the same pin, above)."""
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(orig) == 1, f"pattern for '{name}' not found exactly once"
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        c_path, so = os.path.join(d, "oracle.c"), os.path.join(d, "libmut.so")
        open(c_path, "w").write(src.replace(orig, mut))
        subprocess.run([gcc, "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-w", "-I", os.path.join(ROOT, "oracle"), c_path, "-o", so, "-lm"], check=True)
        code = (
            "import importlib.util, sys\n"
            f"sys.path.insert(0, {ROOT!r})\n"
            "import oracle\n"
            f"oracle.LIB_PATH = {so!r}\n"
            f"spec = importlib.util.spec_from_file_location('pins', {os.path.abspath(__file__)!r})\n"
            "m = importlib.util.module_from_spec(spec); spec.loader.exec_module(m)\n"
            "try:\n"
            f"    m.{pin}\n"
            "except AssertionError:\n"
            "    print('PIN FAILED'); sys.exit(0)\n"
            "print('PIN PASSED'); sys.exit(0)\n")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "PIN FAILED" in r.stdout, f"the pin did not catch '{name}': {r.stdout}"
