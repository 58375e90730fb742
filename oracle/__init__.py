"""FP64 CPU oracle of the path-guiding hot path (arXiv 2112.09728).

TEST INFRASTRUCTURE ONLY: the parity tests, the smoke check and the CPU
baseline of the benchmark load this module; the product path never does.
The arithmetic lives in ``oracle.c``; this file only marshals numpy arrays into
the C calls.  It imports nothing from the GPU package.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PG_ORACLE_LIB names another build of the same source (the sanitizer build
# of the CPU test suite uses it)
LIB_PATH = os.environ.get("PG_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

NO_CLAMP = 1
STALE_RESET = 4
STRATEGY_NONE, STRATEGY_BRDF, STRATEGY_GUIDED, STRATEGY_GUIDED_NULL, STRATEGY_BRDF_NULL = range(5)


class View(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_int32),
        ("normal", C.c_void_p), ("view_dir", C.c_void_p), ("depth", C.c_void_p),
        ("roughness", C.c_void_p), ("albedo", C.c_void_p), ("motion", C.c_void_p),
        ("disocc", C.c_void_p),
    ]


class Params(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64), ("frame", C.c_uint32), ("view", C.c_uint32),
        ("k_max", C.c_int32), ("radius", C.c_int32),
        ("pi_init", C.c_float), ("pi_lo", C.c_float), ("pi_hi", C.c_float),
        ("eps_sigma", C.c_float), ("tau_depth", C.c_float), ("tau_normal", C.c_float),
        ("rough_min", C.c_float), ("s_diffuse", C.c_float), ("f0", C.c_float),
        ("flags", C.c_uint32), ("stale_tau", C.c_float),
    ]


class Ceiling(C.Structure):
    _fields_ = [("z", C.c_double), ("period", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("ambient", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32), ("lamps", C.c_void_p)]


def ceiling(c):
    """Ceiling struct from the workload's dict (the lamp table is kept alive on the struct)."""
    lamps = _f32(c["lamps"])
    C_ = Ceiling(float(c["z"]), float(c["period"]), float(c["x0"]), float(c["y0"]), float(c["ambient"]),
                 lamps.shape[1], lamps.shape[0], _ptr(lamps))
    C_._keep = lamps
    return C_


class Rect(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32)]


DEFAULTS = dict(k_max=16, radius=3, pi_init=0.05, pi_lo=0.05, pi_hi=0.95, eps_sigma=2.5e-4,
                tau_depth=0.1, tau_normal=0.9, rough_min=0.1, s_diffuse=0.5, f0=0.04, flags=0,
                stale_tau=0.0)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L):
    P = C.c_void_p
    i64, i32 = C.c_int64, C.c_int32
    L.orc_philox4x32_10.argtypes = [P, P, P]
    for name in ("orc_sq2hemi_n", "orc_hemi2sq_n"):
        getattr(L, name).argtypes = [i64, P, P]
    L.orc_onb_n.argtypes = [i64, P, P, P]
    L.orc_brdf_f_n.argtypes = [i64, P, P, P, P, C.c_double, P]
    L.orc_brdf_pdf_n.argtypes = [i64, P, P, P, C.c_double, P]
    L.orc_brdf_sample_n.argtypes = [i64, P, P, C.c_double, P, P, P]
    L.orc_gauss_pdf_sq_n.argtypes = [P, C.c_double, i64, P, P]
    L.orc_gauss_sample_n.argtypes = [P, C.c_double, i64, P, P]
    L.orc_guide_pdf_n.argtypes = [P, C.c_double, i64, P, P]
    L.orc_batch_stats.argtypes = [i64, P, P, P, P]
    L.orc_merge.argtypes = [P, P, P, P]
    L.orc_training_set.argtypes = [P, P, i32, P, i32, i32, i32, P, P, P, i32]
    L.orc_training_set.restype = i32
    L.orc_reproject.argtypes = [P, P, P, P, P, P, Rect]
    L.orc_sample.argtypes = [P, P, P, i32, P, P, P, P, P, Rect]
    L.orc_pdf.argtypes = [P, P, P, i32, P, P, P, P, Rect]
    L.orc_light.argtypes = [i32, P, C.c_double, P, i32, i32, i32, i32, P, P, P, Rect]
    L.orc_em.argtypes = [P, P, i32, P, P, P, P, P, i32, i32, P, Rect]
    L.orc_nll.argtypes = [P, P, i32, P, P, P, P, P, P, P, P, Rect]
    L.orc_estimate.argtypes = [P, P, i32, P, P, P, P, P, Rect]
    L.orc_stale_margin.argtypes = [P, P, i32, P, P, P, P, P, P, Rect]
    L.orc_reference.argtypes = [P, P, i32, P, C.c_double, P, i32, i64, P, P, P]
    L.orc_reproject_k.argtypes = [P, i32, P, P, P, P, P, Rect]
    L.orc_sample_k.argtypes = [P, i32, P, P, i32, P, P, P, P, P, Rect]
    L.orc_pdf_k.argtypes = [P, i32, P, P, i32, P, P, Rect]
    L.orc_em_k.argtypes = [P, i32, P, i32, P, P, P, P, P, P, Rect]
    L.orc_em_vpl.argtypes = [P, i32, P, P, i32, P, P, P, P, P, P, P, Rect]
    L.orc_light_ceiling.argtypes = [P, P, P, i32, P, P, P, P, Rect]
    L.orc_reference_ceiling.argtypes = [P, P, P, P, i32, P, i64, P, P]
    L.orc_num_threads.restype = i32
    L.orc_set_num_threads.argtypes = [i32]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def params(seed, frame=0, view=0, **kw):
    d = dict(DEFAULTS)
    d.update(kw)
    return Params(seed=seed, frame=frame, view=view, **d)


class OView:
    """Host arrays of one view, held alive for the C calls ([c][H][W] float32)."""

    def __init__(self, scene, motion=None, disocc=None):
        self.normal = _f32(scene["normal"])
        self.view_dir = _f32(scene["view_dir"])
        self.depth = _f32(scene["depth"])
        self.roughness = _f32(scene["roughness"])
        self.albedo = _f32(scene["albedo"])
        self.motion = None if motion is None else _f32(motion)
        self.disocc = None if disocc is None else np.ascontiguousarray(disocc, dtype=np.uint8)
        self.height, self.width = self.depth.shape[-2:]
        self.c = View(self.width, self.height, self.width, _ptr(self.normal), _ptr(self.view_dir),
                      _ptr(self.depth), _ptr(self.roughness), _ptr(self.albedo),
                      _ptr(self.motion), _ptr(self.disocc))


def _rect(v, rect):
    if rect is None:
        return Rect(0, 0, v.width, v.height)
    x0, y0, x1, y1 = rect
    return Rect(x0, y0, x1, y1)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sq2hemi(u):
    u = _f64(u).reshape(-1, 2)
    w = np.zeros((u.shape[0], 3))
    lib().orc_sq2hemi_n(u.shape[0], _ptr(u), _ptr(w))
    return w


def hemi2sq(w):
    w = _f64(w).reshape(-1, 3)
    u = np.zeros((w.shape[0], 2))
    lib().orc_hemi2sq_n(w.shape[0], _ptr(w), _ptr(u))
    return u


def onb(n):
    n = _f64(n).reshape(-1, 3)
    t = np.zeros_like(n)
    b = np.zeros_like(n)
    lib().orc_onb_n(n.shape[0], _ptr(n), _ptr(t), _ptr(b))
    return t, b


def brdf_f(wo, wi, alpha, albedo, f0=0.04):
    wo, wi = _f64(wo).reshape(-1, 3), _f64(wi).reshape(-1, 3)
    n = wi.shape[0]
    alpha = _f64(np.broadcast_to(alpha, (n,)))
    albedo = _f64(np.broadcast_to(albedo, (n,)))
    wo = _f64(np.broadcast_to(wo, (n, 3)))
    out = np.zeros(n)
    lib().orc_brdf_f_n(n, _ptr(wo), _ptr(wi), _ptr(alpha), _ptr(albedo), f0, _ptr(out))
    return out


def brdf_pdf(wo, wi, alpha, s_diffuse=0.5):
    wi = _f64(wi).reshape(-1, 3)
    n = wi.shape[0]
    wo = _f64(np.broadcast_to(_f64(wo).reshape(-1, 3), (n, 3)))
    alpha = _f64(np.broadcast_to(alpha, (n,)))
    out = np.zeros(n)
    lib().orc_brdf_pdf_n(n, _ptr(wo), _ptr(wi), _ptr(alpha), s_diffuse, _ptr(out))
    return out


def brdf_sample(wo, alpha, xi, s_diffuse=0.5):
    xi = _f64(xi).reshape(-1, 3)
    n = xi.shape[0]
    wo = _f64(np.broadcast_to(_f64(wo).reshape(-1, 3), (n, 3)))
    alpha = _f64(np.broadcast_to(alpha, (n,)))
    wi = np.zeros((n, 3))
    valid = np.zeros(n, np.int32)
    lib().orc_brdf_sample_n(n, _ptr(wo), _ptr(alpha), s_diffuse, _ptr(xi), _ptr(wi), _ptr(valid))
    return wi, valid.astype(bool)


def gauss_pdf_sq(g5, u, eps=2.5e-4):
    g5, u = _f64(g5), _f64(u).reshape(-1, 2)
    out = np.zeros(u.shape[0])
    lib().orc_gauss_pdf_sq_n(_ptr(g5), eps, u.shape[0], _ptr(u), _ptr(out))
    return out


def gauss_sample(g5, xi, eps=2.5e-4):
    g5, xi = _f64(g5), _f64(xi).reshape(-1, 2)
    u = np.zeros((xi.shape[0], 2))
    lib().orc_gauss_sample_n(_ptr(g5), eps, xi.shape[0], _ptr(xi), _ptr(u))
    return u


def guide_pdf(g5, w, eps=2.5e-4):
    g5, w = _f64(g5), _f64(w).reshape(-1, 3)
    out = np.zeros(w.shape[0])
    lib().orc_guide_pdf_n(_ptr(g5), eps, w.shape[0], _ptr(w), _ptr(out))
    return out


def batch_stats(u, w, gam):
    u, w, gam = _f64(u).reshape(-1, 2), _f64(w), _f64(gam)
    out = np.zeros(7)
    lib().orc_batch_stats(u.shape[0], _ptr(u), _ptr(w), _ptr(gam), _ptr(out))
    return out


def merge(P, g_in, stats):
    g_in, stats = _f64(g_in), _f64(stats)
    out = np.zeros(8)
    lib().orc_merge(C.byref(P), _ptr(g_in), _ptr(stats), _ptr(out))
    return out


def training_set(P, view, spp, strategy, x, y, k, cap=64):
    strategy = np.ascontiguousarray(strategy, dtype=np.uint8)
    q = np.zeros(cap, np.int32)
    s = np.zeros(cap, np.int32)
    keep = np.zeros(cap, np.int32)
    n = lib().orc_training_set(C.byref(P), C.byref(view.c), spp, _ptr(strategy), x, y, k,
                               _ptr(q), _ptr(s), _ptr(keep), cap)
    return q[:n], s[:n], keep[:n].astype(bool)


def reproject(P, cur, prev, gamma_prev, rect=None, out=None):
    H, W = cur.height, cur.width
    g_out = np.zeros((8, H, W)) if out is None else out
    src = np.full((H, W), -2, np.int32)
    gp = None if gamma_prev is None else _f64(gamma_prev)
    lib().orc_reproject(C.byref(P), C.byref(cur.c), None if prev is None else C.byref(prev.c),
                        _ptr(gp), _ptr(g_out), _ptr(src), _rect(cur, rect))
    return g_out, src


def sample(P, view, gamma, spp, rect=None):
    H, W = view.height, view.width
    gamma = _f64(gamma)
    dir_ = np.zeros((3, spp, H, W))
    pmix = np.zeros((spp, H, W))
    pb = np.zeros((spp, H, W))
    strat = np.zeros((spp, H, W), np.uint8)
    margin = np.full((spp, H, W), np.inf)
    lib().orc_sample(C.byref(P), C.byref(view.c), _ptr(gamma), spp, _ptr(dir_), _ptr(pmix),
                     _ptr(pb), _ptr(strat), _ptr(margin), _rect(view, rect))
    return dict(dir=dir_, pdf_mix=pmix, pdf_brdf=pb, strategy=strat, margin=margin)


def pdf(P, view, gamma, dirs, rect=None):
    """dirs: [3][n][H][W] world directions."""
    H, W = view.height, view.width
    dirs = _f64(dirs)
    n = dirs.shape[1]
    gamma = _f64(gamma)
    pmix = np.zeros((n, H, W))
    pg = np.zeros((n, H, W))
    pb = np.zeros((n, H, W))
    lib().orc_pdf(C.byref(P), C.byref(view.c), _ptr(gamma), n, _ptr(dirs), _ptr(pmix), _ptr(pg),
                  _ptr(pb), _rect(view, rect))
    return pmix, pg, pb


def light(lights, ambient, vis, dirs, strategy, rect=None):
    lights = _f32(lights)
    vis = np.ascontiguousarray(vis, dtype=np.uint8)
    dirs = _f64(dirs)
    strategy = np.ascontiguousarray(strategy, dtype=np.uint8)
    spp, H, W = strategy.shape
    L = np.zeros((spp, H, W))
    r = Rect(0, 0, W, H) if rect is None else Rect(*rect)
    lib().orc_light(lights.shape[0], _ptr(lights), ambient, _ptr(vis), W, H, W, spp, _ptr(dirs),
                    _ptr(strategy), _ptr(L), r)
    return L


def em(P, view, rec, gamma, iterations=1, batch=False, rect=None, with_stats=False):
    """Returns the updated state (the input array is not modified), and with
    with_stats the (B0, B1) evidences [2][H][W] of each pixel's last E-step."""
    g = _f64(gamma).copy()
    spp = rec["strategy"].shape[0]
    d, pb = _f64(rec["dir"]), _f64(rec["pdf_brdf"])
    st = np.ascontiguousarray(rec["strategy"], dtype=np.uint8)
    L = _f64(rec["radiance"])
    stats = np.zeros((2,) + g.shape[1:]) if with_stats else None
    lib().orc_em(C.byref(P), C.byref(view.c), spp, _ptr(d), _ptr(pb), _ptr(st), _ptr(L), _ptr(g),
                 iterations, int(bool(batch)), _ptr(stats), _rect(view, rect))
    return (g, stats) if with_stats else g


def stale_margin(P, view, rec, gamma, rect=None):
    """Per-pixel margin of the stale-history decision (negative = reset; NaN
    where it does not apply)."""
    spp = rec["strategy"].shape[0]
    d, pb = _f64(rec["dir"]), _f64(rec["pdf_brdf"])
    st = np.ascontiguousarray(rec["strategy"], dtype=np.uint8)
    L = _f64(rec["radiance"])
    g = _f64(gamma)
    out = np.zeros((view.height, view.width))
    lib().orc_stale_margin(C.byref(P), C.byref(view.c), spp, _ptr(d), _ptr(pb), _ptr(st), _ptr(L), _ptr(g),
                           _ptr(out), _rect(view, rect))
    return out


def estimate(P, view, rec, rect=None):
    """Per-pixel mean of f_r L cos / D over the records' samples [H][W]."""
    spp = rec["strategy"].shape[0]
    d, pm = _f64(rec["dir"]), _f64(rec["pdf_mix"])
    st = np.ascontiguousarray(rec["strategy"], dtype=np.uint8)
    L = _f64(rec["radiance"])
    out = np.zeros((view.height, view.width))
    lib().orc_estimate(C.byref(P), C.byref(view.c), spp, _ptr(d), _ptr(pm), _ptr(st), _ptr(L), _ptr(out),
                       _rect(view, rect))
    return out


def reference(P, view, lights, ambient, vis, pixels, n_samples=16384):
    """Reference int f_r L cos for flat pixel indices `pixels` (y*W + x):
    (mean, standard error) arrays."""
    lights = _f32(lights)
    vis = np.ascontiguousarray(vis, dtype=np.uint8)
    idx = np.ascontiguousarray(pixels, dtype=np.int64)
    mean = np.zeros(idx.shape[0])
    se = np.zeros(idx.shape[0])
    lib().orc_reference(C.byref(P), C.byref(view.c), lights.shape[0], _ptr(lights), float(ambient), _ptr(vis),
                        int(n_samples), idx.shape[0], _ptr(idx), _ptr(mean), _ptr(se))
    return mean, se


def nll(P, view, rec, theta, grad_out=None, rect=None):
    H, W = view.height, view.width
    spp = rec["strategy"].shape[0]
    d, pb = _f64(rec["dir"]), _f64(rec["pdf_brdf"])
    st = np.ascontiguousarray(rec["strategy"], dtype=np.uint8)
    L = _f64(rec["radiance"])
    th = _f64(theta)
    go = None if grad_out is None else _f64(grad_out)
    grad = np.zeros((8, H, W))
    out = np.zeros((H, W))
    lib().orc_nll(C.byref(P), C.byref(view.c), spp, _ptr(d), _ptr(pb), _ptr(st), _ptr(L),
                  _ptr(th), _ptr(go), _ptr(grad), _ptr(out), _rect(view, rect))
    return out, grad


# --- K Gaussian lobes per pixel: state [6K + 2][H][W] ------------------------

def reproject_k(P, K, cur, prev, gamma_prev, rect=None, out=None):
    H, W = cur.height, cur.width
    g_out = np.zeros((6 * K + 2, H, W)) if out is None else out
    src = np.full((H, W), -2, np.int32)
    gp = None if gamma_prev is None else _f64(gamma_prev)
    lib().orc_reproject_k(C.byref(P), K, C.byref(cur.c), None if prev is None else C.byref(prev.c),
                          _ptr(gp), _ptr(g_out), _ptr(src), _rect(cur, rect))
    return g_out, src


def sample_k(P, K, view, gamma, spp, rect=None):
    H, W = view.height, view.width
    gamma = _f64(gamma)
    assert gamma.shape[0] == 6 * K + 2
    dir_ = np.zeros((3, spp, H, W))
    pmix = np.zeros((spp, H, W))
    pb = np.zeros((spp, H, W))
    strat = np.zeros((spp, H, W), np.uint8)
    margin = np.full((spp, H, W), np.inf)
    lib().orc_sample_k(C.byref(P), K, C.byref(view.c), _ptr(gamma), spp, _ptr(dir_), _ptr(pmix),
                       _ptr(pb), _ptr(strat), _ptr(margin), _rect(view, rect))
    return dict(dir=dir_, pdf_mix=pmix, pdf_brdf=pb, strategy=strat, margin=margin)


def pdf_k(P, K, view, gamma, dirs, rect=None):
    H, W = view.height, view.width
    dirs = _f64(dirs)
    gamma = _f64(gamma)
    assert gamma.shape[0] == 6 * K + 2
    n = dirs.shape[1]
    pmix = np.zeros((n, H, W))
    lib().orc_pdf_k(C.byref(P), K, C.byref(view.c), _ptr(gamma), n, _ptr(dirs), _ptr(pmix), _rect(view, rect))
    return pmix


def em_k(P, K, view, rec, gamma, rect=None, with_stats=False):
    """The updated K-lobe state; with with_stats also [K+1][H][W] holding B0
    and each lobe's B1_j."""
    g = _f64(gamma).copy()
    assert g.shape[0] == 6 * K + 2
    spp = rec["strategy"].shape[0]
    d, pb = _f64(rec["dir"]), _f64(rec["pdf_brdf"])
    st = np.ascontiguousarray(rec["strategy"], dtype=np.uint8)
    L = _f64(rec["radiance"])
    stats = np.zeros((K + 1,) + g.shape[1:]) if with_stats else None
    lib().orc_em_k(C.byref(P), K, C.byref(view.c), spp, _ptr(d), _ptr(pb), _ptr(st), _ptr(L), _ptr(g),
                   _ptr(stats), _rect(view, rect))
    return (g, stats) if with_stats else g


# --- positional reuse of virtual point lights and the ceiling workload --------

def em_vpl(P, K, view, position, rec, gamma, rect=None, with_stats=False):
    """The K-lobe update with training directions re-derived from each
    sample's virtual point light (rec["hit_dist"] [spp][H][W])."""
    g = _f64(gamma).copy()
    assert g.shape[0] == 6 * K + 2
    pos = _f32(position)
    spp = rec["strategy"].shape[0]
    d, pb, L, t = _f64(rec["dir"]), _f64(rec["pdf_brdf"]), _f64(rec["radiance"]), _f64(rec["hit_dist"])
    st = np.ascontiguousarray(rec["strategy"], dtype=np.uint8)
    stats = np.zeros((K + 1,) + g.shape[1:]) if with_stats else None
    lib().orc_em_vpl(C.byref(P), K, C.byref(view.c), _ptr(pos), spp, _ptr(d), _ptr(pb), _ptr(st), _ptr(L),
                     _ptr(t), _ptr(g), _ptr(stats), _rect(view, rect))
    return (g, stats) if with_stats else g


def light_ceiling(ceil, view, position, dirs, strategy, rect=None):
    """(radiance, hit distance) [spp][H][W] of the ceiling stand-in."""
    Cc = ceiling(ceil) if isinstance(ceil, dict) else ceil
    pos = _f32(position)
    dirs = _f64(dirs)
    strategy = np.ascontiguousarray(strategy, dtype=np.uint8)
    spp = strategy.shape[0]
    L = np.zeros(strategy.shape)
    t = np.zeros(strategy.shape)
    lib().orc_light_ceiling(C.byref(Cc), C.byref(view.c), _ptr(pos), spp, _ptr(dirs), _ptr(strategy), _ptr(L),
                            _ptr(t), _rect(view, rect))
    return L, t


def reference_ceiling(P, view, position, ceil, pixels, n_samples=16384):
    """Reference int f_r E cos under the ceiling for flat pixel indices:
    (mean, standard error), BRDF sampling with n_samples <= 65536 draws."""
    assert 0 < n_samples <= 65536
    Cc = ceiling(ceil) if isinstance(ceil, dict) else ceil
    pos = _f32(position)
    idx = np.ascontiguousarray(pixels, dtype=np.int64)
    mean = np.zeros(idx.shape[0])
    se = np.zeros(idx.shape[0])
    lib().orc_reference_ceiling(C.byref(P), C.byref(view.c), _ptr(pos), C.byref(Cc), idx.shape[0], _ptr(idx),
                                int(n_samples), _ptr(mean), _ptr(se))
    return mean, se


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


class Frames:
    """Plain frame sequence of the oracle: reproject -> sample -> light -> EM.

    ``step(t, fr)`` takes frame t's scene dict (G-buffer, lights, vis, motion,
    disocc) and returns the per-frame intermediates."""

    def __init__(self, seed, spp, view=0, lobes=1, **kw):
        self.seed = seed
        self.spp = spp
        self.lobes = lobes
        self.view_id = view
        self.kw = kw
        self.view_prev = None
        self.gamma = None
        self.last = None

    def step(self, t, fr, rect=None, gamma_prev=None):
        v = OView(fr, fr.get("motion"), fr.get("disocc"))
        P = params(self.seed, frame=t, view=self.view_id, **self.kw)
        gp = self.gamma if gamma_prev is None else gamma_prev
        prev = self.view_prev if self.view_prev is not None else v
        K = self.lobes
        if K == 1:
            g1, src = reproject(P, v, prev, gp, rect=rect)
            rec = sample(P, v, g1, self.spp, rect=rect)
        else:
            g1, src = reproject_k(P, K, v, prev, gp, rect=rect)
            rec = sample_k(P, K, v, g1, self.spp, rect=rect)
        rec["radiance"] = light(fr["lights"], float(fr["ambient"]), fr["vis"], rec["dir"],
                                rec["strategy"], rect=rect)
        g2 = em(P, v, rec, g1, rect=rect) if K == 1 else em_k(P, K, v, rec, g1, rect=rect)
        self.gamma = g2
        self.view_prev = v
        self.last = dict(gamma_reproj=g1, src=src, rec=rec, gamma=g2)
        return self.last
