"""Python binding of libpmmguide (screen-space path guiding, arXiv 2112.09728).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libpmmguide.so``; torch provides device memory and the current stream.
The library must be built (``python -m paper_2112_09728_amd.build``); without
it every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmmguide.so")

PG_OK, PG_ERR_ARG, PG_ERR_UNSUPPORTED, PG_ERR_HIP = 0, 1, 2, 3
PG_F32, PG_F16, PG_BF16 = 0, 1, 2
PG_NO_CLAMP, PG_EM_BATCH, PG_STALE_RESET = 1, 2, 4
MAX_LIGHTS = 8

STRATEGY_NONE, STRATEGY_BRDF, STRATEGY_GUIDED, STRATEGY_GUIDED_NULL, STRATEGY_BRDF_NULL = range(5)


class PgView(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_int32),
        ("normal", C.c_void_p), ("view_dir", C.c_void_p), ("depth", C.c_void_p),
        ("roughness", C.c_void_p), ("albedo", C.c_void_p), ("motion", C.c_void_p),
        ("disocc", C.c_void_p),
    ]


class PgGamma(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("data", C.c_void_p)]


class PgSamples(C.Structure):
    _fields_ = [
        ("spp", C.c_int32), ("dir", C.c_void_p), ("pdf_mix", C.c_void_p),
        ("pdf_brdf", C.c_void_p), ("strategy", C.c_void_p), ("radiance", C.c_void_p),
    ]


class PgParams(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64), ("frame", C.c_uint32), ("view", C.c_uint32),
        ("k_max", C.c_int32), ("radius", C.c_int32),
        ("pi_init", C.c_float), ("pi_lo", C.c_float), ("pi_hi", C.c_float),
        ("eps_sigma", C.c_float), ("tau_depth", C.c_float), ("tau_normal", C.c_float),
        ("rough_min", C.c_float), ("s_diffuse", C.c_float), ("f0", C.c_float),
        ("flags", C.c_uint32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
        ("stale_tau", C.c_float),
    ]


class PgLights(C.Structure):
    _fields_ = [("count", C.c_int32), ("ambient", C.c_float),
                ("light", (C.c_float * 5) * MAX_LIGHTS)]


class PgCeiling(C.Structure):
    _fields_ = [("z", C.c_float), ("period", C.c_float), ("x0", C.c_float), ("y0", C.c_float),
                ("ambient", C.c_float), ("nx", C.c_int32), ("ny", C.c_int32), ("lamps", C.c_void_p)]


class PgBatchView(C.Structure):
    _fields_ = [("params", PgParams), ("cur", PgView), ("prev", PgView), ("gamma_in", PgGamma),
                ("gamma_out", PgGamma), ("samples", PgSamples), ("vis", C.c_void_p),
                ("lights", PgLights)]


EXPORTS = ("pg_params_default", "pg_reproject", "pg_sample_mis", "pg_reproject_sample", "pg_pdf",
           "pg_light_field", "pg_em_update", "pg_nll_backward", "pg_estimate", "pg_batch_table_bytes",
           "pg_batch_pack", "pg_frame_batched", "pg_frame_batched_noalloc", "pg_reproject_sample_lobes", "pg_em_update_lobes",
           "pg_pdf_lobes", "pg_em_update_vpl", "pg_light_ceiling", "pg_philox", "pg_last_error")
MAX_LOBES = 4

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded libpmmguide (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is missing: build it with `python -m paper_2112_09728_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pg_params_default.argtypes = [P]
        L.pg_reproject.argtypes = [P, P, P, PgGamma, PgGamma, P, P]
        L.pg_sample_mis.argtypes = [P, P, PgGamma, P, P]
        L.pg_reproject_sample.argtypes = [P, P, P, PgGamma, PgGamma, P, P]
        L.pg_pdf.argtypes = [P, P, PgGamma, C.c_int32, P, P, P, P, P]
        L.pg_light_field.argtypes = [P, P, P, P, P]
        L.pg_em_update.argtypes = [P, P, P, PgGamma, C.c_int32, P]
        L.pg_nll_backward.argtypes = [P, P, P, P, P, P, P, P]
        L.pg_estimate.argtypes = [P, P, P, P, P]
        L.pg_batch_table_bytes.argtypes = [C.c_int32]
        L.pg_batch_pack.argtypes = [P, C.c_int32, P, C.c_size_t]
        L.pg_frame_batched.argtypes = [P, P, C.c_size_t, P]
        L.pg_frame_batched_noalloc.argtypes = [P, C.c_size_t, P]
        L.pg_reproject_sample_lobes.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.pg_em_update_lobes.argtypes = [P, C.c_int32, P, P, P, P]
        L.pg_pdf_lobes.argtypes = [P, C.c_int32, P, P, C.c_int32, P, P, P]
        L.pg_em_update_vpl.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.pg_light_ceiling.argtypes = [P, P, P, P, P, P]
        L.pg_philox.argtypes = [C.c_int32, P, C.c_uint64, P, P]
        L.pg_last_error.restype = C.c_char_p
        for name in EXPORTS[:-1]:
            getattr(L, name).restype = C.c_int
        L.pg_batch_table_bytes.restype = C.c_size_t
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != PG_OK:
        msg = lib().pg_last_error().decode()
        raise RuntimeError(f"{what} failed with status {status}: {msg}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def gamma_dtype_code(dtype) -> int:
    import torch
    codes = {torch.float32: PG_F32, torch.float16: PG_F16, torch.bfloat16: PG_BF16}
    if dtype not in codes:
        raise TypeError(f"unsupported Gamma storage dtype {dtype}")
    return codes[dtype]


def _gamma(t) -> PgGamma:
    if t is None:
        return PgGamma(PG_F32, None)
    _require(t, None, "gamma")
    return PgGamma(gamma_dtype_code(t.dtype), t.data_ptr())


def _require(t, dtype, name):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def params(seed: int = 0, frame: int = 0, view: int = 0, **overrides) -> PgParams:
    """pg_params with the library defaults, then the given fields."""
    p = PgParams()
    _check(lib().pg_params_default(C.byref(p)), "pg_params_default")
    p.seed, p.frame, p.view = seed, frame, view
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class View:
    """Device G-buffer of one view ([c][H][W] float32 tensors, contiguous)."""

    def __init__(self, normal, view_dir, depth, roughness, albedo, motion=None, disocc=None):
        import torch
        self.normal, self.view_dir, self.depth = normal, view_dir, depth
        self.roughness, self.albedo, self.motion, self.disocc = roughness, albedo, motion, disocc
        self.height, self.width = depth.shape[-2:]
        for name in ("normal", "view_dir", "depth", "roughness", "albedo", "motion"):
            _require(getattr(self, name), torch.float32, name)
        _require(disocc, torch.uint8, "disocc")
        H, W = self.height, self.width
        for name, shape in (("normal", (3, H, W)), ("view_dir", (3, H, W)), ("depth", (H, W)),
                            ("roughness", (H, W)), ("albedo", (H, W)), ("motion", (2, H, W)),
                            ("disocc", (H, W))):
            t = getattr(self, name)
            if t is not None and tuple(t.shape) != shape:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
        self.c = PgView(W, H, W, normal.data_ptr(), view_dir.data_ptr(), depth.data_ptr(),
                        roughness.data_ptr(), None if albedo is None else albedo.data_ptr(),
                        None if motion is None else motion.data_ptr(),
                        None if disocc is None else disocc.data_ptr())

    def with_motion(self, motion, disocc):
        return View(self.normal, self.view_dir, self.depth, self.roughness, self.albedo, motion,
                    disocc)

    @staticmethod
    def from_scene(scene: dict, device="cuda", motion=None, disocc=None) -> "View":
        import torch

        def dev(a):
            return None if a is None else torch.as_tensor(a).to(device).contiguous()
        return View(dev(scene["normal"]), dev(scene["view_dir"]), dev(scene["depth"]),
                    dev(scene["roughness"]), dev(scene["albedo"]), dev(motion), dev(disocc))


class Samples:
    """Sample records of a view: dir [3][spp][H][W], pdfs and radiance [spp][H][W]."""

    def __init__(self, spp: int, height: int, width: int, device="cuda"):
        import torch
        self.spp, self.height, self.width = spp, height, width
        f = dict(dtype=torch.float32, device=device)
        self.dir = torch.empty((3, spp, height, width), **f)
        self.pdf_mix = torch.empty((spp, height, width), **f)
        self.pdf_brdf = torch.empty((spp, height, width), **f)
        self.radiance = torch.empty((spp, height, width), **f)
        self.strategy = torch.empty((spp, height, width), dtype=torch.uint8, device=device)
        self.c = PgSamples(spp, self.dir.data_ptr(), self.pdf_mix.data_ptr(),
                           self.pdf_brdf.data_ptr(), self.strategy.data_ptr(),
                           self.radiance.data_ptr())

    @staticmethod
    def wrap(dir, pdf_mix, pdf_brdf, strategy, radiance) -> "Samples":
        s = Samples.__new__(Samples)
        s.spp, s.height, s.width = strategy.shape
        s.dir, s.pdf_mix, s.pdf_brdf, s.strategy, s.radiance = dir, pdf_mix, pdf_brdf, strategy, radiance
        s.c = PgSamples(s.spp, _ptr(dir), _ptr(pdf_mix), _ptr(pdf_brdf), _ptr(strategy), _ptr(radiance))
        return s


def new_gamma(height: int, width: int, dtype=None, device="cuda"):
    import torch
    return torch.zeros((8, height, width), dtype=dtype or torch.float32, device=device)


def lights_struct(lights, ambient) -> PgLights:
    import numpy as np
    lights = np.asarray(lights, dtype=np.float32).reshape(-1, 5)
    if lights.shape[0] > MAX_LIGHTS:
        raise ValueError("too many lights")
    L = PgLights()
    L.count = lights.shape[0]
    L.ambient = float(ambient)
    for k in range(lights.shape[0]):
        for c in range(5):
            L.light[k][c] = float(lights[k, c])
    return L


# ---------------------------------------------------------------- the calls
def reproject(p: PgParams, cur: View, prev: View | None, gamma_prev, gamma_out, src_index=None):
    import torch
    _require(src_index, torch.int32, "src_index")
    _check(lib().pg_reproject(C.byref(p), C.byref(cur.c), None if prev is None else C.byref(prev.c),
                              _gamma(gamma_prev), _gamma(gamma_out), _ptr(src_index), _stream()),
           "pg_reproject")


def sample_mis(p: PgParams, view: View, gamma, samples: Samples):
    _check(lib().pg_sample_mis(C.byref(p), C.byref(view.c), _gamma(gamma), C.byref(samples.c),
                               _stream()), "pg_sample_mis")


def reproject_sample(p: PgParams, cur: View, prev: View | None, gamma_prev, gamma_out,
                     samples: Samples):
    _check(lib().pg_reproject_sample(C.byref(p), C.byref(cur.c),
                                     None if prev is None else C.byref(prev.c), _gamma(gamma_prev),
                                     _gamma(gamma_out), C.byref(samples.c), _stream()),
           "pg_reproject_sample")


def pdf(p: PgParams, view: View, gamma, dirs, components: bool = False):
    """Densities of directions dirs [3][n][H][W]; returns D (and p_g, p_b)."""
    import torch
    _require(dirs, torch.float32, "dirs")
    n = dirs.shape[1]
    shape = (n, view.height, view.width)
    pmix = torch.empty(shape, dtype=torch.float32, device=dirs.device)
    pg = torch.empty_like(pmix) if components else None
    pb = torch.empty_like(pmix) if components else None
    _check(lib().pg_pdf(C.byref(p), C.byref(view.c), _gamma(gamma), n, _ptr(dirs), _ptr(pmix),
                        _ptr(pg), _ptr(pb), _stream()), "pg_pdf")
    return (pmix, pg, pb) if components else pmix


def light_field(lights: PgLights, view: View, vis, samples: Samples):
    import torch
    _require(vis, torch.uint8, "vis")
    _check(lib().pg_light_field(C.byref(lights), C.byref(view.c), _ptr(vis), C.byref(samples.c),
                                _stream()), "pg_light_field")


def em_update(p: PgParams, view: View, samples: Samples, gamma, iterations: int = 1):
    _check(lib().pg_em_update(C.byref(p), C.byref(view.c), C.byref(samples.c), _gamma(gamma),
                              iterations, _stream()), "pg_em_update")


def nll_backward(p: PgParams, view: View, samples: Samples, theta, grad_out=None,
                 want_grad: bool = True, want_nll: bool = True):
    import torch
    _require(theta, torch.float32, "theta")
    _require(grad_out, torch.float32, "grad_out")
    grad = torch.empty_like(theta) if want_grad else None
    nll = torch.empty(theta.shape[1:], dtype=torch.float32, device=theta.device) if want_nll else None
    _check(lib().pg_nll_backward(C.byref(p), C.byref(view.c), C.byref(samples.c), _ptr(theta),
                                 _ptr(grad_out), _ptr(grad), _ptr(nll), _stream()),
           "pg_nll_backward")
    return nll, grad


def estimate(p: PgParams, view: View, samples: Samples):
    """Per-pixel first-bounce estimate: mean of f_r L cos / D over the samples [H][W]."""
    import torch
    out = torch.empty((view.height, view.width), dtype=torch.float32, device=samples.dir.device)
    _check(lib().pg_estimate(C.byref(p), C.byref(view.c), C.byref(samples.c), _ptr(out), _stream()),
           "pg_estimate")
    return out


def batch_table_bytes(n_views: int) -> int:
    return int(lib().pg_batch_table_bytes(n_views))


def batch_pack(views, host_table) -> None:
    """Pack a sequence of PgBatchView into host_table (a uint8 CPU tensor,
    pinned for graph capture)."""
    if host_table.is_cuda or not host_table.is_contiguous():
        raise ValueError("host_table must be a contiguous host tensor")
    arr = (PgBatchView * len(views))(*views)
    _check(lib().pg_batch_pack(arr, len(views), C.c_void_p(host_table.data_ptr()),
                               host_table.numel() * host_table.element_size()), "pg_batch_pack")


def frame_batched(host_table, device_table) -> None:
    """Upload the packed table and run the batched frame on the current stream."""
    _require(device_table, None, "device_table")
    n = min(host_table.numel() * host_table.element_size(),
            device_table.numel() * device_table.element_size())
    _check(lib().pg_frame_batched(C.c_void_p(host_table.data_ptr()), _ptr(device_table), n,
                                  _stream()), "pg_frame_batched")


NOALLOC_TABLE_BYTES = 65536  # PG_NOALLOC_TABLE_BYTES


def frame_batched_noalloc(host_table) -> None:
    """pg_frame_batched with the device table in the library's own array (no
    device buffer from the caller; calls on one GPU must not overlap)."""
    if host_table.is_cuda or not host_table.is_contiguous():
        raise ValueError("host_table must be a contiguous host tensor")
    _check(lib().pg_frame_batched_noalloc(C.c_void_p(host_table.data_ptr()),
                                          host_table.numel() * host_table.element_size(), _stream()),
           "pg_frame_batched_noalloc")


# ------------------------------------------------- K Gaussian lobes per pixel
def new_lobes_gamma(lobes: int, height: int, width: int, device="cuda"):
    """FP32 state of K lobes, [6K + 2][H][W]."""
    import torch
    return torch.zeros((6 * lobes + 2, height, width), dtype=torch.float32, device=device)


def _lobes_state(t, lobes, name, view):
    import torch
    if t is None:
        return None
    _require(t, torch.float32, name)
    want = (6 * lobes + 2, view.height, view.width)
    if tuple(t.shape) != want:
        raise ValueError(f"{name} must have shape {want} for {lobes} lobes, got {tuple(t.shape)}")
    return _ptr(t)


def _samples_fit(samples, view):
    if (samples.height, samples.width) != (view.height, view.width):
        raise ValueError(f"samples are {samples.height}x{samples.width}, the view {view.height}x{view.width}")


def reproject_sample_lobes(p: PgParams, lobes: int, cur: View, prev: View | None, gamma_prev, gamma_out,
                           samples: Samples):
    _samples_fit(samples, cur)
    if prev is not None and (prev.height, prev.width) != (cur.height, cur.width):
        raise ValueError("prev must have cur's size")
    _check(lib().pg_reproject_sample_lobes(C.byref(p), lobes, C.byref(cur.c),
                                           None if prev is None else C.byref(prev.c),
                                           _lobes_state(gamma_prev, lobes, "gamma_prev", cur),
                                           _lobes_state(gamma_out, lobes, "gamma_out", cur), C.byref(samples.c),
                                           _stream()), "pg_reproject_sample_lobes")


def em_update_lobes(p: PgParams, lobes: int, view: View, samples: Samples, gamma):
    _samples_fit(samples, view)
    _check(lib().pg_em_update_lobes(C.byref(p), lobes, C.byref(view.c), C.byref(samples.c),
                                    _lobes_state(gamma, lobes, "gamma", view), _stream()), "pg_em_update_lobes")


def pdf_lobes(p: PgParams, lobes: int, view: View, gamma, dirs):
    """D of the K-lobe mixture at directions dirs [3][n][H][W]."""
    import torch
    _require(dirs, torch.float32, "dirs")
    n = dirs.shape[1]
    if dirs.dim() != 4 or tuple(dirs.shape) != (3, n, view.height, view.width):
        raise ValueError(f"dirs must have shape (3, n, {view.height}, {view.width}), got {tuple(dirs.shape)}")
    pmix = torch.empty((n, view.height, view.width), dtype=torch.float32, device=dirs.device)
    _check(lib().pg_pdf_lobes(C.byref(p), lobes, C.byref(view.c), _lobes_state(gamma, lobes, "gamma", view), n,
                              _ptr(dirs), _ptr(pmix), _stream()), "pg_pdf_lobes")
    return pmix


# ------------------------------------ positional reuse of virtual point lights
class Ceiling:
    """Device copy of the near-field emitter (lamps [ny][nx][4] FP32) and its struct."""

    def __init__(self, c: dict, device="cuda"):
        import numpy as np
        import torch
        self.lamps = torch.as_tensor(np.ascontiguousarray(c["lamps"], dtype=np.float32)).to(device)
        ny, nx = self.lamps.shape[:2]
        self.c = PgCeiling(float(c["z"]), float(c["period"]), float(c["x0"]), float(c["y0"]), float(c["ambient"]),
                           nx, ny, self.lamps.data_ptr())


def _position(t, view):
    import torch
    _require(t, torch.float32, "position")
    if t is None or tuple(t.shape) != (3, view.height, view.width):
        raise ValueError(f"position must be a (3, {view.height}, {view.width}) device tensor")
    return _ptr(t)


def _hit(t, samples):
    import torch
    _require(t, torch.float32, "hit_dist")
    if t is None or tuple(t.shape) != (samples.spp, samples.height, samples.width):
        raise ValueError(f"hit_dist must be a ({samples.spp}, {samples.height}, {samples.width}) device tensor")
    return _ptr(t)


def light_ceiling(ceiling: Ceiling, view: View, position, samples: Samples, hit_dist):
    _samples_fit(samples, view)
    _check(lib().pg_light_ceiling(C.byref(ceiling.c), C.byref(view.c), _position(position, view),
                                  C.byref(samples.c), _hit(hit_dist, samples), _stream()), "pg_light_ceiling")


def em_update_vpl(p: PgParams, lobes: int, view: View, position, samples: Samples, hit_dist, gamma):
    _samples_fit(samples, view)
    _check(lib().pg_em_update_vpl(C.byref(p), lobes, C.byref(view.c), _position(position, view),
                                  C.byref(samples.c), _hit(hit_dist, samples),
                                  _lobes_state(gamma, lobes, "gamma", view), _stream()), "pg_em_update_vpl")


def philox(counters, seed: int):
    """Philox4x32-10 words for device counters [n][4] (int32 tensor holding uint32 bits)."""
    import torch
    _require(counters, torch.int32, "counters")
    out = torch.empty_like(counters)
    _check(lib().pg_philox(counters.shape[0], _ptr(counters), seed, _ptr(out), _stream()),
           "pg_philox")
    return out


from .guide import BatchedGuide, DeviceFrame, Guide, LobesGuide, NLLFunction  # noqa: E402  (needs the names above)
