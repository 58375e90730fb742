"""Shared helpers of the GPU parity tests: device round trips, one GPU frame
with all its intermediates, and the comparison metrics with their bounds."""
import numpy as np
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl

# Tolerances (directions and densities: 1e-5; EM parameters: 1e-4 after
# the stated frames, 1e-5 for one teacher-forced frame).
TOL_DIR = 1e-5
TOL_PDF = 1e-5
TOL_EM_FRAME = 1e-5
TOL_EM_RUN = 1e-4
MARGIN = 1e-5  # decisions closer than this to their threshold may go either way


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t):
    return t.detach().float().cpu().numpy() if t.dtype in (torch.float16, torch.bfloat16) \
        else t.detach().cpu().numpy()


def gpu_view(scene, motion=None, disocc=None):
    return pg.View.from_scene(scene, "cuda", motion, disocc)


def random_gamma(H, W, rng, k_lo=1, k_hi=16):
    """A valid, varied model state (k >= 1 so that guiding is active)."""
    sxx = rng.uniform(0.0005, 0.03, (H, W))
    syy = rng.uniform(0.0005, 0.03, (H, W))
    rho = rng.uniform(-0.8, 0.8, (H, W))
    g = np.stack([rng.uniform(0.05, 0.95, (H, W)), rng.uniform(0.05, 0.95, (H, W)), sxx,
                  rho * np.sqrt(sxx * syy), syy, rng.uniform(0.05, 0.95, (H, W)),
                  rng.uniform(0.0, 20.0, (H, W)), rng.integers(k_lo, k_hi + 1, (H, W))])
    return g.astype(np.float32)


def records_host(s: pg.Samples):
    return dict(dir=host(s.dir), pdf_mix=host(s.pdf_mix), pdf_brdf=host(s.pdf_brdf),
                strategy=host(s.strategy), radiance=host(s.radiance))


def paired_ratio_ci(err_a, err_b, n_boot=2000, seed=0):
    """sum(err_a) / sum(err_b) and its 95% bootstrap interval, resampling the
    pixels with replacement and keeping each pixel's pair of errors together
    (both runs drew the same random numbers for a pixel, so the pairing
    removes most of the noise the two estimates share)."""
    a = np.asarray(err_a, np.float64).reshape(-1)
    b = np.asarray(err_b, np.float64).reshape(-1)
    rng = np.random.default_rng(seed)
    r = np.empty(n_boot)
    for i0 in range(0, n_boot, 100):
        idx = rng.integers(0, a.size, (min(100, n_boot - i0), a.size), dtype=np.int32)
        r[i0:i0 + idx.shape[0]] = a[idx].sum(1) / b[idx].sum(1)
    return float(a.sum() / b.sum()), float(np.quantile(r, 0.025)), float(np.quantile(r, 0.975))


def rel_err(a, b, floor=1e-30):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def gamma_errors(g_gpu, g_orc):
    """Per-channel error of model states: mu and pi absolute, Sigma relative to
    trace(Sigma) + 2 eps, W relative, k exact."""
    g_gpu = np.asarray(g_gpu, np.float64)
    g_orc = np.asarray(g_orc, np.float64)
    tr = g_orc[2] + g_orc[4] + 2 * 2.5e-4
    e = dict(
        mu=np.maximum(np.abs(g_gpu[0] - g_orc[0]), np.abs(g_gpu[1] - g_orc[1])),
        sigma=np.max(np.abs(g_gpu[2:5] - g_orc[2:5]), axis=0) / tr,
        pi=np.abs(g_gpu[5] - g_orc[5]),
        W=np.abs(g_gpu[6] - g_orc[6]) / np.maximum(np.abs(g_orc[6]), 1e-6),
        k=np.abs(g_gpu[7] - g_orc[7]),
    )
    return e


EVIDENCE_FLOOR = 2.0 ** -100


def underflow_mask(stats):
    """Pixels whose Gaussian evidence B1 is below FP32's reach relative to B0
    (B1 < 2^-100 B0): there an FP32 E-step may see no Gaussian evidence at
    all, so whether the lobe moves is decided by the precision itself."""
    B0, B1 = stats
    return (B1 > 0) & (B1 < EVIDENCE_FLOOR * np.maximum(B0, 1e-300))


def describe_worst(g_gpu, g_orc, g_in=None, key="sigma"):
    """Text naming the worst pixel of one error channel (for failure messages)."""
    e = gamma_errors(g_gpu, g_orc)[key]
    bad = ~np.isfinite(e)
    y, x = (np.argwhere(bad)[0] if bad.any() else np.unravel_index(np.argmax(e), e.shape))
    out = (f"worst {key} at (y={y}, x={x}): nan gpu={int((~np.isfinite(g_gpu)).any(0).sum())} "
           f"nan oracle={int((~np.isfinite(g_orc)).any(0).sum())}\n"
           f"  gpu    {np.array2string(np.asarray(g_gpu)[:, y, x], precision=9)}\n"
           f"  oracle {np.array2string(np.asarray(g_orc)[:, y, x], precision=9)}")
    if g_in is not None:
        out += f"\n  input  {np.array2string(np.asarray(g_in)[:, y, x], precision=9)}"
    return out


def assert_gamma_quantile(g_gpu, g_orc, tol_bulk, tol_max, q=0.999, mask=None, what=""):
    """k exact; every other channel within tol_bulk for a fraction q of the
    pixels and within tol_max everywhere (for adversarial states whose lobes
    sit far from the samples, where FP32 rounding of u is amplified by the
    Mahalanobis gradient |Sigma^-1 (u - mu)|)."""
    e = gamma_errors(g_gpu, g_orc)
    m = np.ones(g_orc.shape[1:], bool) if mask is None else mask
    assert (e["k"][m] == 0).all(), f"{what}: k differs"
    out = {}
    for key in ("mu", "sigma", "pi", "W"):
        v = e[key][m]
        if v.size == 0:
            continue
        out[key] = (float(np.quantile(v, q)), float(v.max()))
        assert np.quantile(v, q) <= tol_bulk, f"{what}: {key} q{q} {np.quantile(v, q):.2e}"
        assert v.max() <= tol_max, f"{what}: {key} max {v.max():.2e}"
    return out


def assert_gamma_close(g_gpu, g_orc, tol, mask=None, what="", g_in=None):
    e = gamma_errors(g_gpu, g_orc)
    m = np.ones(g_orc.shape[1:], bool) if mask is None else mask
    for key in ("mu", "sigma", "pi", "W"):
        if not (e[key][m] <= tol).all() or not (e["k"][m] == 0).all():
            print(describe_worst(g_gpu, g_orc, g_in, key), flush=True)
            break
    assert (e["k"][m] == 0).all(), f"{what}: k differs at {np.argwhere((e['k'] != 0) & m)[:5]}"
    for key in ("mu", "sigma", "pi", "W"):
        worst = e[key][m].max() if m.any() else 0.0
        assert worst <= tol, f"{what}: {key} error {worst:.3e} > {tol:.0e}"
    return {k: float(v[m].max()) if m.any() else 0.0 for k, v in e.items()}


U32 = 2.0 ** -24


def conditioning(scene, gamma, dirs, eps=2.5e-4):
    """Relative sensitivities of the densities to a unit change of an FP32
    direction, from the oracle's quantities (directions [3][n][H][W]):
      GGX lobe    |d ln D_ggx / dh| <= 2 / alpha,
      cosine term |d ln cos / dw|   =  1 / cos,
      Gaussian    |d ln N / du|     =  |(Sigma + eps I)^-1 (u - mu)|.
    Returns (kappa_b, kappa_g) per direction."""
    n = np.asarray(scene["normal"], np.float64)
    n = n / np.linalg.norm(n, axis=0, keepdims=True)
    d = np.asarray(dirs, np.float64)
    cos = np.abs((d * n[:, None]).sum(0))
    alpha = np.asarray(scene["roughness"], np.float64)[None] ** 2
    kb = 2.0 / alpha + 1.0 / np.maximum(cos, 1e-30)
    # Mahalanobis gradient of the Gaussian on the square
    H, W = n.shape[1:]
    kg = np.zeros(d.shape[1:])
    t, b = O.onb(np.moveaxis(n, 0, -1).reshape(-1, 3))
    t = t.reshape(H, W, 3)
    b = b.reshape(H, W, 3)
    nn = np.moveaxis(n, 0, -1)
    g = np.asarray(gamma, np.float64)
    A = g[2] + eps
    Bm = g[3]
    Cm = g[4] + eps
    det = A * Cm - Bm * Bm
    for j in range(d.shape[1]):
        w = np.moveaxis(d[:, j], 0, -1)
        loc = np.stack([(w * t).sum(-1), (w * b).sum(-1), (w * nn).sum(-1)], -1)
        ok = loc[..., 2] > 0
        u = np.full(loc.shape[:-1] + (2,), 0.5)
        if ok.any():
            u[ok] = O.hemi2sq(loc[ok])
        dx, dy = u[..., 0] - g[0], u[..., 1] - g[1]
        vx = (Cm * dx - Bm * dy) / det
        vy = (-Bm * dx + A * dy) / det
        kg[j] = np.where(ok, np.hypot(vx, vy), 0.0)
    return kb, kg


def pdf_bounds(kb, kg):
    """Bounds on the relative error of p_b, p_g and D for FP32 directions:
    TOL_PDF plus 16 FP32 ulps times each density's sensitivity (the direction
    itself is only known to a few ulps, and its evaluation adds a few more)."""
    tb = TOL_PDF + 16 * U32 * kb
    tg = TOL_PDF + 16 * U32 * kg
    return tb, tg, np.maximum(tb, tg)


def compare_samples(rec_gpu, rec_orc, pix_mask=None, scene=None, gamma=None):
    """Strategy codes must agree except where the oracle's decision margin is
    below MARGIN; where they agree, directions and densities are compared:
    99.9% of densities within TOL_PDF, every one within its conditioning
    bound (pdf_bounds) when the scene and state are given."""
    sg, so = rec_gpu["strategy"], rec_orc["strategy"]
    near = rec_orc["margin"] < MARGIN
    m = np.ones(sg.shape, bool) if pix_mask is None else np.broadcast_to(pix_mask, sg.shape)
    bad = (sg != so) & ~near & m
    assert not bad.any(), f"strategy codes differ away from thresholds at {np.argwhere(bad)[:5]}"
    same = (sg == so) & m
    live = same & ((sg == 1) | (sg == 2))
    dd = np.sqrt(((rec_gpu["dir"] - rec_orc["dir"]) ** 2).sum(0))
    stats = dict(n=int(live.sum()), flips=int(((sg != so) & m).sum()),
                 dir_max=float(dd[live].max()) if live.any() else 0.0)
    if scene is not None:
        tb, _, tm = pdf_bounds(*conditioning(scene, gamma, rec_orc["dir"]))
    for key in ("pdf_mix", "pdf_brdf"):
        r_all = rel_err(rec_gpu[key], rec_orc[key])
        r = r_all[live]
        stats[key + "_max"] = float(r.max()) if r.size else 0.0
        stats[key + "_p999"] = float(np.quantile(r, 0.999)) if r.size else 0.0
        if scene is not None:
            bound = (tm if key == "pdf_mix" else tb)
            over = live & (r_all > bound)
            assert not over.any(), f"{key}: {r_all[over].max():.2e} beyond its bound at {np.argwhere(over)[:3]}"
            stats[key + "_bound_ratio"] = float((r_all[live] / bound[live]).max()) if r.size else 0.0
    nulls = same & (sg != 1) & (sg != 2)
    assert (rec_gpu["pdf_mix"][nulls] == 0).all() and (rec_gpu["dir"][:, nulls] == 0).all()
    return stats, live


class GpuFrames:
    """The GPU path frame by frame, keeping every intermediate on request."""

    def __init__(self, width, height, lights, ambient, spp, seed, gamma_dtype=torch.float32,
                 fused=True, view_id=0, **over):
        self.g = pg.Guide(width, height, lights, ambient, spp=spp, seed=seed, view_id=view_id,
                          gamma_dtype=gamma_dtype, fused=fused, **over)
        self.prev = None

    def step(self, t, fr, keep=True):
        cur = pg.DeviceFrame(fr)
        g_prev = self.g.state.clone() if keep else None
        if keep:
            # the reprojected state this frame samples and trains with
            g_reproj = torch.empty_like(g_prev)
            pg.reproject(self.g.params(t), cur.view, self.prev.view if (self.prev is not None and t) else None,
                         g_prev if t else None, g_reproj)
        out = self.g.step(cur, self.prev, frame=t)
        self.prev = cur
        torch.cuda.synchronize()
        if not keep:
            return None
        return dict(gamma_prev=host_gamma(g_prev), gamma_reproj=host_gamma(g_reproj), gamma=host_gamma(out),
                    rec=records_host(self.g.samples))


def oracle_reproject_from(P, scene, mv, mask, gamma_prev):
    v = O.OView(scene, mv, mask)
    return O.reproject(P, v, O.OView(scene), gamma_prev)


# ------------------------------------------------------- storage formats
FMT = {"f16": (torch.float16, 65504.0, 10), "bf16": (torch.bfloat16, 3.38953139e38, 7)}


def _round_format(g, fmt):
    if fmt == "f16":
        return g.astype(np.float16).astype(np.float64)
    f = g.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def round_storage(g, fmt):
    """Round a state to its storage in the format (nearest even; W
    saturates; planes 0 and 1 stored as mu - 1/2), returned as the values it
    represents."""
    g = np.asarray(g, np.float64).copy()
    _, vmax, _ = FMT[fmt]
    g[6] = np.minimum(g[6], vmax)
    g[:2] -= 0.5
    g = _round_format(g, fmt)
    g[:2] += 0.5
    return g


def host_gamma(t):
    """A device state as the values it represents (float64): FP16/BF16 states
    hold mu - 1/2 in planes 0 and 1."""
    g = host(t).astype(np.float64)
    if t.dtype in (torch.float16, torch.bfloat16):
        g[:2] += 0.5
    return g


def ulp(v, fmt):
    """One unit in the last place of the format at |v| (subnormal floor)."""
    _, _, mant = FMT[fmt]
    v = np.maximum(np.abs(np.asarray(v, np.float64)), 2.0 ** -14 if fmt == "f16" else 2.0 ** -126)
    return 2.0 ** (np.floor(np.log2(v)) - mant)


def ulp_gamma(g, fmt):
    """One unit in the last place of each stored channel of state values g
    (planes 0 and 1 are stored as mu - 1/2)."""
    g = np.asarray(g, np.float64).copy()
    g[:2] -= 0.5
    return ulp(g, fmt)
