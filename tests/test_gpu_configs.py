"""The workloads at their full sizes, through the C ABI, against the FP64
oracle on crops.

Gamma_t on a crop depends on Gamma_{t-1} within 5 px (2 px of motion, 3 px of
neighbour picks), so the oracle free-runs a crop exactly by stepping the crop
grown by 5 px per remaining frame (its dependency cone) on the full-size
frame arrays; teacher-forced checks step the crop (grown by the 3 px the picks
need) from the GPU's previous state and records.

* 1920x1080, spp 1, 64-frame pan, FP32 Gamma: the 256x256 crop at (832, 412)
  teacher-forced at every frame, and free-running after 64 frames (bounded
  through a twin of the oracle's run whose state is rounded to FP32 every
  frame, see assert_free_run).
* 3840x2160, spp 1, 64-frame pan, Gamma stored as FP16 and BF16 (and FP32 for
  reference): per-parameter and per-density errors on the crop at
  (1792, 952) against the free-running FP64 oracle, and the last frame against
  a storage-rounding oracle.
* 3840x2160, spp 4, frame 0: gradient fit of the NLL through NLLFunction
  against 16 batch-EM iterations on the same samples; the adjoint against
  FP64 central differences on the 32x32 crop at (1904, 1064).
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import (TOL_DIR, TOL_EM_FRAME, assert_gamma_close, compare_samples, dev, gamma_errors,
                    host, records_host, rel_err, underflow_mask)
from pgtest import host_gamma, round_storage, ulp_gamma

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

CONE = 5  # px of dependency per frame


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def grow(rect, d, W, H):
    x0, y0, x1, y1 = rect
    return max(0, x0 - d), max(0, y0 - d), min(W, x1 + d), min(H, y1 + d)


def crop_mask(rect, W, H):
    m = np.zeros((H, W), bool)
    x0, y0, x1, y1 = rect
    m[y0:y1, x0:x1] = True
    return m


class OracleCone:
    """FP64 free run of the oracle on the dependency cone of a crop.  With
    round32 the state is rounded to FP32 after every frame: the oracle's own
    trajectory under a perturbation of FP32's size."""

    def __init__(self, seed, spp, crop, frames, W, H, round32=False):
        self.seed, self.spp, self.crop, self.T, self.W, self.H = seed, spp, crop, frames, W, H
        self.round32 = round32
        self.v_prev = None
        self.gamma = None

    def step(self, t, fr):
        W, H = self.W, self.H
        R = grow(self.crop, CONE * (self.T - 1 - t), W, H)
        rr = grow(R, 3, W, H)
        P = O.params(self.seed, frame=t)
        v = O.OView(fr, fr["motion"], fr["disocc"])
        g1, _ = O.reproject(P, v, self.v_prev if self.v_prev is not None else v, self.gamma, rect=rr)
        rec = O.sample(P, v, g1, self.spp, rect=rr)
        rec["radiance"] = O.light(fr["lights"], float(fr["ambient"]), fr["vis"], rec["dir"],
                                  rec["strategy"], rect=rr)
        self.gamma = O.em(P, v, rec, g1, rect=R)
        if self.round32:
            self.gamma = self.gamma.astype(np.float32).astype(np.float64)
        self.v_prev = v
        return v


def teacher_forced_crop(seed, t, fr, v_prev, gamma_prev, rec_gpu, gamma_gpu, crop, W, H, spp=1,
                        storage=None, reproj_gpu=None):
    """Step the crop from the GPU's previous state and records; returns
    (sample stats, EM errors or ulp stats).  With a stored format, the
    reprojection is checked within one unit of the format against the
    storage-rounding oracle, and the sampling and EM steps are taken from the
    GPU's own reprojected state reproj_gpu (the two roundings of a value that
    lies near a boundary of the format may land one unit apart)."""
    P = O.params(seed, frame=t)
    v = O.OView(fr, fr["motion"], fr["disocc"])
    rr = grow(crop, 3, W, H)
    g1, _ = O.reproject(P, v, v_prev if v_prev is not None else v, gamma_prev if t else None, rect=rr)
    if storage:
        g1 = round_storage(g1, storage)
        x0, y0, x1, y1 = rr
        d = np.abs(reproj_gpu - g1)[:, y0:y1, x0:x1]
        over = d > ulp_gamma(g1, storage)[:, y0:y1, x0:x1] + 1e-5 * (np.abs(g1[:, y0:y1, x0:x1]) + 1e-3)
        assert over.sum() <= 1e-3 * over.size, f"reprojection: {int(over.sum())} channels beyond 1 ulp"
        assert (reproj_gpu[7][y0:y1, x0:x1] == g1[7][y0:y1, x0:x1]).all()
        g1 = reproj_gpu
    ro = O.sample(P, v, g1, spp, rect=rr)
    st, _ = compare_samples(rec_gpu, ro, pix_mask=crop_mask(rr, W, H), scene=fr, gamma=g1)
    assert st["dir_max"] <= TOL_DIR, st
    g2, stats = O.em(P, v, rec_gpu, g1, rect=crop, with_stats=True)
    ok = ~underflow_mask(stats) & crop_mask(crop, W, H)
    if storage is None:
        return st, assert_gamma_close(gamma_gpu, g2, TOL_EM_FRAME, mask=ok, what=f"frame {t}")
    g2r = round_storage(g2, storage)
    d = np.abs(gamma_gpu - g2r)
    bound = ulp_gamma(g2r, storage) + 1e-5 * (np.abs(g2r) + 1e-3)
    over = (d > bound) & ok[None]
    assert over.sum() <= 1e-3 * ok.sum() * 8, int(over.sum())
    assert (gamma_gpu[7][ok] == g2r[7][ok]).all()
    return st, {"beyond_1ulp": int(over.sum()), "max_d_over_ulp": float((d / ulp_gamma(g2r, storage))[:, ok].max())}


def free_run_table(name, g_gpu, g_orc, crop):
    x0, y0, x1, y1 = crop
    e = gamma_errors(g_gpu[:, y0:y1, x0:x1].astype(np.float64), g_orc[:, y0:y1, x0:x1])
    say(f"  {name:5s} vs FP64 free run on the crop: " + ", ".join(
        f"{k} max {float(v.max()):.2e} q99.9 {float(np.quantile(v, 0.999)):.2e} median {float(np.median(v)):.2e}"
        for k, v in e.items()))
    return e


# A free-running FP32 state drifts from the FP64 one by the per-frame
# rounding, carried and at some pixels amplified by the trajectory (the EM
# map of a lobe still moving amplifies changes of its inputs).  The twin
# cone measures that carrying on the oracle itself: the same FP64 run with
# its state rounded to FP32 after every frame.  Each quantile of the GPU's
# error (median to max) is bounded by the one-step tolerance or by
# TWIN_FACTOR times the twin's error at that quantile (the GPU's per-frame
# arithmetic rounds a few times more than storing the state does), and by
# FREE_RUN_CAP everywhere.
TWIN_FACTOR = 10.0
FREE_RUN_CAP = 1e-3


def assert_free_run(e, e_twin, what):
    assert (e["k"] == 0).all(), f"{what}: epochs differ"
    for name in ("mu", "sigma", "pi", "W"):
        g, tw = np.asarray(e[name], float).ravel(), np.asarray(e_twin[name], float).ravel()
        assert g.max() <= FREE_RUN_CAP, (what, name, g.max())
        for q in (0.5, 0.9, 0.99, 0.999, 1.0):
            gq, tq = np.quantile(g, q), np.quantile(tw, q)
            assert gq <= max(TOL_EM_FRAME, TWIN_FACTOR * tq), (what, name, q, gq, tq)


def test_1080p_pan_64_frames_crop():
    cfg = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]
    W, H, seed, crop, T = 1920, 1080, cfg["seed"], cfg["crop"], cfg["frames"]
    say(f"case: 1080p pan {T} frames, crop {crop}")
    seq = wl.Sequence(W, H, seed)
    cone = OracleCone(seed, 1, crop, T, W, H)
    twin = OracleCone(seed, 1, crop, T, W, H, round32=True)
    guide = None
    prev_dev = v_prev = None
    worst = {}
    for t in range(T):
        fr = seq.frame(t)
        if guide is None:
            guide = pg.Guide(W, H, fr["lights"], float(fr["ambient"]), spp=1, seed=seed)
        cur = pg.DeviceFrame(fr)
        g_prev = host(guide.state)
        guide.step(cur, prev_dev, frame=t)
        torch.cuda.synchronize()
        st, e = teacher_forced_crop(seed, t, fr, v_prev, g_prev, records_host(guide.samples), host(guide.state),
                                    crop, W, H)
        for k, val in e.items():
            worst[k] = max(worst.get(k, 0.0), float(val))
        worst["dir"] = max(worst.get("dir", 0.0), st["dir_max"])
        worst["flips"] = worst.get("flips", 0) + st["flips"]
        v_prev = cone.step(t, fr)
        twin.step(t, fr)
        prev_dev = cur
    say(f"  teacher-forced, worst over {T} frames: {worst}")
    e = free_run_table("f32", host(guide.state), cone.gamma, crop)
    e_twin = free_run_table("twin", twin.gamma, cone.gamma, crop)
    k = host(guide.state)[7, crop[1]:crop[3], crop[0]:crop[2]]
    say(f"  k after {T} frames: mean {k.mean():.2f}, share at kMax {(k == 16).mean():.3f}")
    assert_free_run(e, e_twin, "1080p free run")


@pytest.mark.parametrize("W,H,crop", [(1920, 1080, (832, 412, 1088, 668)), (3840, 2160, (1792, 952, 2048, 1208))],
                         ids=["1080p", "4k"])
def test_pan_64_frames_lowprec_crop(W, H, crop):
    """FP16/BF16 (and FP32) Gamma over the 64-frame pan: the last frame
    against the storage-rounding oracle (implementation), and the
    free-running stored states and their densities against the free-running
    FP64 oracle on the crop (format error), printed per parameter."""
    cfg = wl.CONFIGS["1080p_4k_spp1_64f_fp16_bf16"]
    seed, T = cfg["seed"], cfg["frames"]
    say(f"case: {W}x{H} pan {T} frames, FP16/BF16/FP32 Gamma, crop {crop}")
    seq = wl.Sequence(W, H, seed)
    cone = OracleCone(seed, 1, crop, T, W, H)
    twin = OracleCone(seed, 1, crop, T, W, H, round32=True)
    dts = {"f16": torch.float16, "bf16": torch.bfloat16, "f32": torch.float32}
    guides = {}
    prev_dev = v_prev = None
    keep = {}
    for t in range(T):
        fr = seq.frame(t)
        if not guides:
            guides = {k: pg.Guide(W, H, fr["lights"], float(fr["ambient"]), spp=1, seed=seed, gamma_dtype=d)
                      for k, d in dts.items()}
        cur = pg.DeviceFrame(fr)
        last = t == T - 1
        for k, g in guides.items():
            if last and k != "f32":
                keep[k] = host_gamma(g.state)
                # the reprojected state this frame samples and trains with
                tmp = torch.empty_like(g.state)
                pg.reproject(g.params(t), cur.view, prev_dev.view, g.state, tmp)
                keep[k + "_reproj"] = host_gamma(tmp)
            g.step(cur, prev_dev, frame=t)
            if last and k != "f32":
                torch.cuda.synchronize()
                keep[k + "_rec"] = records_host(g.samples)
                keep[k + "_out"] = host_gamma(g.state)
        if last:
            v_last_prev = v_prev
            fr_last = fr
        v_prev = cone.step(t, fr)
        twin.step(t, fr)
        prev_dev = cur
    torch.cuda.synchronize()
    # implementation: the last frame against the storage-rounding oracle
    for k in ("f16", "bf16"):
        st, u = teacher_forced_crop(seed, T - 1, fr_last, v_last_prev, keep[k], keep[k + "_rec"], keep[k + "_out"],
                                    crop, W, H, storage=k, reproj_gpu=keep[k + "_reproj"])
        say(f"  {k} frame {T - 1} vs storage-rounding oracle: samples dir max {st['dir_max']:.2e}, "
            f"flips {st['flips']}; {u}")
    # format error: free-running states against the FP64 oracle
    errs = {k: free_run_table(k, host_gamma(g.state), cone.gamma, crop) for k, g in guides.items()}
    e_twin = free_run_table("twin", twin.gamma, cone.gamma, crop)
    # densities of one set of directions under each stored state and under the FP64 state
    v = O.OView(fr_last, fr_last["motion"], fr_last["disocc"])
    P = O.params(seed, frame=T - 1)
    dirs = records_host(guides["f32"].samples)["dir"]
    Do, _, _ = O.pdf(P, v, cone.gamma, dirs, rect=crop)
    m = crop_mask(crop, W, H)[None] & (Do > 1e-30)
    p = pg.params(seed, frame=T - 1)
    for k, g in guides.items():
        D = host(pg.pdf(p, cur.view, g.state, dev(dirs)))
        r = rel_err(D[m], Do[m])
        say(f"  {k:5s} D vs FP64 on the crop: max {r.max():.2e} q99 {np.quantile(r, 0.99):.2e} "
            f"median {np.median(r):.2e}")
    for k, lim in (("f16", 2e-3), ("bf16", 2e-2)):
        assert (errs[k]["k"] == 0).mean() > 0.99
        assert np.median(errs[k]["mu"]) <= lim and np.median(errs[k]["pi"]) <= lim, k
    assert_free_run(errs["f32"], e_twin, f"{W}x{H} FP32 free run")


def test_4k_spp4_gradient_fit_and_adjoint():
    cfg = wl.CONFIGS["4k_spp4_gradient_fit"]
    W, H, spp, seed = 3840, 2160, cfg["spp"], cfg["seed"]
    x0, y0, x1, y1 = cfg["fd_crop"]
    say(f"case: 4K spp {spp} gradient fit, FD crop {cfg['fd_crop']}")
    scene = wl.make_scene(W, H, seed)
    view = pg.View.from_scene(scene)
    p0 = pg.params(seed, frame=0)
    g0 = torch.zeros((8, H, W), dtype=torch.float32, device="cuda")
    s = pg.Samples(spp, H, W)
    pg.reproject_sample(p0, view, None, None, g0, s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), view, dev(scene["vis"]), s)
    torch.cuda.synchronize()
    g0h = host(g0)
    # 16 batch-EM iterations (no clamp), scored by the same NLL
    pb = pg.params(seed, frame=0, flags=pg.PG_NO_CLAMP | pg.PG_EM_BATCH)
    ge = g0.clone()
    pg.em_update(pb, view, s, ge, iterations=16)
    gem = host(ge)
    l11 = np.sqrt(np.maximum(gem[2], 0))
    l21 = np.where(l11 > 0, gem[3] / np.where(l11 > 0, l11, 1), 0)
    l22 = np.sqrt(np.maximum(gem[4] - l21 ** 2, 0))
    pi = np.clip(gem[5], 1e-6, 1 - 1e-6)
    th_em = np.stack([gem[0], gem[1], l11, l21, l22, np.log(pi / (1 - pi)), gem[6], gem[7]]).astype(np.float32)
    pn = pg.params(seed, frame=0, flags=pg.PG_NO_CLAMP)
    nll_em, _ = pg.nll_backward(pn, view, s, dev(th_em), want_grad=False)
    total_em = float(nll_em.double().sum())
    # gradient fit from the new-model state: Adam, 300 steps, lr 0.02
    th0 = np.stack([g0h[0], g0h[1], np.sqrt(g0h[2]), g0h[3], np.sqrt(g0h[4]), np.log(g0h[5] / (1 - g0h[5])),
                    g0h[6], g0h[7]]).astype(np.float32)
    theta = torch.tensor(th0, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([theta], lr=0.02)
    mask = torch.zeros_like(theta)
    mask[:6] = 1
    first = last = None
    for it in range(300):
        opt.zero_grad()
        loss = pg.NLLFunction.apply(theta, pn, view, s).double().sum()
        loss.backward()
        theta.grad.mul_(mask)
        opt.step()
        if it == 0:
            first = float(loss.detach())
        last = float(loss.detach())
    torch.cuda.synchronize()
    say(f"  summed NLL over {W * H} px: EM(16) {total_em:.1f}, gradient fit start {first:.1f} end {last:.1f}")
    assert np.isfinite(total_em) and last < first
    assert last <= total_em + 0.01 * abs(total_em)
    # adjoint against FP64 central differences (h = 1e-4) on the crop
    rng = np.random.default_rng(seed)
    th = th_em.copy()
    th[0] = rng.uniform(0.3, 0.7, (H, W))
    th[1] = rng.uniform(0.3, 0.7, (H, W))
    th[2] = rng.uniform(0.05, 0.2, (H, W))
    th[3] = rng.uniform(-0.05, 0.05, (H, W))
    th[4] = rng.uniform(0.05, 0.2, (H, W))
    th[5] = rng.uniform(-2, 2, (H, W))
    _, grad = pg.nll_backward(pn, view, s, dev(th))
    torch.cuda.synchronize()
    grad = host(grad)
    rec = records_host(s)
    rec = {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in rec.items()}
    P = O.params(seed, frame=0, flags=pg.PG_NO_CLAMP)
    ov = O.OView(scene)
    rect = (x0, y0, x1, y1)
    th64 = th.astype(np.float64)
    # the oracle's analytic gradient at the GPU's inputs
    _, grad_o = O.nll(P, ov, rec, th64, rect=rect)
    for c in range(6):
        go = grad_o[c, y0:y1, x0:x1]
        gg = grad[c, y0:y1, x0:x1]
        sc = np.abs(go).max() + 1e-30
        e = np.abs(gg - go) / (np.abs(go) + 1e-3 * sc)
        say(f"  channel {c} vs oracle gradient: rel err p99 {np.quantile(e, 0.99):.2e} max {e.max():.2e}")
        assert np.quantile(e, 0.99) <= 1e-4 and e.max() <= 1e-3, c
    h = 1e-4
    for c in range(6):
        tp, tm = th64.copy(), th64.copy()
        tp[c, y0:y1, x0:x1] += h
        tm[c, y0:y1, x0:x1] -= h
        fd = (O.nll(P, ov, rec, tp, rect=rect)[0] - O.nll(P, ov, rec, tm, rect=rect)[0]) / (2 * h)
        fd = fd[y0:y1, x0:x1]
        gg = grad[c, y0:y1, x0:x1]
        sc = np.abs(fd).max() + 1e-30
        e = np.abs(gg - fd) / (np.abs(fd) + 1e-2 * sc)
        say(f"  channel {c}: rel err p99 {np.quantile(e, 0.99):.2e} max {e.max():.2e}")
        assert np.quantile(e, 0.99) <= 1e-4 and e.max() <= 1e-3, c
