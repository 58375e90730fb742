"""Parity of the K-lobe HIP path (pg_reproject_sample_lobes, pg_em_update_lobes,
pg_pdf_lobes) with the oracle's K-lobe functions, through the C ABI.

Same-input checks per call on ragged sizes that span several tiles, a
teacher-forced run over a moving sequence, K = 1 against the single-lobe
kernels, and sampled pixels of the 1080p pan at K = 2 in the launch
configuration the bench times.  Reset flags, epochs and strategy codes away
from their thresholds must match exactly; floating point within the
tolerances of tests/pgtest.py."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import (MARGIN, paired_ratio_ci, TOL_DIR, TOL_EM_FRAME, TOL_EM_RUN, TOL_PDF, EVIDENCE_FLOOR, assert_gamma_close,
                    assert_gamma_quantile, dev, gpu_view, host, records_host, rel_err)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _p(seed, frame, **kw):
    return pg.params(seed, frame=frame, **kw), O.params(seed, frame=frame, **kw)


def random_lobes(K, H, W, rng, k_lo=1, k_hi=16):
    """A valid, varied K-lobe state (weights summing to at most 0.95)."""
    planes = []
    for _ in range(K):
        sxx = rng.uniform(0.0005, 0.03, (H, W))
        syy = rng.uniform(0.0005, 0.03, (H, W))
        rho = rng.uniform(-0.8, 0.8, (H, W))
        planes += [rng.uniform(0.05, 0.95, (H, W)), rng.uniform(0.05, 0.95, (H, W)), sxx,
                   rho * np.sqrt(sxx * syy), syy, rng.uniform(0.05, 0.95, (H, W)) / K]
    planes += [rng.uniform(0.0, 20.0, (H, W)), rng.integers(k_lo, k_hi + 1, (H, W))]
    return np.stack(planes).astype(np.float32)


def lobe_slices(g, K):
    """The K single-lobe views [8][H][W] of a K-lobe state (lobe j, W, k)."""
    return [np.concatenate([g[6 * j:6 * j + 6], g[6 * K:6 * K + 2]]) for j in range(K)]


def lobes_underflow(stats):
    """Pixels where some lobe's evidence is below FP32's reach (B1_j < 2^-100 B0)."""
    B0 = np.maximum(stats[0], 1e-300)
    B1 = stats[1:]
    return ((B1 > 0) & (B1 < EVIDENCE_FLOOR * B0)).any(0)


def compare_records(rec_g, rec_o, what):
    """Strategy codes equal away from the oracle's decision margins; where
    they agree and the sample is live: directions within TOL_DIR, densities
    within TOL_PDF for 99.9% and 1e-3 for all (FP32 directions amplify the
    rounding by the lobes' Mahalanobis gradients); nulls record zeros."""
    sg, so = rec_g["strategy"], rec_o["strategy"]
    near = rec_o["margin"] < MARGIN
    bad = (sg != so) & ~near
    assert not bad.any(), f"{what}: strategy differs at {np.argwhere(bad)[:5]}"
    live = (sg == so) & ((sg == 1) | (sg == 2))
    dd = np.sqrt(((rec_g["dir"] - rec_o["dir"]) ** 2).sum(0))
    assert dd[live].max(initial=0) <= TOL_DIR, f"{what}: dir {dd[live].max():.2e}"
    out = dict(n=int(live.sum()), guided=int((live & (sg == 2)).sum()), flips=int((sg != so).sum()),
               dir=float(dd[live].max(initial=0)))
    for key in ("pdf_mix", "pdf_brdf"):
        r = rel_err(rec_g[key][live], rec_o[key][live])
        if r.size:
            assert np.quantile(r, 0.999) <= TOL_PDF, f"{what}: {key} q999 {np.quantile(r, 0.999):.2e}"
            assert r.max() <= 1e-3, f"{what}: {key} max {r.max():.2e}"
            out[key] = (float(np.quantile(r, 0.999)), float(r.max()))
    nulls = (sg == so) & (sg != 1) & (sg != 2)
    assert (rec_g["pdf_mix"][nulls] == 0).all() and (rec_g["dir"][:, nulls] == 0).all()
    return out


def rim_margin(g, K):
    """Smallest cos(theta) of a lobe mean of each pixel (a reprojection that
    lands this close to the horizon may keep or reset in either precision)."""
    m = np.full(g.shape[1:], np.inf)
    for j in range(K):
        u = np.clip(np.stack([g[6 * j], g[6 * j + 1]], -1).reshape(-1, 2), 0, 1)
        m = np.minimum(m, O.sq2hemi(u)[:, 2].reshape(g.shape[1:]))
    return m


def _is_reset(g, K, P):
    ref = O.reproject_k(P, K, O.OView(wl.make_scene(1, 1, 0)), None, None)[0][:, 0, 0].astype(np.float32)
    return (g == ref[:, None, None]).all(0)


# ------------------------------------------------------- reprojection + sampling
@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("W,H,spp,frame", [(83, 45, 2, 3), (130, 21, 1, 5), (67, 70, 5, 0)])
def test_reproject_sample_parity(K, W, H, spp, frame):
    say(f"case: lobes reproject+sample K {K} {W}x{H} spp {spp} frame {frame}")
    seed = 12000 + 31 * K + W + H
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    g_prev = random_lobes(K, H, W, rng, k_lo=0)
    g_prev[2, 0, 0] = np.nan
    mv, mask = wl.make_motion(W, H, seed, frame)
    p, P = _p(seed, frame)
    cur, prev = gpu_view(scene, dev(mv), dev(mask)), gpu_view(scene)
    gp = dev(g_prev)
    go = torch.full_like(gp, float("nan"))
    s = pg.Samples(spp, H, W)
    pg.reproject_sample_lobes(p, K, cur, prev if frame else None, gp if frame else None, go, s)
    torch.cuda.synchronize()
    gg = host(go)
    vo = O.OView(scene, mv, mask)
    g_o, src_o = O.reproject_k(P, K, vo, O.OView(scene), g_prev if frame else None)
    kept_o = src_o >= 0
    reset_g = _is_reset(gg, K, P)
    near = (rim_margin(g_o, K) < 1e-4) | (rim_margin(gg, K) < 1e-4)
    bad = (reset_g == kept_o) & ~near
    assert not bad.any(), f"reset decisions differ at {np.argwhere(bad)[:5]}"
    if frame == 0:
        assert reset_g.all()
    both = kept_o & ~reset_g
    qy, qx = np.divmod(src_o[both], W)
    for j in range(K):
        assert (gg[6 * j + 2:6 * j + 6, both] == g_prev[6 * j + 2:6 * j + 6, qy, qx]).all()
        assert np.abs(gg[6 * j:6 * j + 2, both] - g_o[6 * j:6 * j + 2, both]).max(initial=0) <= TOL_DIR
    assert (gg[6 * K:, both] == g_prev[6 * K:, qy, qx]).all()
    assert np.abs(gg[:, ~kept_o & reset_g] - g_o[:, ~kept_o & reset_g]).max(initial=0) <= 1e-7
    # the records, with the oracle sampling the GPU's reprojected state
    rec_o = O.sample_k(P, K, vo, gg, spp)
    st = compare_records(records_host(s), rec_o, f"K {K}")
    assert st["guided"] > 0 or frame == 0
    say(f"  kept {int(both.sum())}, resets {int(reset_g.sum())}, {st}")


# ------------------------------------------------------------------ EM update
def _records(scene, p, spp, view):
    """Records of a new model (BRDF draws only) and their radiance."""
    s = pg.Samples(spp, scene["height"], scene["width"])
    g0 = pg.new_gamma(scene["height"], scene["width"])
    pg.reproject_sample(p, view, None, None, g0, s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), view, dev(scene["vis"]), s)
    return s


@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("W,H,spp", [(83, 45, 1), (67, 29, 2), (40, 37, 5)])
@pytest.mark.parametrize("kreg", ["new", "random", "saturated"])
def test_em_parity_same_input(K, W, H, spp, kreg):
    say(f"case: lobes em K {K} {W}x{H} spp {spp} {kreg}")
    seed = 13000 + 17 * K + W + 7 * H + spp
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    p, P = _p(seed, 6)
    if kreg == "new":
        g = O.reproject_k(P, K, O.OView(scene), None, None)[0].astype(np.float32)
    else:
        g = random_lobes(K, H, W, rng, k_lo=0)
        if kreg == "saturated":
            g[6 * K + 1] = 16
    view = gpu_view(scene)
    s = _records(scene, pg.params(seed, frame=0), spp, view)
    gt = dev(g)
    pg.em_update_lobes(p, K, view, s, gt)
    torch.cuda.synchronize()
    g_o, stats = O.em_k(P, K, O.OView(scene), records_host(s), g, with_stats=True)
    gg = host(gt)
    uf = lobes_underflow(stats)
    assert (gg[6 * K + 1] == g_o[6 * K + 1]).all()
    out = []
    for j, (a, b) in enumerate(zip(lobe_slices(gg, K), lobe_slices(g_o, K))):
        if kreg == "new":
            out.append(assert_gamma_close(a, b, TOL_EM_FRAME, mask=~uf, what=f"lobe {j}"))
        else:
            out.append(assert_gamma_quantile(a, b, TOL_EM_FRAME, TOL_EM_RUN, mask=~uf, what=f"lobe {j}"))
    assert np.isfinite(gg).all()
    trained = stats[0] > 0
    tot = sum(gg[6 * j + 5] for j in range(K))
    assert (tot[trained] <= np.float32(0.95) * (1 + 1e-6)).all() and (tot[trained] >= np.float32(0.05) * (1 - 1e-6)).all()
    say(f"  trained {int(trained.sum())}, underflow {int(uf.sum())}, worst {out[0]}")


def test_em_parity_without_clamp():
    K, W, H, spp, seed = 2, 71, 33, 2, 13500
    say("case: lobes em without the clamp")
    scene = wl.make_scene(W, H, seed)
    p, P = _p(seed, 4, flags=pg.PG_NO_CLAMP)
    g = random_lobes(K, H, W, np.random.default_rng(seed), k_lo=0)
    view = gpu_view(scene)
    s = _records(scene, pg.params(seed, frame=0), spp, view)
    gt = dev(g)
    pg.em_update_lobes(p, K, view, s, gt)
    torch.cuda.synchronize()
    g_o, stats = O.em_k(P, K, O.OView(scene), records_host(s), g, with_stats=True)
    gg = host(gt)
    uf = lobes_underflow(stats)
    for j, (a, b) in enumerate(zip(lobe_slices(gg, K), lobe_slices(g_o, K))):
        assert_gamma_quantile(a, b, TOL_EM_FRAME, TOL_EM_RUN, mask=~uf, what=f"lobe {j}")


@pytest.mark.parametrize("K", [2, 3])
def test_pdf_parity(K):
    W, H, n, seed = 77, 39, 3, 13600 + K
    say(f"case: lobes pdf K {K}")
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    g = random_lobes(K, H, W, rng, k_lo=0)
    d = rng.normal(size=(3, n, H, W)).astype(np.float32)
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    d[:, 0, 0, 0] = 0
    p, P = _p(seed, 2)
    D = host(pg.pdf_lobes(p, K, gpu_view(scene), dev(g), dev(d)))
    Do = O.pdf_k(P, K, O.OView(scene), g, d)
    r = rel_err(D, Do)
    pos = Do > 0
    assert (D[~pos] == 0).all()
    assert np.quantile(r[pos], 0.999) <= TOL_PDF and r[pos].max() <= 1e-3, (np.quantile(r[pos], 0.999), r.max())


@pytest.mark.parametrize("spp", [2, 4])
def test_one_lobe_matches_the_single_lobe_kernels(spp):
    """K = 1 through the K-lobe kernels against the single-lobe kernels on the
    same inputs: the same reprojected state, strategies and directions bit
    for bit, densities within 1e-5 (99.9%; the single-lobe kernel takes each
    strategy's density in its sample space), and after the update the same
    epochs and every channel within 1e-6 at spp 2 (mu and pi absolute, Sigma
    relative to its trace, W relative: the two kernels are contracted into
    fused multiply-adds in different places, and the weight clamp is a
    scaling).  From spp 4 the single-lobe kernel visits the samples of the
    last half of the sample planes after those of the first (its two-pass
    tile) while the K-lobe kernel keeps the training set's order, so the FP32
    sums round differently: within the one-step tolerance TOL_EM_FRAME."""
    W, H, seed = 93, 50, 13700 + spp
    say(f"case: K = 1 against the single-lobe kernels, spp {spp}")
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    g_prev = random_lobes(1, H, W, rng, k_lo=0)
    mv, mask = wl.make_motion(W, H, seed, 2)
    p = pg.params(seed, frame=2)
    cur, prev = gpu_view(scene, dev(mv), dev(mask)), gpu_view(scene)
    gp = dev(g_prev)
    a_g, b_g = torch.empty_like(gp), torch.empty_like(gp)
    a_s, b_s = pg.Samples(spp, H, W), pg.Samples(spp, H, W)
    pg.reproject_sample(p, cur, prev, gp, a_g, a_s)
    pg.reproject_sample_lobes(p, 1, cur, prev, gp, b_g, b_s)
    lt = pg.lights_struct(scene["lights"], float(scene["ambient"]))
    pg.light_field(lt, cur, dev(scene["vis"]), a_s)
    pg.light_field(lt, cur, dev(scene["vis"]), b_s)
    torch.cuda.synchronize()
    assert torch.equal(a_g.view(torch.int32), b_g.view(torch.int32))
    assert torch.equal(a_s.strategy, b_s.strategy)
    assert torch.equal(a_s.dir.view(torch.int32), b_s.dir.view(torch.int32))
    live = (a_s.strategy == 1) | (a_s.strategy == 2)
    r = rel_err(host(b_s.pdf_mix)[host(live)], host(a_s.pdf_mix)[host(live)])
    assert np.quantile(r, 0.999) <= 1e-5 and r.max() <= 1e-3, (np.quantile(r, 0.999), r.max())
    pg.em_update(p, cur, a_s, a_g)
    pg.em_update_lobes(p, 1, cur, a_s, b_g)
    torch.cuda.synchronize()
    ga, gb = host(a_g), host(b_g)
    e = assert_gamma_close(gb, ga, 1e-6 if spp < 4 else TOL_EM_FRAME, what="K = 1 against the single lobe")
    say(f"  after the update: {e}")


# ------------------------------------------------------------ teacher-forced run
def test_run_teacher_forced_pan():
    """Six frames of a moving sequence at K = 2: each frame the oracle steps
    from the GPU's previous state and uses the GPU's records for its update."""
    K, W, H, spp, seed = 2, 93, 57, 2, 13800
    say("case: lobes run 93x57 spp2 pan, K 2")
    seq = wl.Sequence(W, H, seed)
    fr = seq.frame(0)
    guide = pg.LobesGuide(W, H, fr["lights"], float(fr["ambient"]), lobes=K, spp=spp, seed=seed)
    v_prev = None
    prev = None
    worst = {}
    for t in range(6):
        if t:
            fr = seq.frame(t)
        cur = pg.DeviceFrame(fr)
        g_in = host(guide.state).copy()
        guide.step(cur, prev, frame=t)
        torch.cuda.synchronize()
        prev = cur
        P = O.params(seed, frame=t)
        v = O.OView(fr, fr["motion"], fr["disocc"])
        g1, src = O.reproject_k(P, K, v, v_prev if v_prev is not None else v, g_in if t else None)
        rec = records_host(guide.samples)
        # the oracle samples the state it reprojected (FP64): decisions near
        # a threshold may differ, which the margins cover
        ro = O.sample_k(P, K, v, g1, spp)
        st = compare_records(rec, ro, f"frame {t}")
        g2, stats = O.em_k(P, K, v, rec, g1, with_stats=True)
        uf = lobes_underflow(stats)
        for j, (a, b) in enumerate(zip(lobe_slices(host(guide.state), K), lobe_slices(g2, K))):
            e = assert_gamma_close(a, b, TOL_EM_FRAME, mask=~uf, what=f"frame {t} lobe {j}")
            for k_, v_ in e.items():
                worst[k_] = max(worst.get(k_, 0.0), v_)
        say(f"  frame {t}: {st}")
        v_prev = v
    say(f"  teacher-forced worst {worst}")


# ------------------------------------------------------------ full size, sampled
def test_1080p_pan_k2_sampled_pixels():
    """The 1080p pan at K = 2, 1 spp, through LobesGuide (the launches the
    bench times) for 6 frames; on frame 5 the reprojection, the records and
    the update of 32 crops of 16x16 pixels are recomputed by the oracle from
    the GPU's inputs."""
    K, W, H, spp = 2, 1920, 1080, 1
    cfg = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]
    seed = cfg["seed"]
    say("case: 1080p pan K 2, sampled crops")
    seq = wl.Sequence(W, H, seed)
    fr = seq.frame(0)
    guide = pg.LobesGuide(W, H, fr["lights"], float(fr["ambient"]), lobes=K, spp=spp, seed=seed)
    prev = None
    T = 6
    for t in range(T):
        if t:
            fr_prev = fr
            fr = seq.frame(t)
        cur = pg.DeviceFrame(fr)
        if t == T - 1:
            g_in = host(guide.state).copy()
            # reprojection + sampling alone, then the update
            p = guide.params(t)
            g_out = guide.gamma[1 - guide.cur]
            pg.reproject_sample_lobes(p, K, cur.view, prev.view, guide.state, g_out, guide.samples)
            pg.light_field(guide.lights, cur.view, cur.vis, guide.samples)
            torch.cuda.synchronize()
            g_rs = host(g_out).copy()
            pg.em_update_lobes(p, K, cur.view, guide.samples, g_out)
            torch.cuda.synchronize()
            g_em = host(g_out)
            rec = records_host(guide.samples)
        else:
            guide.step(cur, prev, frame=t)
        prev = cur
    P = O.params(seed, frame=T - 1)
    v = O.OView(fr, fr["motion"], fr["disocc"])
    g_in, g_rs = g_in.astype(np.float64), g_rs.astype(np.float64)
    rec = {k_: (a.astype(np.float64) if a.dtype == np.float32 else a) for k_, a in rec.items()}
    vp = O.OView(fr_prev)
    rng = np.random.default_rng(seed)
    worst = {}
    for c in range(32):
        x0, y0 = int(rng.integers(0, W - 16)), int(rng.integers(0, H - 16))
        rect = (x0, y0, x0 + 16, y0 + 16)
        sl = (slice(None), slice(y0, y0 + 16), slice(x0, x0 + 16))
        g1, src = O.reproject_k(P, K, v, vp, g_in, rect=rect)
        near = (rim_margin(g1[sl], K) < 1e-4) | (rim_margin(g_rs[sl], K) < 1e-4)
        reset_g = _is_reset(g_rs[sl].astype(np.float32), K, P)
        assert ((reset_g != (src[sl[1:]] >= 0)) | near).all()
        ok = ~reset_g & (src[sl[1:]] >= 0)
        for j in range(K):
            assert np.abs(g_rs[sl][6 * j:6 * j + 2][:, ok] - g1[sl][6 * j:6 * j + 2][:, ok]).max(initial=0) <= TOL_DIR
        ro = O.sample_k(P, K, v, g_rs, spp, rect=rect)
        rsub = {k_: a[..., y0:y0 + 16, x0:x0 + 16] for k_, a in rec.items()}
        osub = {k_: a[..., y0:y0 + 16, x0:x0 + 16] for k_, a in ro.items()}
        compare_records(rsub, osub, f"crop {c}")
        g2, stats = O.em_k(P, K, v, rec, g_rs, rect=rect, with_stats=True)
        uf = lobes_underflow(stats[sl])
        for j, (a, b) in enumerate(zip(lobe_slices(g_em[sl], K), lobe_slices(g2[sl], K))):
            e = assert_gamma_close(a, b, TOL_EM_FRAME, mask=~uf, what=f"crop {c} lobe {j}")
            for k_, v_ in e.items():
                worst[k_] = max(worst.get(k_, 0.0), v_)
    say(f"  32 crops of frame {T - 1}: worst {worst}")


# ----------------------------------------------------------------- what it is for
def _lobes_study(all_visible):
    cfg = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]
    W, H, seed, frames = 1920, 1080, cfg["seed"], 24
    evals = (4, 8, 16, 23)  # errors compared over frames 8, 16 and 23
    n_px, n_ref = 32768, 1024
    say(f"case: lobes study, 1080p pan, {n_px} px, {'every light visible' if all_visible else 'visibility coins'}")
    seq = wl.Sequence(W, H, seed)

    def frame(t):
        fr = seq.frame(t)
        if all_visible:
            fr["vis"] = np.full_like(fr["vis"], 7)
        return fr
    fr = frame(0)
    amb = float(fr["ambient"])
    runs = {1: pg.Guide(W, H, fr["lights"], amb, spp=1, seed=seed),
            2: pg.LobesGuide(W, H, fr["lights"], amb, lobes=2, spp=1, seed=seed),
            3: pg.LobesGuide(W, H, fr["lights"], amb, lobes=3, spp=1, seed=seed)}
    rng = np.random.default_rng(seed + 2)
    prev = None
    rows = []
    errs = {k: [] for k in runs}
    for t in range(frames):
        if t:
            fr = frame(t)
        cur = pg.DeviceFrame(fr)
        for g in runs.values():
            g.step(cur, prev, frame=t)
        prev = cur
        if t not in evals:
            continue
        est = {k: host(pg.estimate(g.params(t), cur.view, g.samples)) for k, g in runs.items()}
        torch.cuda.synchronize()
        valid = (np.einsum("chw,chw->hw", fr["normal"], fr["view_dir"]) > 0) & (fr["roughness"] >= 0.1)
        px = np.sort(rng.choice(np.flatnonzero(valid.reshape(-1)), size=n_px, replace=False))
        ref, se = O.reference(O.params(seed, frame=t), O.OView(fr), fr["lights"], amb, fr["vis"], px, n_ref)
        r2 = float((ref ** 2).sum())
        mse = {k: float(((e.reshape(-1)[px] - ref) ** 2).sum()) / r2 for k, e in est.items()}
        rows.append((t, mse))
        if t != evals[0]:
            for k, e in est.items():
                errs[k].append((e.reshape(-1)[px] - ref) ** 2 / r2)
        say(f"  frame {t:2d}: rel. MSE " + ", ".join(f"K={k} {v:.4f}" for k, v in mse.items()))
    mean = {k: float(np.mean([r[1][k] for r in rows[1:]])) for k in runs}
    say(f"  mean rel. MSE over frames {evals[1:]}: " + ", ".join(f"K={k} {v:.4f}" for k, v in mean.items()))
    ci = {}
    for k in (2, 3):
        ci[k] = paired_ratio_ci(np.concatenate(errs[k]), np.concatenate(errs[1]))
        say(f"  K = {k} / K = 1 MSE: {ci[k][0]:.3f}, paired bootstrap 95% [{ci[k][1]:.3f}, {ci[k][2]:.3f}]")
    assert all(np.isfinite(v) for r in rows for v in r[1].values())
    return mean, ci


def test_lobes_study_1080p_pan():
    """What more lobes buy on the 1080p pan (three spherical-Gaussian lights,
    per-pixel visibility coins, 1 spp): the relative MSE of the first-bounce
    estimate against the FP64 reference (1024 samples per pixel) on 32768
    pixels at a few frames, for K = 1 (the single-lobe kernels), 2 and 3, with
    paired bootstrap intervals (reported: no effect on this field, whose
    neighbours see other lights than the pixel; the guard is that K lobes
    never cost more than 10% over one)."""
    mean, ci = _lobes_study(all_visible=False)
    assert mean[2] <= 1.1 * mean[1] and mean[3] <= 1.1 * mean[1], mean


def test_lobes_study_every_light_visible():
    """The same with every light visible from every pixel, so that each
    pixel's incident radiance has up to three stable lobes (the case a single
    Gaussian cannot fit): the MSE ratios of K = 2 and 3 against one lobe lie
    below one (by 1.5-3%, at the edge of their paired intervals)."""
    mean, ci = _lobes_study(all_visible=True)
    assert ci[3][0] < 1.0 and ci[2][0] < 1.0, ci

# ------------------------------------------------------------------ edge cases
@pytest.mark.parametrize("K,W,H,spp", [(2, 1, 1, 1), (3, 70, 1, 2), (2, 1, 37, 3), (4, 45, 13, 8), (1, 33, 9, 8)])
def test_degenerate_shapes_and_largest_lds(K, W, H, spp):
    """1x1, one row, one column, and spp 8 at K = 4 (the largest LDS request
    of the training kernel): reprojection + sampling and the update against
    the oracle, a NaN history resetting, and the positional variant with
    finite hit distances."""
    say(f"case: lobes edge K {K} {W}x{H} spp {spp}")
    seed = 15000 + K + W + H + spp
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    g_prev = random_lobes(K, H, W, rng, k_lo=1)
    g_prev[0, 0, 0] = np.nan
    mv, mask = wl.make_motion(W, H, seed, 2)
    p, P = _p(seed, 2)
    cur, prev = gpu_view(scene, dev(mv), dev(mask)), gpu_view(scene)
    go = torch.empty_like(dev(g_prev))
    s = pg.Samples(spp, H, W)
    pg.reproject_sample_lobes(p, K, cur, prev, dev(g_prev), go, s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), cur, dev(scene["vis"]), s)
    torch.cuda.synchronize()
    gg = host(go)
    vo = O.OView(scene, mv, mask)
    g_o, src_o = O.reproject_k(P, K, vo, O.OView(scene), g_prev)
    assert np.isfinite(gg).all()
    both = (src_o >= 0) & ~_is_reset(gg, K, P)
    for j in range(K):
        assert np.abs(gg[6 * j:6 * j + 2, both] - g_o[6 * j:6 * j + 2, both]).max(initial=0) <= TOL_DIR
    compare_records(records_host(s), O.sample_k(P, K, vo, gg, spp), f"K {K} {W}x{H}")
    g_in = gg.copy()
    gt = dev(g_in)
    pg.em_update_lobes(p, K, cur, s, gt)
    torch.cuda.synchronize()
    g_e, stats = O.em_k(P, K, vo, records_host(s), g_in, with_stats=True)
    for j, (a, b) in enumerate(zip(lobe_slices(host(gt), K), lobe_slices(g_e, K))):
        assert_gamma_quantile(a, b, TOL_EM_FRAME, TOL_EM_RUN, mask=~lobes_underflow(stats), what=f"lobe {j}")
    # positional reuse on a flat grid of positions with finite hit distances
    pos = np.stack(list(np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)) + [np.zeros((H, W))]).astype(np.float32)
    hit = rng.uniform(5.0, 50.0, (spp, H, W)).astype(np.float32)
    gv = dev(g_in)
    pg.em_update_vpl(p, K, cur, dev(pos), s, dev(hit), gv)
    torch.cuda.synchronize()
    rec = records_host(s)
    rec["hit_dist"] = hit
    g_v, stats = O.em_vpl(P, K, vo, pos, rec, g_in, with_stats=True)
    for j, (a, b) in enumerate(zip(lobe_slices(host(gv), K), lobe_slices(g_v, K))):
        assert_gamma_quantile(a, b, TOL_EM_FRAME, TOL_EM_RUN, mask=~lobes_underflow(stats), what=f"vpl lobe {j}")
