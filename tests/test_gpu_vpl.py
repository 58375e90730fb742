"""Positional reuse of virtual point lights on the GPU (pg_em_update_vpl) and
its near-field stand-in for the trace (pg_light_ceiling), against the
oracle's orc_em_vpl and orc_light_ceiling through the C ABI; then what the
reuse is for, on the 1080p pan under the ceiling."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import (paired_ratio_ci, TOL_EM_FRAME, TOL_EM_RUN, EVIDENCE_FLOOR, assert_gamma_close, assert_gamma_quantile, dev, host,
                    records_host, rel_err)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def lobe_slices(g, K):
    return [np.concatenate([g[6 * j:6 * j + 6], g[6 * K:6 * K + 2]]) for j in range(K)]


def lobes_underflow(stats):
    B0 = np.maximum(stats[0], 1e-300)
    return ((stats[1:] > 0) & (stats[1:] < EVIDENCE_FLOOR * B0)).any(0)


def random_lobes(K, H, W, rng, k_lo=0, k_hi=16):
    planes = []
    for _ in range(K):
        sxx = rng.uniform(0.0005, 0.03, (H, W))
        syy = rng.uniform(0.0005, 0.03, (H, W))
        rho = rng.uniform(-0.8, 0.8, (H, W))
        planes += [rng.uniform(0.05, 0.95, (H, W)), rng.uniform(0.05, 0.95, (H, W)), sxx,
                   rho * np.sqrt(sxx * syy), syy, rng.uniform(0.05, 0.95, (H, W)) / K]
    planes += [rng.uniform(0.0, 20.0, (H, W)), rng.integers(k_lo, k_hi + 1, (H, W))]
    return np.stack(planes).astype(np.float32)


def _frame_records(W, H, spp, seed, K=1, frame=2):
    """A pan frame under the ceiling: records sampled by the K-lobe kernels
    from a random trained state (guided and BRDF draws), radiance and hit
    distances from the GPU's ceiling stand-in."""
    seq = wl.Sequence(W, H, seed)
    fr = seq.frame(0)
    cur = pg.DeviceFrame(fr)
    ceil = pg.Ceiling(fr["ceiling"])
    g = random_lobes(K, H, W, np.random.default_rng(seed), k_lo=1)
    s = pg.Samples(spp, H, W)
    gout = torch.empty_like(dev(g))
    p = pg.params(seed, frame=frame)
    pg.reproject_sample_lobes(p, K, cur.view, cur.view, dev(g), gout, s)
    hit = torch.empty((spp, H, W), dtype=torch.float32, device="cuda")
    pg.light_ceiling(ceil, cur.view, cur.position, s, hit)
    torch.cuda.synchronize()
    return fr, cur, s, hit, host(gout)


@pytest.mark.parametrize("W,H,spp", [(83, 45, 2), (64, 33, 5)])
def test_light_ceiling_parity(W, H, spp):
    say(f"case: ceiling light field {W}x{H} spp {spp}")
    seed = 14000 + W + spp
    fr, cur, s, hit, _ = _frame_records(W, H, spp, seed)
    rec = records_host(s)
    L_o, t_o = O.light_ceiling(fr["ceiling"], O.OView(fr), fr["position"], rec["dir"], rec["strategy"])
    L_g, t_g = rec["radiance"], host(hit)
    live = (rec["strategy"] == 1) | (rec["strategy"] == 2)
    esc_o, esc_g = np.isinf(t_o), np.isinf(t_g)
    # rising or not is decided on the normalised direction's z in each precision
    wz = rec["dir"][2] / np.sqrt((rec["dir"].astype(np.float64) ** 2).sum(0))
    near = np.abs(wz) < 1e-6
    assert not ((esc_o != esc_g) & live & ~near).any()
    hit_live = live & ~esc_o & ~esc_g
    assert rel_err(t_g[hit_live], t_o[hit_live]).max(initial=0) <= 1e-5
    # E is evaluated at y = x + t w, whose FP32 rounding (~|y| 2^-24) is
    # amplified near a lamp's edge by |grad log E| <= 3/r
    r = rel_err(L_g[live & (esc_o == esc_g)], L_o[live & (esc_o == esc_g)])
    assert np.quantile(r, 0.999) <= 1e-4 and r.max() <= 1e-3, (np.quantile(r, 0.999), r.max())
    assert (L_g[~live] == 0).all() and (t_g[~live] == 0).all()
    say(f"  live {int(live.sum())}, escaping {int((esc_g & live).sum())}, L q999 {np.quantile(r, 0.999):.2e} "
        f"max {r.max():.2e}")


@pytest.mark.parametrize("K", [1, 2])
@pytest.mark.parametrize("W,H,spp", [(83, 45, 1), (67, 29, 2), (40, 37, 5)])
def test_em_vpl_parity(K, W, H, spp):
    say(f"case: em vpl K {K} {W}x{H} spp {spp}")
    seed = 14100 + 13 * K + W + spp
    fr, cur, s, hit, g = _frame_records(W, H, spp, seed, K=K)
    p, P = pg.params(seed, frame=5), O.params(seed, frame=5)
    gt = dev(g)
    pg.em_update_vpl(p, K, cur.view, cur.position, s, hit, gt)
    torch.cuda.synchronize()
    rec = records_host(s)
    rec["hit_dist"] = host(hit)
    g_o, stats = O.em_vpl(P, K, O.OView(fr), fr["position"], rec, g, with_stats=True)
    gg = host(gt)
    uf = lobes_underflow(stats)
    assert (gg[6 * K + 1] == g_o[6 * K + 1]).all()
    out = [assert_gamma_quantile(a, b, TOL_EM_FRAME, TOL_EM_RUN, mask=~uf, what=f"lobe {j}")
           for j, (a, b) in enumerate(zip(lobe_slices(gg, K), lobe_slices(g_o, K)))]
    # the re-derived directions changed the update (against the directional one)
    g_d = O.em_k(P, K, O.OView(fr), rec, g)
    moved = np.abs(g_o[:2] - g_d[:2]).max(0)
    assert (moved > 1e-4).mean() > 0.2
    say(f"  trained {int((stats[0] > 0).sum())}, underflow {int(uf.sum())}, worst lobe 0 {out[0]}; "
        f"pixels moved by positional reuse {float((moved > 1e-4).mean()):.2f}")


def test_infinite_hit_distances_give_the_lobes_update():
    W, H, spp, K, seed = 77, 41, 2, 2, 14200
    say("case: em vpl with every hit distance +inf")
    fr, cur, s, hit, g = _frame_records(W, H, spp, seed, K=K)
    hit.fill_(float("inf"))
    p = pg.params(seed, frame=5)
    a, b = dev(g), dev(g)
    pg.em_update_vpl(p, K, cur.view, cur.position, s, hit, a)
    pg.em_update_lobes(p, K, cur.view, s, b)
    torch.cuda.synchronize()
    e = assert_gamma_close(host(a), host(b), 1e-6, what="+inf hit distances")
    say(f"  {e}; bit-identical: {bool(torch.equal(a.view(torch.int32), b.view(torch.int32)))}")


def test_run_teacher_forced_pan_under_the_ceiling():
    """Six frames at K = 1 with positional reuse under the ceiling; each frame
    the oracle's update runs on the GPU's reprojected state and records."""
    W, H, spp, K, seed = 93, 57, 1, 1, 14300
    say("case: vpl run 93x57 pan")
    seq = wl.Sequence(W, H, seed)
    fr = seq.frame(0)
    ceil = pg.Ceiling(fr["ceiling"])
    s = pg.Samples(spp, H, W)
    hit = torch.empty((spp, H, W), dtype=torch.float32, device="cuda")
    gam = [pg.new_lobes_gamma(K, H, W), pg.new_lobes_gamma(K, H, W)]
    prev = None
    worst = {}
    for t in range(6):
        if t:
            fr = seq.frame(t)
        cur = pg.DeviceFrame(fr)
        p = pg.params(seed, frame=t)
        g_in, g_out = gam[t % 2], gam[1 - t % 2]
        pg.reproject_sample_lobes(p, K, cur.view, prev.view if t else None, g_in if t else None, g_out, s)
        pg.light_ceiling(ceil, cur.view, cur.position, s, hit)
        torch.cuda.synchronize()
        g_rs = host(g_out).copy()
        pg.em_update_vpl(p, K, cur.view, cur.position, s, hit, g_out)
        torch.cuda.synchronize()
        rec = records_host(s)
        rec["hit_dist"] = host(hit)
        g_o, stats = O.em_vpl(O.params(seed, frame=t), K, O.OView(fr), fr["position"], rec, g_rs, with_stats=True)
        e = assert_gamma_close(host(g_out), g_o, TOL_EM_FRAME, mask=~lobes_underflow(stats), what=f"frame {t}")
        for k_, v_ in e.items():
            worst[k_] = max(worst.get(k_, 0.0), v_)
        prev = cur
    say(f"  teacher-forced worst {worst}")


def test_vpl_study_1080p_pan_under_the_ceiling():
    """What positional reuse buys: the 1080p pan lit by the ceiling's lamps
    (1 spp, one lobe), trained with the neighbours' directions reused as they
    are (every hit distance +inf) and with positional reuse; relative MSE of
    the first-bounce estimate against the FP64 reference (2048 BRDF draws per
    pixel) on 32768 guided pixels at frames 8, 16 and 23 (reported; the guard is
    that positional reuse never costs more than 10%)."""
    cfg = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]
    W, H, seed, frames, K = 1920, 1080, cfg["seed"], 24, 1
    evals = (8, 16, 23)
    n_px, n_ref = 32768, 2048
    say(f"case: vpl study, 1080p pan under the ceiling, {n_px} px")
    seq = wl.Sequence(W, H, seed)
    fr = seq.frame(0)
    ceil = pg.Ceiling(fr["ceiling"])
    runs = {m: dict(g=[pg.new_lobes_gamma(K, H, W), pg.new_lobes_gamma(K, H, W)], s=pg.Samples(1, H, W),
                    hit=torch.empty((1, H, W), dtype=torch.float32, device="cuda")) for m in ("dir", "pos")}
    inf_hit = torch.full((1, H, W), float("inf"), device="cuda")
    rng = np.random.default_rng(seed + 3)
    prev = None
    rows = []
    errs = {m: [] for m in runs}
    for t in range(frames):
        if t:
            fr = seq.frame(t)
        cur = pg.DeviceFrame(fr)
        p = pg.params(seed, frame=t)
        for m, r in runs.items():
            g_in, g_out = r["g"][t % 2], r["g"][1 - t % 2]
            pg.reproject_sample_lobes(p, K, cur.view, prev.view if t else None, g_in if t else None, g_out, r["s"])
            pg.light_ceiling(ceil, cur.view, cur.position, r["s"], r["hit"])
            if m == "pos":
                pg.em_update_vpl(p, K, cur.view, cur.position, r["s"], r["hit"], g_out)
            else:
                pg.em_update_vpl(p, K, cur.view, cur.position, r["s"], inf_hit, g_out)
        prev = cur
        if t not in evals:
            continue
        est = {m: host(pg.estimate(p, cur.view, r["s"])) for m, r in runs.items()}
        torch.cuda.synchronize()
        valid = (np.einsum("chw,chw->hw", fr["normal"], fr["view_dir"]) > 0) & (fr["roughness"] >= 0.1)
        px = np.sort(rng.choice(np.flatnonzero(valid.reshape(-1)), size=n_px, replace=False))
        ref, se = O.reference_ceiling(O.params(seed, frame=t), O.OView(fr), fr["position"], fr["ceiling"], px, n_ref)
        r2 = float((ref ** 2).sum())
        mse = {m: float(((e.reshape(-1)[px] - ref) ** 2).sum()) / r2 for m, e in est.items()}
        rows.append(mse)
        for m, e in est.items():
            errs[m].append((e.reshape(-1)[px] - ref) ** 2 / r2)
        say(f"  frame {t:2d}: rel. MSE, directions reused {mse['dir']:.4f}, positions reused {mse['pos']:.4f} "
            f"(reference rel. s.e. {float(np.median(se / np.maximum(ref, 1e-30))):.4f})")
    mean = {m: float(np.mean([r[m] for r in rows])) for m in runs}
    say(f"  mean rel. MSE: directions reused {mean['dir']:.4f}, positions reused {mean['pos']:.4f}")
    rr, lo, hi = paired_ratio_ci(np.concatenate(errs["pos"]), np.concatenate(errs["dir"]))
    say(f"  positions / directions reused MSE: {rr:.3f}, paired bootstrap 95% [{lo:.3f}, {hi:.3f}]")
    assert all(np.isfinite(v) for r in rows for v in r.values())
    assert mean["pos"] <= 1.1 * mean["dir"], mean


def test_1080p_pan_vpl_sampled_crops():
    """The 1080p pan under the ceiling with positional reuse (one lobe, the
    launches bench.py --vpl times) for 6 frames; on frame 5 the ceiling
    field and the update of 32 crops of 16x16 pixels are recomputed by the
    oracle from the GPU's inputs."""
    W, H, spp, K = 1920, 1080, 1, 1
    seed = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]["seed"]
    say("case: 1080p pan under the ceiling, positional reuse, sampled crops")
    seq = wl.Sequence(W, H, seed)
    fr = seq.frame(0)
    ceil = pg.Ceiling(fr["ceiling"])
    s = pg.Samples(spp, H, W)
    hit = torch.empty((spp, H, W), dtype=torch.float32, device="cuda")
    gam = [pg.new_lobes_gamma(K, H, W), pg.new_lobes_gamma(K, H, W)]
    prev = None
    T = 6
    for t in range(T):
        if t:
            fr = seq.frame(t)
        cur = pg.DeviceFrame(fr)
        p = pg.params(seed, frame=t)
        g_in, g_out = gam[t % 2], gam[1 - t % 2]
        pg.reproject_sample_lobes(p, K, cur.view, prev.view if t else None, g_in if t else None, g_out, s)
        pg.light_ceiling(ceil, cur.view, cur.position, s, hit)
        if t == T - 1:
            torch.cuda.synchronize()
            g_rs = host(g_out).astype(np.float64)
        pg.em_update_vpl(p, K, cur.view, cur.position, s, hit, g_out)
        prev = cur
    torch.cuda.synchronize()
    g_em = host(gam[T % 2])
    rec = {k_: (a.astype(np.float64) if a.dtype == np.float32 else a) for k_, a in records_host(s).items()}
    rec["hit_dist"] = host(hit).astype(np.float64)
    P = O.params(seed, frame=T - 1)
    v = O.OView(fr, fr["motion"], fr["disocc"])
    rng = np.random.default_rng(seed + 5)
    worst = {}
    for c in range(32):
        x0, y0 = int(rng.integers(0, W - 16)), int(rng.integers(0, H - 16))
        rect = (x0, y0, x0 + 16, y0 + 16)
        sl = (slice(None), slice(y0, y0 + 16), slice(x0, x0 + 16))
        L_o, t_o = O.light_ceiling(fr["ceiling"], v, fr["position"], rec["dir"], rec["strategy"], rect=rect)
        live = ((rec["strategy"] == 1) | (rec["strategy"] == 2))[sl]
        fin = live & np.isfinite(t_o[sl]) & np.isfinite(rec["hit_dist"][sl])
        assert rel_err(rec["hit_dist"][sl][fin], t_o[sl][fin]).max(initial=0) <= 1e-5
        assert rel_err(rec["radiance"][sl][live], L_o[sl][live]).max(initial=0) <= 1e-3
        g2, stats = O.em_vpl(P, K, v, fr["position"], rec, g_rs, rect=rect, with_stats=True)
        e = assert_gamma_close(g_em[sl], g2[sl], TOL_EM_FRAME, mask=~lobes_underflow(stats[sl]), what=f"crop {c}")
        for k_, v_ in e.items():
            worst[k_] = max(worst.get(k_, 0.0), v_)
    say(f"  32 crops of frame {T - 1}: worst {worst}")
