"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Same-input checks per call, teacher-forced checks per frame (the oracle steps
from the GPU's state), and free-running multi-frame runs.  Integer outputs
(RNG words, source addresses, reset flags, strategy codes away from their
thresholds, epochs) must match exactly; floating-point outputs within the
tolerances of tests/pgtest.py.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import (MARGIN, TOL_DIR, TOL_EM_FRAME, TOL_EM_RUN, TOL_PDF, GpuFrames, assert_gamma_close,
                    assert_gamma_quantile,
                    compare_samples, conditioning, dev, gamma_errors, gpu_view, host, pdf_bounds,
                    random_gamma, records_host, rel_err, underflow_mask)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SHAPES = [(64, 64), (67, 45), (1, 1), (70, 1), (1, 37), (131, 29)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _p(seed, frame, **kw):
    return pg.params(seed, frame=frame, **kw), O.params(seed, frame=frame, **kw)


# --------------------------------------------------------------------- RNG
def test_philox_words_match_oracle():
    say("case: philox words")
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(4000, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x1234567890ABCDEF
    out = host(pg.philox(dev(ctr.view(np.int32)), seed)).view(np.uint32)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint64).astype(np.uint32)
    ref = np.stack([O.philox(c, key) for c in ctr])
    assert (out == ref).all()


# ------------------------------------------------------------- reprojection
@pytest.mark.parametrize("W,H", SHAPES)
@pytest.mark.parametrize("frame", [0, 3])
def test_reproject_parity(W, H, frame):
    say(f"case: reproject {W}x{H} frame {frame}")
    seed = 1000 + W + H
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    g_prev = random_gamma(H, W, rng, k_lo=0)
    g_prev[5, 0, 0] = np.nan if W * H > 4 else g_prev[5, 0, 0]
    mv, mask = wl.make_motion(W, H, seed, frame)
    p, P = _p(seed, frame)
    cur, prev = gpu_view(scene, dev(mv), dev(mask)), gpu_view(scene)
    gp = dev(g_prev)
    go = torch.empty_like(gp)
    src = torch.empty((H, W), dtype=torch.int32, device="cuda")
    pg.reproject(p, cur, prev if frame else None, gp if frame else None, go, src)
    torch.cuda.synchronize()
    g_o, src_o = O.reproject(P, O.OView(scene, mv, mask), O.OView(scene), g_prev)
    src_g = host(src)
    assert (src_g == src_o).all(), np.argwhere(src_g != src_o)[:5]
    gg = host(go)
    kept = src_o >= 0
    if frame == 0:
        assert not kept.any()
    qy, qx = np.divmod(src_o[kept], W)
    # copied channels are carried over bit for bit
    assert (gg[2:, kept] == g_prev[2:, qy, qx]).all()
    e = gamma_errors(gg, g_o)
    assert e["mu"].max() <= TOL_DIR, e["mu"].max()
    assert np.abs(gg[:, ~kept] - g_o[:, ~kept]).max(initial=0) <= 1e-7


def test_reproject_static_identity():
    """Zero motion and one G-buffer: Gamma' = Gamma bit for bit."""
    say("case: reproject static identity")
    W, H, seed = 64, 64, wl.SEED_BASE + 1
    scene = wl.make_scene(W, H, seed)
    g_prev = random_gamma(H, W, np.random.default_rng(2))
    p, _ = _p(seed, 5)
    view = gpu_view(scene)
    gp = dev(g_prev)
    go = torch.empty_like(gp)
    pg.reproject(p, view, view, gp, go)
    torch.cuda.synchronize()
    guided = scene["roughness"] >= np.float32(0.1)
    assert (host(go)[:, guided] == g_prev[:, guided]).all()


# ----------------------------------------------------------------- sampling
@pytest.mark.parametrize("W,H", SHAPES)
@pytest.mark.parametrize("spp", [1, 3, 8])
def test_sample_parity(W, H, spp):
    say(f"case: sample {W}x{H} spp {spp}")
    seed = 2000 + W * 3 + H + spp
    scene = wl.make_scene(W, H, seed)
    g = random_gamma(H, W, np.random.default_rng(seed))
    p, P = _p(seed, 7)
    s = pg.Samples(spp, H, W)
    pg.sample_mis(p, gpu_view(scene), dev(g), s)
    torch.cuda.synchronize()
    rg = records_host(s)
    ro = O.sample(P, O.OView(scene), g, spp)
    st, live = compare_samples(rg, ro, scene=scene, gamma=g)
    say(f"  {st}")
    assert st["dir_max"] <= TOL_DIR
    assert st["pdf_brdf_p999"] <= TOL_PDF and st["pdf_mix_p999"] <= TOL_PDF


def test_sample_new_models_take_the_brdf():
    """k = 0 everywhere: only BRDF strategies (Sec. 3.1)."""
    say("case: sample k=0")
    W, H, seed = 48, 40, 77
    scene = wl.make_scene(W, H, seed)
    g = random_gamma(H, W, np.random.default_rng(3))
    g[7] = 0
    p, P = _p(seed, 2)
    s = pg.Samples(4, H, W)
    pg.sample_mis(p, gpu_view(scene), dev(g), s)
    torch.cuda.synchronize()
    st = host(s.strategy)
    assert set(np.unique(st)) <= {1, 4}
    assert (st == O.sample(P, O.OView(scene), g, 4)["strategy"]).all()


# ---------------------------------------------------------------- densities
@pytest.mark.parametrize("W,H", [(64, 64), (67, 45)])
def test_pdf_parity_same_input(W, H):
    """pg_pdf against the oracle at the same FP32 directions: the GPU's own
    samples and random directions over the whole sphere."""
    say(f"case: pdf {W}x{H}")
    seed = 3000 + W + H
    scene = wl.make_scene(W, H, seed)
    g = random_gamma(H, W, np.random.default_rng(seed))
    p, P = _p(seed, 4)
    view = gpu_view(scene)
    s = pg.Samples(4, H, W)
    pg.sample_mis(p, view, dev(g), s)
    rng = np.random.default_rng(seed + 1)
    rnd = rng.normal(size=(3, 4, H, W))
    rnd /= np.linalg.norm(rnd, axis=0, keepdims=True)
    dirs = np.concatenate([host(s.dir), rnd.astype(np.float32)], axis=1)
    D, pgd, pbd = pg.pdf(p, view, dev(g), dev(dirs), components=True)
    torch.cuda.synchronize()
    Do, pgo, pbo = O.pdf(P, O.OView(scene), g, dirs)
    tb, tg, tm = pdf_bounds(*conditioning(scene, g, dirs))
    sampled = np.zeros(Do.shape, bool)
    sampled[:4] = True
    for name, a, b, bound in (("D", host(D), Do, tm), ("p_g", host(pgd), pgo, tg),
                              ("p_b", host(pbd), pbo, tb)):
        pos = b > 1e-30
        assert (a[~pos] == 0).all() or np.abs(a[~pos]).max() < 1e-30, name
        r = rel_err(a[pos], b[pos])
        rs = rel_err(a[pos & sampled], b[pos & sampled])
        say(f"  {name}: max {r.max():.2e} p99.9 {np.quantile(r, 0.999):.2e} "
            f"(sampled directions p99.9 {np.quantile(rs, 0.999):.2e}) "
            f"max/bound {(r / bound[pos]).max():.2f}")
        assert (r <= bound[pos]).all(), name
        if name != "p_g":  # p_g alone is ill-conditioned in the far tail of the lobe
            assert np.quantile(r, 0.999) <= TOL_PDF, name


# -------------------------------------------------------------- light field
def test_light_field_parity():
    say("case: light field")
    W, H, seed = 80, 50, 4000
    scene = wl.make_scene(W, H, seed)
    g = random_gamma(H, W, np.random.default_rng(seed))
    p, _ = _p(seed, 4)
    view = gpu_view(scene)
    s = pg.Samples(2, H, W)
    pg.sample_mis(p, view, dev(g), s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), view,
                   dev(scene["vis"]), s)
    torch.cuda.synchronize()
    rg = records_host(s)
    Lo = O.light(scene["lights"], float(scene["ambient"]), scene["vis"], rg["dir"], rg["strategy"])
    live = (rg["strategy"] == 1) | (rg["strategy"] == 2)
    assert (rg["radiance"][~live] == 0).all()
    assert rel_err(rg["radiance"][live], Lo[live]).max() <= 1e-5


# ----------------------------------------------------------------------- EM
def _gpu_records(scene, g, p, spp, view):
    s = pg.Samples(spp, scene["height"], scene["width"])
    pg.sample_mis(p, view, dev(g), s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), view,
                   dev(scene["vis"]), s)
    return s


@pytest.mark.parametrize("W,H", [(64, 64), (67, 45), (1, 1), (5, 90)])
@pytest.mark.parametrize("spp", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("kreg", ["new", "random_new", "mixed", "saturated"])
def test_em_parity_same_input(W, H, spp, kreg):
    """One EM update from the same state and the same records.  "new" is the
    state every model starts from (k = 0 after a reset); the other regimes are
    random states, whose narrow lobes may sit far from the samples.  Every
    spp runs the library's default tile: one pass up to spp 3, from spp 4 the
    two-pass tile (16x16), whose split of the sample planes is uneven at odd
    spp (spp 7: four planes, then three)."""
    say(f"case: em {W}x{H} spp {spp} {kreg}")
    seed = 5000 + W + 7 * H + spp
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    g = random_gamma(H, W, rng, k_lo=0)
    if kreg == "new":
        g[:] = np.array([0.5, 0.5, 1 / 12, 0, 1 / 12, 0.05, 0, 0], np.float32)[:, None, None]
    elif kreg == "random_new":
        g[7] = 0
        g[6] = 0
    elif kreg == "saturated":
        g[7] = 16
    p, P = _p(seed, 6)
    view = gpu_view(scene)
    s = _gpu_records(scene, g, p, spp, view)
    gt = dev(g)
    pg.em_update(p, view, s, gt)
    torch.cuda.synchronize()
    g_o, stats = O.em(P, O.OView(scene), records_host(s), g, with_stats=True)
    gg = host(gt)
    uf = underflow_mask(stats)
    if kreg == "new":
        st = assert_gamma_close(gg, g_o, TOL_EM_FRAME, mask=~uf, what=f"em {kreg}", g_in=g)
    else:
        st = assert_gamma_quantile(gg, g_o, TOL_EM_FRAME, TOL_EM_RUN, mask=~uf, what=f"em {kreg}")
    # where the Gaussian evidence is below FP32 range the state stays valid
    assert np.isfinite(gg[:, uf]).all() and (gg[7, uf] == g_o[7, uf]).all()
    say(f"  {st}  evidence-underflow pixels: {int(uf.sum())}")


@pytest.mark.parametrize("spp", [1, 2, 3, 4, 5, 7, 8])
def test_em_tile_shapes_bitwise_identical(spp):
    """Every built training tile gives the same bits (above spp 1 the tiles
    whose LDS would exceed 64 KiB are refused with PG_ERR_UNSUPPORTED)."""
    say(f"case: em tile invariance, spp {spp}")
    W, H, seed = 99, 61, 6001
    scene = wl.make_scene(W, H, seed)
    g = random_gamma(H, W, np.random.default_rng(seed), k_lo=0)
    view = gpu_view(scene)
    outs, fitted = [], []
    for tw, th in ((32, 8), (16, 16), (64, 4), (32, 4), (16, 8), (64, 2), (32, 16), (64, 8)):
        p = pg.params(seed, frame=3, tile_w=tw, tile_h=th)
        s = _gpu_records(scene, g, p, spp, view)
        gt = dev(g)
        try:
            pg.em_update(p, view, s, gt)
        except RuntimeError as e:
            assert "LDS" in str(e) and spp > 1, e
            continue
        outs.append(host(gt))
        fitted.append((tw, th))
    torch.cuda.synchronize()
    say(f"  tiles run: {fitted}")
    assert fitted == [tl for tl in pg.guide.TILES if pg.guide._tile_lds(tl, spp) <= 64 * 1024]
    assert len(fitted) == 8 if spp == 1 else len(fitted) >= 2
    for o in outs[1:]:
        assert (o.view(np.uint32) == outs[0].view(np.uint32)).all()


def _amplification(P, ov, rec, g, iters, delta=1e-6):
    """Per pixel, how much the oracle's own iters-step batch-EM map amplifies
    a change of the starting state: max over a shift of mu_x, mu_y or pi by
    delta of (change of the final state, in the error metric) / delta."""
    base = O.em(P, ov, rec, g, iterations=iters, batch=True)
    amp = np.zeros(g.shape[1:])
    for ch in (0, 1, 5):
        gp = np.asarray(g, np.float64).copy()
        gp[ch] += delta
        e = gamma_errors(O.em(P, ov, rec, gp, iterations=iters, batch=True), base)
        for key in ("mu", "sigma", "pi"):
            amp = np.maximum(amp, e[key] / delta)
    return amp


@pytest.mark.parametrize("iters", [1, 4, 16])
@pytest.mark.parametrize("start", ["new", "random"])
def test_batch_em_parity(iters, start):
    """Batch EM on a fixed training set.  "new" starts from the state every
    model starts from (the gradient-fit workload's start); "random" from
    random lobes.  Each iteration is checked teacher-forced (the oracle steps
    from the GPU's state after the previous iteration) to the one-frame
    tolerance.  Free-running, the FP32 rounding of the steps is carried by the
    EM map itself, which at pixels whose lobe is still moving several
    iterations in (a random start far from the samples) amplifies a change of
    its input by 100x and more; there the free-running error is held to the
    teacher-forced errors of the steps times the oracle's own measured
    amplification of that pixel, elsewhere to the run tolerance."""
    say(f"case: batch em {iters} from {start}")
    W, H, seed = 40, 36, 6100 + iters
    scene = wl.make_scene(W, H, seed)
    g = random_gamma(H, W, np.random.default_rng(seed))
    if start == "new":
        g[:] = np.array([0.5, 0.5, 1 / 12, 0, 1 / 12, 0.05, 0, 0], np.float32)[:, None, None]
    g[7] = 0
    p, P = _p(seed, 0, flags=pg.PG_EM_BATCH)
    view = gpu_view(scene)
    ov = O.OView(scene)
    s = _gpu_records(scene, g, p, 4, view)
    rec = records_host(s)
    # the GPU's state after every iteration (batch EM from the same start
    # and training set is deterministic)
    states = [g.astype(np.float32)]
    for i in range(1, iters + 1):
        gt = dev(g)
        pg.em_update(p, view, s, gt, iterations=i)
        torch.cuda.synchronize()
        states.append(host(gt))
    g_o, stats = O.em(P, ov, rec, g, iterations=iters, batch=True, with_stats=True)
    uf = underflow_mask(stats)
    # teacher-forced: one oracle iteration from each GPU state
    step_err = np.zeros((iters,) + g.shape[1:])
    for i in range(1, iters + 1):
        o = O.em(P, ov, rec, states[i - 1], iterations=1, batch=True)
        e = gamma_errors(states[i], o)
        step_err[i - 1] = np.maximum(np.maximum(e["mu"], e["sigma"]), e["pi"])
        assert (e["k"] == 0).all()
    tf = step_err[:, ~uf]
    say(f"  teacher-forced per iteration: max {tf.max():.2e}, q0.999 {np.quantile(tf, 0.999):.2e}")
    assert tf.max() <= TOL_EM_FRAME, f"batch em {iters}: a teacher-forced iteration is off by {tf.max():.2e}"
    e = gamma_errors(states[-1], g_o)
    free = np.maximum(np.maximum(e["mu"], e["sigma"]), e["pi"])
    if start == "new" or iters == 1:
        tol = TOL_EM_FRAME if iters == 1 else TOL_EM_RUN
        assert_gamma_close(states[-1], g_o, tol, mask=~uf, what=f"batch em {iters}", g_in=g)
    else:
        amp = _amplification(P, ov, rec, g, iters)
        bound = np.maximum(TOL_EM_RUN, 2.0 * np.maximum(amp, 1.0) * step_err.sum(0))
        over = (free > bound) & ~uf
        need = (free > TOL_EM_RUN) & ~uf
        say(f"  free-running: max {free[~uf].max():.2e}; {int(need.sum())} pixel(s) above {TOL_EM_RUN:.0e}, "
            f"their amplification {np.round(amp[need], 1).tolist()}")
        assert not over.any(), (f"batch em {iters}: free-running error beyond the amplified step errors at "
                                f"{np.argwhere(over)[:3].tolist()}: {free[over][:3]} > {bound[over][:3]}")
        assert (e["k"][~uf] == 0).all()


# -------------------------------------------------------------------- fused
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_fused_equals_two_calls(dtype):
    say(f"case: fused {dtype}")
    W, H, seed = 77, 41, 7000
    scene = wl.make_scene(W, H, seed)
    g_prev = dev(random_gamma(H, W, np.random.default_rng(seed)), dtype)
    mv, mask = wl.make_motion(W, H, seed, 2)
    p = pg.params(seed, frame=2)
    cur, prev = gpu_view(scene, dev(mv), dev(mask)), gpu_view(scene)
    a_g, b_g = torch.empty_like(g_prev), torch.empty_like(g_prev)
    a_s, b_s = pg.Samples(3, H, W), pg.Samples(3, H, W)
    pg.reproject(p, cur, prev, g_prev, a_g)
    pg.sample_mis(p, cur, a_g, a_s)
    pg.reproject_sample(p, cur, prev, g_prev, b_g, b_s)
    torch.cuda.synchronize()
    assert torch.equal(a_g.view(torch.int16 if dtype != torch.float32 else torch.int32),
                       b_g.view(torch.int16 if dtype != torch.float32 else torch.int32))
    for name in ("dir", "pdf_mix", "pdf_brdf", "strategy"):
        assert torch.equal(getattr(a_s, name), getattr(b_s, name)), name


# ------------------------------------------------------------- whole frames
def _shuffle_frames(W, H, seed):
    """Static G-buffer with independent per-pixel motion: every pixel's
    history comes from a random neighbour within 2 px."""
    scene = wl.make_scene(W, H, seed)
    t = 0
    while True:
        mv, mask = wl.make_motion(W, H, seed, t)
        yield dict(scene, motion=mv, disocc=mask)
        t += 1


def _pan_frames(W, H, seed, moving=True):
    seq = wl.Sequence(W, H, seed, moving=moving)
    t = 0
    while True:
        yield seq.frame(t)
        t += 1


def _run_parity(W, H, spp, frames, seed, source):
    """GPU and oracle side by side.  Each frame is checked teacher-forced (the
    oracle steps from the GPU's previous state and uses the GPU's records for
    its EM); the oracle also runs free for the final comparison."""
    gen = source(W, H, seed)
    fr0 = next(gen)
    gf = GpuFrames(W, H, fr0["lights"], fr0["ambient"], spp, seed)
    of = O.Frames(seed=seed, spp=spp)
    worst = {}
    v_prev = None
    fr = fr0
    for t in range(frames):
        if t > 0:
            fr = next(gen)
        say(f"  frame {t}")
        r = gf.step(t, fr)
        P = O.params(seed, frame=t)
        v = O.OView(fr, fr["motion"], fr["disocc"])
        g1, src = O.reproject(P, v, v_prev if v_prev is not None else v,
                              r["gamma_prev"] if t else None)
        ro = O.sample(P, v, g1, spp)
        st, live = compare_samples(r["rec"], ro, scene=fr, gamma=g1)
        assert st["dir_max"] <= TOL_DIR, st
        Lo = O.light(fr["lights"], float(fr["ambient"]), fr["vis"], r["rec"]["dir"], r["rec"]["strategy"])
        lv = (r["rec"]["strategy"] == 1) | (r["rec"]["strategy"] == 2)
        assert rel_err(r["rec"]["radiance"][lv], Lo[lv]).max(initial=0) <= 1e-5
        g2, stats = O.em(P, v, r["rec"], g1, with_stats=True)
        e = assert_gamma_close(r["gamma"], g2, TOL_EM_FRAME, mask=~underflow_mask(stats),
                               what=f"frame {t}")
        for k_, v_ in e.items():
            worst[k_] = max(worst.get(k_, 0.0), v_)
        of.step(t, fr)
        v_prev = v
    return gf, of, worst


def test_run_64x64_spp1_8_frames_static():
    """The small static workload: every output of every frame, then the
    free-running states after 8 frames."""
    say("case: run 64x64 spp1 8 frames")
    cfg = wl.CONFIGS["64x64_spp1_8f_fp32_static"]
    gf, of, worst = _run_parity(64, 64, 1, 8, cfg["seed"],
                                lambda W, H, s: _pan_frames(W, H, s, moving=False))
    say(f"  teacher-forced worst {worst}")
    st = assert_gamma_close(host(gf.g.state), of.gamma, TOL_EM_RUN, what="free run")
    say(f"  free-running after 8 frames {st}")


@pytest.mark.parametrize("spp", [2, 5])
def test_run_ragged_pan(spp):
    say(f"case: run 93x57 spp{spp} pan")
    gf, of, worst = _run_parity(93, 57, spp, 6, 8100 + spp, _pan_frames)
    say(f"  teacher-forced worst {worst}")


def test_run_ragged_shuffle():
    say("case: run 71x43 spp1 independent motion")
    gf, of, worst = _run_parity(71, 43, 1, 6, 8200, _shuffle_frames)
    say(f"  teacher-forced worst {worst}")


# ------------------------------------------------------- non-finite inputs
def test_nonfinite_gbuffer_inputs():
    """NaN and Inf sprinkled into the normals, view directions, depths,
    roughness, albedo and motion vectors: reprojection decisions, strategy
    codes and the update agree with the oracle pixel for pixel, and a state
    is finite exactly where the oracle's is (an infinite normal component can
    pass the validity test and carry a history into a frame that is not
    finite; the next frame restarts such a model, as any non-finite
    history)."""
    W, H, spp, seed = 71, 43, 2, 16000
    say("case: non-finite G-buffer inputs")
    scene = wl.make_scene(W, H, seed)
    rng = np.random.default_rng(seed)
    bad = dict(scene)
    for key in ("normal", "view_dir", "depth", "roughness", "albedo"):
        a = np.array(scene[key], copy=True)
        m = rng.uniform(size=a.shape[-2:]) < 0.03
        vals = rng.choice([np.nan, np.inf, -np.inf], size=int(m.sum())).astype(np.float32)
        if a.ndim == 3:
            a[rng.integers(0, a.shape[0]), m] = vals
        else:
            a[m] = vals
        bad[key] = a
    mv, mask = wl.make_motion(W, H, seed, 3)
    mm = rng.uniform(size=(H, W)) < 0.03
    mv[0, mm] = rng.choice([np.nan, np.inf], size=int(mm.sum()))
    g_prev = random_gamma(H, W, rng, k_lo=0)
    p, P = _p(seed, 3)
    cur, prev = gpu_view(bad, dev(mv), dev(mask)), gpu_view(scene)
    go = torch.empty_like(dev(g_prev))
    src = torch.empty((H, W), dtype=torch.int32, device="cuda")
    pg.reproject(p, cur, prev, dev(g_prev), go, src)
    s = pg.Samples(spp, H, W)
    pg.sample_mis(p, cur, go, s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), cur, dev(scene["vis"]), s)
    torch.cuda.synchronize()
    vo = O.OView(bad, mv, mask)
    g_o, src_o = O.reproject(P, vo, O.OView(scene), g_prev)
    assert (host(src) == src_o).all()
    gg = host(go)
    fin_state = np.isfinite(g_o).all(0)
    assert (np.isfinite(gg).all(0) == fin_state).all()
    assert gamma_errors(gg[:, fin_state], g_o[:, fin_state])["mu"].max(initial=0) <= TOL_DIR
    rec_g = records_host(s)
    rec_o = O.sample(P, vo, gg, spp)
    fin = fin_state & np.isfinite(rec_o["pdf_mix"]).all(0) & np.isfinite(rec_o["dir"]).all((0, 1))
    near = rec_o["margin"] < MARGIN
    assert ((rec_g["strategy"] == rec_o["strategy"]) | near | ~fin[None]).all()
    live = ((rec_g["strategy"] == 1) | (rec_g["strategy"] == 2)) & fin[None]
    assert np.isfinite(rec_g["dir"][:, live]).all() and np.isfinite(rec_g["pdf_mix"][live]).all()
    gt = dev(gg)
    pg.em_update(p, cur, s, gt)
    torch.cuda.synchronize()
    g_e, stats = O.em(P, vo, rec_g, gg, with_stats=True)
    ge = host(gt)
    ok = np.isfinite(g_e).all(0) & ~underflow_mask(stats)
    assert np.isfinite(ge[:, ok]).all()
    st = assert_gamma_quantile(ge, g_e, TOL_EM_FRAME, TOL_EM_RUN, mask=ok, what="non-finite inputs")
    say(f"  non-finite states {int((~fin_state).sum())}, resets {int((src_o < 0).sum())}, EM {st}")
