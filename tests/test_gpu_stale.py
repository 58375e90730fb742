"""Rejection of stale histories (PG_STALE_RESET): a trained model whose
weighted log-likelihood of its training set falls below a new model's by more
than stale_tau per unit weight is reset before the E-step.

Parity of the decisions and of the updated states with the oracle (pixels
whose decision margin is within 1e-4 of the threshold may go either way and
are set aside), the flag with an infinite threshold against the default
update (bit for bit), and what it is for: on the 1080p pan, the most
powerful light jumps to a new direction at frame 16; the 1-spp estimate's
relative MSE against the FP64 reference (1024 samples per pixel, 32768
pixels) after the jump, with and without the reset, with a paired bootstrap
interval (reported; the gain on this workload is small)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import paired_ratio_ci, TOL_EM_FRAME, assert_gamma_close, dev, gpu_view, host, underflow_mask

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

MARGIN = 1e-4


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _setup(W, H, spp, seed):
    """Frame-0 records of the oracle (rounded to FP32, the GPU's input) and
    trained histories with lobes at random places."""
    sc = wl.make_scene(W, H, seed)
    v = O.OView(sc)
    P = O.params(seed, frame=0)
    g0, _ = O.reproject(P, v, None, None)
    rec = O.sample(P, v, g0, spp)
    rec["radiance"] = O.light(sc["lights"], float(sc["ambient"]), sc["vis"], rec["dir"], rec["strategy"])
    rec = {k: (a.astype(np.float32) if a.dtype == np.float64 else a) for k, a in rec.items()}
    rng = np.random.default_rng(seed)
    g = np.zeros((8, H, W), np.float32)
    g[0] = rng.uniform(0.1, 0.9, (H, W))
    g[1] = rng.uniform(0.1, 0.9, (H, W))
    g[2] = g[4] = 0.002
    g[5] = rng.uniform(0.3, 0.9, (H, W))
    g[6] = rng.uniform(1.0, 5.0, (H, W))
    g[7] = rng.integers(1, 17, (H, W))
    return sc, v, rec, g


def _gpu_samples(rec):
    spp, H, W = rec["strategy"].shape
    return pg.Samples.wrap(dev(rec["dir"]), dev(rec["pdf_mix"]), dev(rec["pdf_brdf"]), dev(rec["strategy"]),
                           dev(rec["radiance"]))


@pytest.mark.parametrize("tau", [0.5, 0.0])
def test_stale_reset_parity(tau):
    W, H, spp, seed = 96, 64, 2, 9400
    say(f"case: stale reset parity, tau {tau}")
    sc, v, rec, g = _setup(W, H, spp, seed)
    kw = dict(frame=3, flags=pg.PG_STALE_RESET, stale_tau=tau)
    gt = dev(g)
    pg.em_update(pg.params(seed, **kw), gpu_view(sc), _gpu_samples(rec), gt)
    torch.cuda.synchronize()
    gg = host(gt)
    P = O.params(seed, **kw)
    go, stats = O.em(P, v, rec, g, with_stats=True)
    margin = O.stale_margin(P, v, rec, g)
    clear = ~np.isnan(margin) & (np.abs(np.nan_to_num(margin)) > MARGIN)
    reset_o, reset_g = go[7] == 1, gg[7] == 1
    say(f"  applicable {int((~np.isnan(margin)).sum())}, reset (oracle) {int(reset_o.sum())}, "
        f"within the margin {int((~np.isnan(margin) & ~clear).sum())}")
    assert (reset_o[clear] == reset_g[clear]).all()
    assert reset_o[clear].sum() > 0
    ok = clear & ~underflow_mask(stats)
    e = assert_gamma_close(gg, go, TOL_EM_FRAME, mask=ok, what="stale reset")
    say(f"  EM {e}")


@pytest.mark.parametrize("spp", [2, 4])
def test_stale_reset_with_infinite_threshold_is_the_default_update(spp):
    """A threshold that never fires leaves the update as it is: bit for bit
    below spp 4.  From spp 4 the default update runs the two-pass training tile,
    which visits the samples of the last half of the sample planes after the
    first, while the stale test needs every record staged at once and keeps
    the training set's order: the FP32 sums round differently, within the
    one-step tolerance, and the epochs agree."""
    W, H, seed = 67, 45, 9500 + spp
    say(f"case: stale reset, tau = +inf, spp {spp}")
    sc, v, rec, g = _setup(W, H, spp, seed)
    view, s = gpu_view(sc), _gpu_samples(rec)
    a, b = dev(g), dev(g)
    pg.em_update(pg.params(seed, frame=3), view, s, a)
    pg.em_update(pg.params(seed, frame=3, flags=pg.PG_STALE_RESET, stale_tau=1e30), view, s, b)
    torch.cuda.synchronize()
    if spp < 4:
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    else:
        assert_gamma_close(host(b), host(a).astype(np.float64), TOL_EM_FRAME, what="tau = +inf against the default")


def test_recovery_after_a_light_moves():
    cfg = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]
    W, H, seed, t_move, frames, tau = 1920, 1080, cfg["seed"], 16, 28, 0.5
    evals = (15, 16, 17, 18, 20, 23, 27)
    n_px, n_ref = 32768, 1024
    say(f"case: light jumps at frame {t_move}; plain vs stale reset (tau {tau}); {n_px} px")
    seq = wl.Sequence(W, H, seed, light_moves_at=t_move)
    fr = seq.frame(0)
    amb = float(fr["ambient"])
    runs = {"plain": pg.Guide(W, H, fr["lights"], amb, spp=1, seed=seed),
            "reset": pg.Guide(W, H, fr["lights"], amb, spp=1, seed=seed, flags=pg.PG_STALE_RESET, stale_tau=tau)}
    rng = np.random.default_rng(seed + 1)
    prev = None
    rows = []
    post_err = {k: [] for k in runs}
    for t in range(frames):
        if t:
            fr = seq.frame(t)
        cur = pg.DeviceFrame(fr)
        for g in runs.values():
            g.lights = pg.lights_struct(fr["lights"], amb)
            g.step(cur, prev, frame=t)
        prev = cur
        if t not in evals:
            continue
        est = {k: host(pg.estimate(g.params(t), cur.view, g.samples)) for k, g in runs.items()}
        torch.cuda.synchronize()
        # models restarted by the test: k = 1 beyond the restarts of the plain
        # run (reprojection resets end the frame at k = 1 in both)
        k1 = {k: float((host(g.state[7]) == 1).mean()) for k, g in runs.items()}
        valid = (np.einsum("chw,chw->hw", fr["normal"], fr["view_dir"]) > 0) & (fr["roughness"] >= 0.1)
        px = np.sort(rng.choice(np.flatnonzero(valid.reshape(-1)), size=n_px, replace=False))
        ref, se = O.reference(O.params(seed, frame=t), O.OView(fr), fr["lights"], amb, fr["vis"], px, n_ref)
        r2 = float((ref ** 2).sum())
        mse = {k: float(((e.reshape(-1)[px] - ref) ** 2).sum()) / r2 for k, e in est.items()}
        if t >= t_move:
            for k, e in est.items():
                post_err[k].append((e.reshape(-1)[px] - ref) ** 2 / r2)
        resets = k1["reset"] - k1["plain"]
        rows.append((t, mse["plain"], mse["reset"], resets))
        say(f"  frame {t:2d}: rel. MSE plain {mse['plain']:.3f}, with reset {mse['reset']:.3f}, "
            f"pixels reset this frame {resets:.4f}")
    pre = [r for r in rows if r[0] < t_move]
    post = [r for r in rows if r[0] >= t_move]
    say(f"  mean rel. MSE after the jump: plain {np.mean([r[1] for r in post]):.3f}, "
        f"with reset {np.mean([r[2] for r in post]):.3f}")
    rr, lo, hi = paired_ratio_ci(np.concatenate(post_err["reset"]), np.concatenate(post_err["plain"]))
    say(f"  with reset / plain MSE after the jump: {rr:.3f}, paired bootstrap 95% [{lo:.3f}, {hi:.3f}]")
    assert all(np.isfinite(r[1]) and np.isfinite(r[2]) for r in rows)
    # measured: a small gain after the jump (the rule, as read, fires on few
    # lobes here); guard that the reset never costs more than 10%
    assert np.mean([r[2] for r in post]) <= 1.1 * np.mean([r[1] for r in post])
