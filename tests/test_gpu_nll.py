"""The radiance-weighted NLL of the mixture and its hand-written adjoint on the
GPU: parity with the oracle, central differences in FP64, and a gradient fit
through torch.autograd against batch EM on the same samples."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import dev, gpu_view, host, records_host

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _setup(W, H, spp, seed):
    """Frame-0 records (every model new: BRDF samples, N(0) = 20 picks)."""
    scene = wl.make_scene(W, H, seed)
    p = pg.params(seed, frame=0)
    view = gpu_view(scene)
    g0 = torch.zeros((8, H, W), dtype=torch.float32, device="cuda")
    s = pg.Samples(spp, H, W)
    pg.reproject_sample(p, view, None, None, g0, s)
    pg.light_field(pg.lights_struct(scene["lights"], float(scene["ambient"])), view,
                   dev(scene["vis"]), s)
    torch.cuda.synchronize()
    return scene, view, s, host(g0)


def _theta(H, W, rng):
    return np.stack([rng.uniform(0.3, 0.7, (H, W)), rng.uniform(0.3, 0.7, (H, W)),
                     rng.uniform(0.05, 0.2, (H, W)), rng.uniform(-0.05, 0.05, (H, W)),
                     rng.uniform(0.05, 0.2, (H, W)), rng.uniform(-2, 2, (H, W)),
                     np.zeros((H, W)), np.zeros((H, W))]).astype(np.float32)


@pytest.mark.parametrize("W,H,spp", [(64, 48, 4), (37, 29, 1)])
def test_nll_and_adjoint_match_oracle(W, H, spp):
    say(f"case: nll {W}x{H} spp {spp}")
    seed = 9000 + W + spp
    scene, view, s, _ = _setup(W, H, spp, seed)
    th = _theta(H, W, np.random.default_rng(seed))
    go = np.random.default_rng(seed + 1).uniform(0.5, 2.0, (H, W)).astype(np.float32)
    p = pg.params(seed, frame=0)
    nll, grad = pg.nll_backward(p, view, s, dev(th), grad_out=dev(go))
    torch.cuda.synchronize()
    P = O.params(seed, frame=0)
    nll_o, grad_o = O.nll(P, O.OView(scene), records_host(s), th, grad_out=go)
    nll_g, grad_g = host(nll), host(grad)
    scale_n = np.abs(nll_o).max() + 1e-30
    en = np.abs(nll_g - nll_o) / (np.abs(nll_o) + 1e-3 * scale_n)
    say(f"  nll rel err max {en.max():.2e}")
    assert en.max() <= 1e-4
    for c in range(6):
        sc = np.abs(grad_o[c]).max() + 1e-30
        e = np.abs(grad_g[c] - grad_o[c]) / (np.abs(grad_o[c]) + 1e-3 * sc)
        say(f"  grad[{c}] rel err max {e.max():.2e} p99 {np.quantile(e, 0.99):.2e}")
        assert np.quantile(e, 0.99) <= 1e-4 and e.max() <= 1e-3, c
    assert (grad_g[6:] == 0).all()


def test_adjoint_against_fp64_central_differences_on_crop():
    """Central differences of the FP64 oracle's NLL (h = 1e-4) on a 32x32
    crop against the GPU adjoint."""
    say("case: adjoint vs FD 32x32 crop")
    W = H = 96
    seed = wl.SEED_BASE + 4
    scene, view, s, _ = _setup(W, H, 4, seed)
    th = _theta(H, W, np.random.default_rng(seed))
    p = pg.params(seed, frame=0)
    _, grad = pg.nll_backward(p, view, s, dev(th))
    torch.cuda.synchronize()
    grad_g = host(grad)
    P = O.params(seed, frame=0)
    ov = O.OView(scene)
    rec = records_host(s)
    rect = (32, 32, 64, 64)
    h = 1e-4
    x0, y0, x1, y1 = rect
    for c in range(6):
        tp, tm = th.astype(np.float64), th.astype(np.float64)
        tp = tp.copy()
        tm = tm.copy()
        tp[c] += h
        tm[c] -= h
        fd = (O.nll(P, ov, rec, tp, rect=rect)[0] - O.nll(P, ov, rec, tm, rect=rect)[0]) / (2 * h)
        fd = fd[y0:y1, x0:x1]
        gg = grad_g[c, y0:y1, x0:x1]
        sc = np.abs(fd).max() + 1e-30
        e = np.abs(gg - fd) / (np.abs(fd) + 1e-2 * sc)
        say(f"  channel {c}: rel err p99 {np.quantile(e, 0.99):.2e} max {e.max():.2e}")
        assert np.quantile(e, 0.99) <= 1e-4 and e.max() <= 1e-3, c


def test_gradient_fit_reaches_batch_em_likelihood():
    """Adam on (mu, Cholesky factor, logit pi) through NLLFunction against 16
    iterations of batch EM on the same samples, both without the pi clamp: the
    fit must reach (or beat) EM's summed NLL within 1%."""
    say("case: gradient fit vs batch EM")
    W, H, spp = 64, 64, 4
    seed = wl.SEED_BASE + 4
    scene, view, s, g0 = _setup(W, H, spp, seed)
    p = pg.params(seed, frame=0, flags=pg.PG_NO_CLAMP | pg.PG_EM_BATCH)
    ge = dev(g0)
    pg.em_update(p, view, s, ge, iterations=16)
    gem = host(ge)
    l11 = np.sqrt(np.maximum(gem[2], 0))
    l21 = np.where(l11 > 0, gem[3] / np.where(l11 > 0, l11, 1), 0)
    l22 = np.sqrt(np.maximum(gem[4] - l21 ** 2, 0))
    pi = np.clip(gem[5], 1e-6, 1 - 1e-6)
    th_em = np.stack([gem[0], gem[1], l11, l21, l22, np.log(pi / (1 - pi)), gem[6], gem[7]])
    pn = pg.params(seed, frame=0, flags=pg.PG_NO_CLAMP)
    nll_em, _ = pg.nll_backward(pn, view, s, dev(th_em.astype(np.float32)), want_grad=False)
    # gradient fit from the new-model state
    th0 = np.stack([g0[0], g0[1], np.sqrt(g0[2]), g0[3], np.sqrt(g0[4]),
                    np.log(g0[5] / (1 - g0[5])), g0[6], g0[7]]).astype(np.float32)
    theta = torch.tensor(th0, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([theta], lr=0.02)
    mask = torch.zeros_like(theta)
    mask[:6] = 1
    hist = []
    for it in range(300):
        opt.zero_grad()
        loss = pg.NLLFunction.apply(theta, pn, view, s).sum()
        loss.backward()
        theta.grad.mul_(mask)
        opt.step()
        hist.append(float(loss.detach()))
    torch.cuda.synchronize()
    total_em = float(nll_em.sum())
    assert np.isfinite(total_em)
    say(f"  summed NLL: EM(16) {total_em:.2f}  gradient fit start {hist[0]:.2f} end {hist[-1]:.2f}")
    assert hist[-1] < hist[0]
    assert hist[-1] <= total_em + 0.01 * abs(total_em)
