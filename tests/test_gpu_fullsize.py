"""Parity at the benchmark's size and launch configuration: the 1920x1080,
1 spp camera-pan sequence with the library's default tiles.

Frames 0-3: every pixel, teacher-forced (the oracle steps from the GPU's
previous state and trains on the GPU's records), and the free-running states
after 4 frames.  Frame 40: the 256x256 crop at (832, 412), teacher-forced
from the GPU's state of frame 39 (the oracle computes only the crop and the
neighbours its picks read)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl
from pgtest import (TOL_DIR, TOL_EM_FRAME, TOL_EM_RUN, GpuFrames, assert_gamma_close, compare_samples,
                    host, rel_err, underflow_mask)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

W, H = 1920, 1080
CFG = wl.CONFIGS["1080p_spp1_64f_fp32_pan"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_frame(t, fr, r, v_prev, rect=None):
    P = O.params(CFG["seed"], frame=t)
    v = O.OView(fr, fr["motion"], fr["disocc"])
    g1, src = O.reproject(P, v, v_prev if v_prev is not None else v,
                          r["gamma_prev"] if t else None, rect=None if rect is None else _grow(rect, 3))
    ro = O.sample(P, v, g1, 1, rect=None if rect is None else _grow(rect, 3))
    if rect is None:
        cmp_mask = None
    else:
        cmp_mask = np.zeros((H, W), bool)
        x0, y0, x1, y1 = _grow(rect, 3)
        cmp_mask[y0:y1, x0:x1] = True
    st, _ = compare_samples(r["rec"], ro, pix_mask=cmp_mask, scene=fr, gamma=g1)
    say(f"  frame {t}: samples {st}")
    assert st["dir_max"] <= TOL_DIR
    g2, stats = O.em(P, v, r["rec"], g1, rect=rect, with_stats=True)
    m = ~underflow_mask(stats)
    if rect is not None:
        x0, y0, x1, y1 = rect
        sub = np.zeros((H, W), bool)
        sub[y0:y1, x0:x1] = True
        m &= sub
    e = assert_gamma_close(r["gamma"], g2, TOL_EM_FRAME, mask=m, what=f"frame {t}")
    say(f"  frame {t}: EM {e}")
    return v


def _grow(rect, d):
    x0, y0, x1, y1 = rect
    return max(0, x0 - d), max(0, y0 - d), min(W, x1 + d), min(H, y1 + d)


def test_1080p_first_frames_every_pixel():
    say("case: 1080p frames 0-3, every pixel")
    seq = wl.Sequence(W, H, CFG["seed"])
    fr = seq.frame(0)
    gf = GpuFrames(W, H, fr["lights"], fr["ambient"], 1, CFG["seed"])
    of = O.Frames(seed=CFG["seed"], spp=1)
    v_prev = None
    for t in range(4):
        if t:
            fr = seq.frame(t)
        r = gf.step(t, fr)
        v_prev = _check_frame(t, fr, r, v_prev)
        of.step(t, fr)
    st = assert_gamma_close(host(gf.g.state), of.gamma, TOL_EM_RUN, what="free run, 4 frames")
    say(f"  free-running after 4 frames: {st}")


def test_1080p_crop_late_frame():
    say("case: 1080p crop at frame 40")
    seq = wl.Sequence(W, H, CFG["seed"])
    fr = seq.frame(0)
    gf = GpuFrames(W, H, fr["lights"], fr["ambient"], 1, CFG["seed"])
    prev = None
    for t in range(40):
        if t:
            fr = seq.frame(t)
        gf.step(t, fr, keep=False)
        prev = fr
    v_prev = O.OView(prev, prev["motion"], prev["disocc"])
    fr = seq.frame(40)
    r = gf.step(40, fr)
    _check_frame(40, fr, r, v_prev, rect=CFG["crop"])
    k = r["gamma"][7]
    say(f"  k at frame 40: mean {k.mean():.2f}, share at kMax {(k == 16).mean():.3f}")
