"""Frame driver and autograd wrapper over the libpmmguide calls.

``Guide`` owns the per-view device state (two Gamma buffers used in turn, the
sample records) and runs one frame of the path: reprojection and sampling
(fused, or as two calls), the analytic light field that stands in for the
trace, and the EM update.  ``NLLFunction`` puts the hand-written adjoint of
the radiance-weighted mixture NLL behind ``torch.autograd``.
"""
from __future__ import annotations

import torch

from . import (PgParams, Samples, View, em_update, light_field, lights_struct, new_gamma, params,
               reproject, reproject_sample, sample_mis, nll_backward)


class Guide:
    def __init__(self, scene: dict, spp: int = 1, seed: int | None = None, view_id: int = 0,
                 gamma_dtype=torch.float32, fused: bool = True, device="cuda", **param_overrides):
        self.scene = scene
        self.spp = spp
        self.seed = scene.get("seed", 0) if seed is None else seed
        self.view_id = view_id
        self.fused = fused
        self.overrides = param_overrides
        H, W = scene["height"], scene["width"]
        self.base = View.from_scene(scene, device)
        # previous-frame G-buffer kept in its own memory, as a renderer would
        self.prev_base = View.from_scene(scene, device)
        self.vis = torch.as_tensor(scene["vis"]).to(device).contiguous()
        self.lights = lights_struct(scene["lights"], float(scene["ambient"]))
        self.gamma = [new_gamma(H, W, gamma_dtype, device), new_gamma(H, W, gamma_dtype, device)]
        self.cur = 0
        self.samples = Samples(spp, H, W, device)
        self.frame = 0

    def params(self, frame: int) -> PgParams:
        return params(self.seed, frame=frame, view=self.view_id, **self.overrides)

    @property
    def state(self):
        return self.gamma[self.cur]

    def view_for(self, motion, disocc) -> View:
        return self.base.with_motion(motion, disocc)

    def step(self, motion=None, disocc=None, frame: int | None = None):
        """One frame on the current stream; returns the updated Gamma tensor."""
        t = self.frame if frame is None else frame
        p = self.params(t)
        cur = self.view_for(motion, disocc)
        prev = self.prev_base if t > 0 else None
        g_prev, g_out = self.gamma[self.cur], self.gamma[1 - self.cur]
        if self.fused:
            reproject_sample(p, cur, prev, g_prev if t > 0 else None, g_out, self.samples)
        else:
            reproject(p, cur, prev, g_prev if t > 0 else None, g_out)
            sample_mis(p, cur, g_out, self.samples)
        light_field(self.lights, cur, self.vis, self.samples)
        em_update(p, cur, self.samples, g_out)
        self.cur = 1 - self.cur
        self.frame = t + 1
        return g_out


class NLLFunction(torch.autograd.Function):
    """NLL(theta) per pixel; backward runs the hand-written adjoint kernel.

    forward(theta, params, view, samples) -> nll [H][W]."""

    @staticmethod
    def forward(ctx, theta, p, view, samples):
        nll, _ = nll_backward(p, view, samples, theta.contiguous(), want_grad=False)
        ctx.save_for_backward(theta)
        ctx.p, ctx.view, ctx.samples = p, view, samples
        return nll

    @staticmethod
    def backward(ctx, grad_nll):
        (theta,) = ctx.saved_tensors
        _, grad = nll_backward(ctx.p, ctx.view, ctx.samples, theta.contiguous(),
                               grad_out=grad_nll.contiguous(), want_nll=False)
        return grad, None, None, None
