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


class DeviceFrame:
    """One frame's inputs resident on the device: the G-buffer view (with
    motion and disocclusion) and the light-visibility bits."""

    def __init__(self, fr: dict, device="cuda"):
        import numpy as np

        def dev(a):
            return None if a is None else torch.as_tensor(np.ascontiguousarray(a)).to(device)
        self.view = View(dev(fr["normal"]), dev(fr["view_dir"]), dev(fr["depth"]),
                         dev(fr["roughness"]), dev(fr["albedo"]), dev(fr.get("motion")),
                         dev(fr.get("disocc")))
        self.vis = dev(fr["vis"])


class Guide:
    """Per-view state of the path (two Gamma buffers used in turn, the sample
    records) and one frame of it per ``step``."""

    def __init__(self, width: int, height: int, lights, ambient, spp: int = 1, seed: int = 0,
                 view_id: int = 0, gamma_dtype=torch.float32, fused: bool = True, device="cuda",
                 **param_overrides):
        self.width, self.height = width, height
        self.spp = spp
        self.seed = seed
        self.view_id = view_id
        self.fused = fused
        self.overrides = param_overrides
        self.lights = lights_struct(lights, ambient)
        self.gamma = [new_gamma(height, width, gamma_dtype, device),
                      new_gamma(height, width, gamma_dtype, device)]
        self.cur = 0
        self.samples = Samples(spp, height, width, device)
        self.frame = 0

    def params(self, frame: int) -> PgParams:
        return params(self.seed, frame=frame, view=self.view_id, **self.overrides)

    @property
    def state(self):
        return self.gamma[self.cur]

    def step(self, cur: DeviceFrame, prev: DeviceFrame | None, frame: int | None = None):
        """One frame on the current stream; returns the updated Gamma tensor."""
        t = self.frame if frame is None else frame
        p = self.params(t)
        pv = prev.view if (prev is not None and t > 0) else None
        g_prev, g_out = self.gamma[self.cur], self.gamma[1 - self.cur]
        if self.fused:
            reproject_sample(p, cur.view, pv, g_prev if t > 0 else None, g_out, self.samples)
        else:
            reproject(p, cur.view, pv, g_prev if t > 0 else None, g_out)
            sample_mis(p, cur.view, g_out, self.samples)
        light_field(self.lights, cur.view, cur.vis, self.samples)
        em_update(p, cur.view, self.samples, g_out)
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
