"""Frame driver and autograd wrapper over the libpmmguide calls.

``Guide`` owns the per-view device state (two Gamma buffers used in turn, the
sample records) and runs one frame of the path: reprojection and sampling
(fused, or as two calls), the analytic light field that stands in for the
trace, and the EM update; ``LobesGuide`` the same with K Gaussian lobes per
pixel.  ``BatchedGuide`` does the same for many views at
once through pg_frame_batched, eagerly or by replaying captured graphs, and
picks its training tile by timing the candidates.  ``NLLFunction`` puts the
hand-written adjoint of the radiance-weighted mixture NLL behind
``torch.autograd``.
"""
from __future__ import annotations

import torch

from . import (PgBatchView, PgParams, Samples, View, _gamma, batch_pack, batch_table_bytes, em_update,
               em_update_lobes, frame_batched, frame_batched_noalloc, light_field, lights_struct, new_gamma, new_lobes_gamma, params,
               reproject, reproject_sample, reproject_sample_lobes, sample_mis, nll_backward)

TILES = ((32, 8), (16, 16), (64, 4), (32, 4), (16, 8), (64, 2), (32, 16), (64, 8))


def _tile_lds(tile, spp: int) -> int:
    """Dynamic LDS bytes of a training tile for online EM, as the library
    sizes it: the records with the 3-pixel halo (from spp 4 half the sample
    planes at a time, with a validity bit per record of all planes and a
    byte per pixel), the training lists and the pick table."""
    w, h = tile
    sa = (w + 6) * (h + 6)
    lists = (spp + 20) * w * h * 2 + ((48 * spp * 2 + 15) & ~15)
    if spp < 4:
        return sa * spp * 16 + lists
    bits = ((spp * sa + 31) // 32 * 4 + 15) & ~15
    return sa * ((spp + 1) // 2) * 16 + bits + lists + w * h


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
        self.position = dev(fr.get("position"))


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


class LobesGuide(Guide):
    """Guide with K Gaussian lobes per pixel (FP32 state [6K + 2][H][W]):
    reprojection + sampling, the light field and the K-lobe EM update."""

    def __init__(self, width: int, height: int, lights, ambient, lobes: int = 2, spp: int = 1, seed: int = 0,
                 view_id: int = 0, device="cuda", **param_overrides):
        super().__init__(width, height, lights, ambient, spp=spp, seed=seed, view_id=view_id, device=device,
                         **param_overrides)
        self.lobes = lobes
        self.gamma = [new_lobes_gamma(lobes, height, width, device), new_lobes_gamma(lobes, height, width, device)]

    def step(self, cur: DeviceFrame, prev: DeviceFrame | None, frame: int | None = None):
        t = self.frame if frame is None else frame
        p = self.params(t)
        pv = prev.view if (prev is not None and t > 0) else None
        g_prev, g_out = self.gamma[self.cur], self.gamma[1 - self.cur]
        reproject_sample_lobes(p, self.lobes, cur.view, pv, g_prev if t > 0 else None, g_out, self.samples)
        light_field(self.lights, cur.view, cur.vis, self.samples)
        em_update_lobes(p, self.lobes, cur.view, self.samples, g_out)
        self.cur = 1 - self.cur
        self.frame = t + 1
        return g_out


class BatchedGuide:
    """Many views stepped together: per frame one packed table and the
    launches of pg_frame_batched over the tiles of all views, run eagerly or
    replayed from captured graphs.

    specs: one dict per view with width, height, spp, seed, lights, ambient
    (and optionally view, the view id; default its position).  Two pinned host
    tables are used in turn, so packing frame t+1 only waits for the upload of
    frame t-1; each has its own captured graph.  The caller keeps the
    DeviceFrames of the last two frames alive (the tables point at them).

    tile: the training tile, one (w, h) for every spp group or a dict
    {spp: (w, h)} (groups not named use the library's default); ``autotune``
    picks one per group."""

    def __init__(self, specs, gamma_dtype=torch.float16, device="cuda", tile=None, noalloc=False,
                 **param_overrides):
        self.specs = [dict(s) for s in specs]
        self.n = len(self.specs)
        self.overrides = param_overrides
        self.tile = dict(tile) if isinstance(tile, dict) else tile
        self.noalloc = noalloc  # the device table in the library's own array
        self.gamma = [[new_gamma(s["height"], s["width"], gamma_dtype, device),
                       new_gamma(s["height"], s["width"], gamma_dtype, device)] for s in self.specs]
        self.samples = [Samples(s["spp"], s["height"], s["width"], device) for s in self.specs]
        self.lights = [lights_struct(s["lights"], s["ambient"]) for s in self.specs]
        nbytes = batch_table_bytes(self.n)
        self.host_tables = [torch.empty(nbytes, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.dev_table = None if noalloc else torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.graphs = [None, None]
        self.done = [None, None]
        self.keep = [None, None]
        self.slot = 0
        self.cur = 0
        self.frame = 0

    def state(self, i: int):
        return self.gamma[i][self.cur]

    def tile_of(self, spp: int):
        """The training tile requested for the views of `spp` ((0, 0): default)."""
        if isinstance(self.tile, dict):
            return tuple(self.tile.get(spp, (0, 0)))
        return tuple(self.tile) if self.tile else (0, 0)

    def _views(self, frames, t: int):
        out = []
        for i, (s, (cur, prev)) in enumerate(zip(self.specs, frames)):
            tw, th = self.tile_of(s["spp"])
            b = PgBatchView()
            b.params = params(s["seed"], frame=t, view=s.get("view", i), tile_w=tw, tile_h=th,
                              **self.overrides)
            b.cur = cur.view.c
            if t > 0:
                b.prev = prev.view.c
                b.gamma_in = _gamma(self.gamma[i][self.cur])
            b.gamma_out = _gamma(self.gamma[i][1 - self.cur])
            b.samples = self.samples[i].c
            b.vis = cur.vis.data_ptr()
            b.lights = self.lights[i]
            out.append(b)
        return out

    def _pack(self, frames, t: int, slot: int):
        if self.done[slot] is not None:
            self.done[slot].synchronize()  # the upload that read this table has run
        batch_pack(self._views(frames, t), self.host_tables[slot])
        self.keep[slot] = frames

    def _launch(self, slot: int):
        if self.noalloc:
            frame_batched_noalloc(self.host_tables[slot])
        else:
            frame_batched(self.host_tables[slot], self.dev_table)

    def _run(self, slot: int, graph: bool):
        if graph:
            if self.graphs[slot] is None:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, capture_error_mode="thread_local"):
                    self._launch(slot)
                self.graphs[slot] = g
            self.graphs[slot].replay()
        else:
            self._launch(slot)
        ev = torch.cuda.Event()
        ev.record()
        self.done[slot] = ev

    def step(self, frames, t: int | None = None, graph: bool = False):
        """One frame of every view.  frames: per view (cur, prev) DeviceFrames
        (prev may be None at frame 0)."""
        t = self.frame if t is None else t
        slot = self.slot
        self._pack(frames, t, slot)
        self._run(slot, graph)
        self.slot = 1 - slot
        self.cur = 1 - self.cur
        self.frame = t + 1

    def _time_frame(self, frames, t: int, reps: int):
        """ms of one batched frame with the current tiles (recomputed from the
        same inputs, so the state is not advanced); None if a tile does not
        fit its group."""
        try:
            self._pack(frames, t, self.slot)
        except RuntimeError:
            return None
        self._run(self.slot, graph=False)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            self._launch(self.slot)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def autotune(self, frames, t: int | None = None, reps: int = 3, candidates=TILES):
        """Pick a training tile per spp group: for each group in turn, time
        the whole batched frame with each candidate tile for that group (the
        other groups keep their current choice) and keep the fastest.  Only
        the group's own launch changes between candidates, so the differences
        are that launch's.  Returns {spp: {tile: ms}}."""
        t = self.frame if t is None else t
        groups = sorted({s["spp"] for s in self.specs})
        chosen = {spp: self.tile_of(spp) for spp in groups}
        chosen = {spp: (tl if tl != (0, 0) else None) for spp, tl in chosen.items()}
        out = {}
        for spp in groups:
            times = {}
            for tile in candidates:
                # a tile that does not fit this spp's LDS would fall back to
                # the default tile: skip it
                if _tile_lds(tile, spp) > 64 * 1024:
                    continue
                self.tile = {g: (tile if g == spp else chosen[g]) for g in groups if (g == spp or chosen[g])}
                ms = self._time_frame(frames, t, reps)
                if ms is not None:
                    times[tile] = ms
            if times:
                chosen[spp] = min(times, key=times.get)
            out[spp] = times
        self.tile = {g: tl for g, tl in chosen.items() if tl}
        self.graphs = [None, None]  # captured with the previous tiles
        return out


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
