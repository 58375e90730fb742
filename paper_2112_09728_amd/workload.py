"""Seeded synthetic inputs for the path-guiding hot path.

The paper renders its own scenes (Sponza, Bistro Exterior, San Miguel, Glossy
Sponza; Sec. 4) with a ray tracer; none of that is available here, so these
generators stand in for the rasterised G-buffer, the camera motion and the
traced radiance with seeded synthetic data of the same shape:

* a G-buffer from a smooth value-noise heightfield (normals from its analytic
  gradient, tilt at most 35 degrees), a pinhole view direction above the
  plane, per-pixel roughness U[0.05, 1] and albedo U[0.2, 0.9];
* three spherical-Gaussian lights (axis uniform on the upper hemisphere,
  sharpness U[10, 200], intensity U[1, 20]), ambient 0.05, and a binary
  visibility bit per (pixel, light) with probability 1/2;
* per frame (``Sequence``): a camera pan.  The G-buffer is a window onto a
  larger world texture; the window moves by a step drawn from U[-2, 2]^2 px
  (quantised to 1/256 px) each frame, so every pixel's motion vector is the
  pan step, the G-buffer of frame t is the nearest world texel under each
  pixel, and a 2% disocclusion mask (none at frame 0) marks pixels whose
  history is discarded.  ``make_motion`` instead draws independent motion
  per pixel over a static G-buffer, a harder case for the reprojection
  gather used by the tests;
* for the positional reuse of virtual point lights, each texel's world
  position (x + 1/2, y + 1/2, height) and a near-field emitter above the
  surface (``make_ceiling``): the plane z = 32 with a jittered lattice of
  Gaussian lamps (period 48 texels, radius U[3, 8], intensity U[2, 30]).

This module holds no arithmetic of the method itself: it only draws inputs.
Both the GPU path and the CPU oracle consume the arrays it returns.
"""
from __future__ import annotations

import numpy as np

AMBIENT = 0.05
N_LIGHTS = 3
SEED_BASE = 211209728

# stream ids of the generator (kept apart so that each input is independent)
_S_HEIGHT, _S_MATERIAL, _S_LIGHTS, _S_VIS, _S_MOTION, _S_MASK, _S_CEILING = 2, 3, 4, 5, 6, 7, 8


def _rng(seed: int, stream: int, frame: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, stream, frame])))


def _value_noise(width: int, height: int, cell: float, rng: np.random.Generator):
    """Value noise with quintic fade on a lattice of spacing ``cell`` px.

    Returns (h, dh/dx, dh/dy) sampled at pixel centres, in float64."""
    nx = int(np.ceil(width / cell)) + 2
    ny = int(np.ceil(height / cell)) + 2
    lat = rng.uniform(-1.0, 1.0, size=(ny, nx))
    xs = (np.arange(width) + 0.5) / cell
    ys = (np.arange(height) + 0.5) / cell
    ix = np.floor(xs).astype(np.int64)
    iy = np.floor(ys).astype(np.int64)
    tx = xs - ix
    ty = ys - iy
    fx = tx * tx * tx * (tx * (6 * tx - 15) + 10)
    fy = ty * ty * ty * (ty * (6 * ty - 15) + 10)
    dfx = 30 * tx * tx * (tx - 1) ** 2
    dfy = 30 * ty * ty * (ty - 1) ** 2
    v00 = lat[iy[:, None], ix[None, :]]
    v10 = lat[iy[:, None], ix[None, :] + 1]
    v01 = lat[iy[:, None] + 1, ix[None, :]]
    v11 = lat[iy[:, None] + 1, ix[None, :] + 1]
    FX, FY = fx[None, :], fy[:, None]
    a = v00 + (v10 - v00) * FX
    b = v01 + (v11 - v01) * FX
    h = a + (b - a) * FY
    dx = ((v10 - v00) * (1 - FY) + (v11 - v01) * FY) * dfx[None, :] / cell
    dy = (b - a) * dfy[:, None] / cell
    return h, dx, dy


def make_scene(width: int, height: int, seed: int, margin: int = 0) -> dict:
    """Static G-buffer, lights and visibility of one synthetic view.

    Arrays are float32 (uint8 for ``vis``), laid out [channel][H][W].  With a
    margin the surface arrays cover (H + 2 margin) x (W + 2 margin) texels
    while the view direction stays that of the W x H screen."""
    sw, sh = width, height
    width, height = width + 2 * margin, height + 2 * margin
    rng_h = _rng(seed, _S_HEIGHT)
    h = np.zeros((height, width))
    gx = np.zeros((height, width))
    gy = np.zeros((height, width))
    amp = 2.5
    for octave in range(3):
        cell = 32.0 * 2.0 ** (-octave)
        vh, vx, vy = _value_noise(width, height, cell, rng_h)
        w = amp * 2.0 ** (-octave)
        h += w * vh
        gx += w * vx
        gy += w * vy
    # limit the tilt of the surface to 35 degrees
    slope = np.sqrt(gx * gx + gy * gy)
    lim = np.tan(np.radians(35.0))
    scale = np.where(slope > lim, lim / np.maximum(slope, 1e-30), 1.0)
    gx *= scale
    gy *= scale
    n = np.stack([-gx, -gy, np.ones_like(gx)])
    n /= np.sqrt((n * n).sum(0, keepdims=True))
    depth = 1000.0 - h
    wx, wy = np.meshgrid(np.arange(width) + 0.5, np.arange(height) + 0.5)
    position = np.stack([wx, wy, h])
    xs = np.arange(sw) + 0.5
    ys = np.arange(sh) + 0.5
    cam_h = float(max(sw, sh))
    vd = np.stack(np.broadcast_arrays(sw / 2.0 - xs[None, :], sh / 2.0 - ys[:, None],
                                      np.full((sh, sw), cam_h)))
    vd = vd / np.sqrt((vd * vd).sum(0, keepdims=True))
    rng_m = _rng(seed, _S_MATERIAL)
    roughness = rng_m.uniform(0.05, 1.0, size=(height, width))
    albedo = rng_m.uniform(0.2, 0.9, size=(height, width))
    rng_l = _rng(seed, _S_LIGHTS)
    z = rng_l.uniform(0.0, 1.0, size=N_LIGHTS)
    phi = rng_l.uniform(0.0, 2 * np.pi, size=N_LIGHTS)
    s = np.sqrt(1.0 - z * z)
    axis = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    sharp = rng_l.uniform(10.0, 200.0, size=N_LIGHTS)
    inten = rng_l.uniform(1.0, 20.0, size=N_LIGHTS)
    lights = np.concatenate([axis, sharp[:, None], inten[:, None]], axis=1).astype(np.float32)
    rng_v = _rng(seed, _S_VIS)
    bits = rng_v.integers(0, 2, size=(N_LIGHTS, height, width), dtype=np.uint8)
    vis = np.zeros((height, width), np.uint8)
    for k in range(N_LIGHTS):
        vis |= bits[k] << k
    return dict(
        width=sw, height=sh, seed=seed, margin=margin,
        normal=n.astype(np.float32),
        view_dir=vd.astype(np.float32),
        depth=depth.astype(np.float32),
        roughness=roughness.astype(np.float32),
        albedo=albedo.astype(np.float32),
        lights=lights, ambient=np.float32(AMBIENT), vis=vis,
        position=position.astype(np.float32),
        ceiling=make_ceiling(width, height, seed),
    )


def make_ceiling(width: int, height: int, seed: int, z: float = 32.0, period: float = 48.0) -> dict:
    """Near-field emitter over a world of width x height texels: the plane at
    height z, lamps on a lattice of the given period covering the world and
    one cell beyond each edge, each lamp at a uniform position in the middle
    half of its cell with radius U[3, 8] and intensity U[2, 30].  lamps
    [ny][nx][4] float32 holds (sx, sy, r, c)."""
    rng = _rng(seed, _S_CEILING)
    x0 = y0 = -period
    nx = int(np.ceil((width + 2 * period) / period))
    ny = int(np.ceil((height + 2 * period) / period))
    sx = x0 + (np.arange(nx)[None, :] + rng.uniform(0.25, 0.75, (ny, nx))) * period
    sy = y0 + (np.arange(ny)[:, None] + rng.uniform(0.25, 0.75, (ny, nx))) * period
    r = rng.uniform(3.0, 8.0, (ny, nx))
    c = rng.uniform(2.0, 30.0, (ny, nx))
    return dict(z=z, period=period, x0=x0, y0=y0, ambient=AMBIENT,
                lamps=np.stack([sx, sy, r, c], -1).astype(np.float32))


def make_motion(width: int, height: int, seed: int, frame: int, moving: bool = True,
                disocc_rate: float = 0.02):
    """Motion vectors [2][H][W] (px, dyadic 1/256) and the disocclusion mask.

    Frame 0 and ``moving=False`` give zero motion and no disocclusion."""
    if not moving or frame == 0:
        return np.zeros((2, height, width), np.float32), np.zeros((height, width), np.uint8)
    rng = _rng(seed, _S_MOTION, frame)
    mv = np.round(rng.uniform(-2.0, 2.0, size=(2, height, width)) * 256.0) / 256.0
    rng_m = _rng(seed, _S_MASK, frame)
    mask = (rng_m.uniform(0.0, 1.0, size=(height, width)) < disocc_rate).astype(np.uint8)
    return mv.astype(np.float32), mask


class Sequence:
    """Frames of a camera pan over a static world (see the module docstring).

    ``frame(t)`` returns a scene dict for frame t with ``motion`` [2][H][W]
    (px, current minus previous position, the same for every pixel) and
    ``disocc`` [H][W]; frames must be requested in order 0, 1, 2, ..."""

    def __init__(self, width: int, height: int, seed: int, moving: bool = True,
                 disocc_rate: float = 0.02, margin: int = 64, light_moves_at: int | None = None):
        self.width, self.height, self.seed = width, height, seed
        self.moving, self.disocc_rate, self.margin = moving, disocc_rate, margin
        self.light_moves_at = light_moves_at
        self.world = make_scene(width, height, seed, margin=margin if moving else 0)
        self.offset = np.zeros(2)
        self.t = -1

    def _window(self, ox: float, oy: float) -> dict:
        W, H, M = self.width, self.height, self.world["margin"]
        ix = np.floor(np.arange(W) + 0.5 + ox).astype(np.int64) + M
        iy = np.floor(np.arange(H) + 0.5 + oy).astype(np.int64) + M
        out = dict(self.world)
        out["width"], out["height"] = W, H
        for key in ("normal", "position"):
            out[key] = np.ascontiguousarray(self.world[key][:, iy[:, None], ix[None, :]])
        for key in ("depth", "roughness", "albedo", "vis"):
            out[key] = np.ascontiguousarray(self.world[key][iy[:, None], ix[None, :]])
        return out

    def frame(self, t: int) -> dict:
        if t != self.t + 1:
            raise ValueError("frames of a Sequence are generated in order")
        self.t = t
        W, H = self.width, self.height
        step = np.zeros(2)
        mask = np.zeros((H, W), np.uint8)
        if self.moving and t > 0:
            rng = _rng(self.seed, _S_MOTION, t)
            step = np.round(rng.uniform(-2.0, 2.0, size=2) * 256.0) / 256.0
            lim = self.margin - 3
            new = np.clip(self.offset + step, -lim, lim)
            step = new - self.offset
            self.offset = new
            rng_m = _rng(self.seed, _S_MASK, t)
            mask = (rng_m.uniform(0.0, 1.0, size=(H, W)) < self.disocc_rate).astype(np.uint8)
        out = self._window(*self.offset)
        # content moves opposite to the window: motion = -(window step)
        out["motion"] = np.broadcast_to((-step).astype(np.float32)[:, None, None], (2, H, W)).copy()
        out["disocc"] = mask
        if self.light_moves_at is not None and t >= self.light_moves_at:
            # the most powerful light (power of an SG lobe ~ c / lambda) jumps
            # to a new direction on the upper hemisphere (a dynamic light:
            # trained lobes become stale)
            lights = np.array(out["lights"], np.float32, copy=True)
            k = int(np.argmax(lights[:, 4] / lights[:, 3]))
            rng = _rng(self.seed, _S_MOTION, 10_000)
            z = rng.uniform(0.3, 0.95)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            new = np.array([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z])
            if np.dot(new, lights[k, :3]) > 0.5:  # make it a real jump
                new[:2] = -new[:2]
            lights[k, :3] = new.astype(np.float32)
            out["lights"] = lights
        return out


def batched_views(n_views: int, sizes, spp_range, seed: int):
    """Views of a batched workload: size uniform over `sizes`, spp uniform
    over spp_range (inclusive), one seed per view.  Returns [(W, H, spp, seed)]."""
    rng = np.random.default_rng([seed, 0xBA7C4])
    out = []
    for i in range(n_views):
        w, h = sizes[int(rng.integers(len(sizes)))]
        spp = int(rng.integers(spp_range[0], spp_range[1] + 1))
        out.append((int(w), int(h), spp, seed + 1000 * (i + 1)))
    return out


def sequence_frames(width: int, height: int, seed: int, n_frames: int, moving: bool = True) -> list:
    """Frames 0 .. n_frames - 1 of one camera-pan Sequence."""
    seq = Sequence(width, height, seed, moving=moving)
    return [seq.frame(t) for t in range(n_frames)]


def many_sequence_frames(views, n_frames: int, workers: int = 8) -> list:
    """sequence_frames for many views [(width, height, seed)] in worker
    processes (spawned, so that they share nothing with a process that has
    initialised a GPU); returns one list of frames per view, in order."""
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=max(1, min(workers, len(views))),
                                mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(sequence_frames, w, h, sd, n_frames) for (w, h, sd) in views]
        return [f.result() for f in futs]


def crop_scene(scene: dict, x0: int, y0: int, x1: int, y1: int) -> dict:
    """A sub-rectangle of a scene as a scene of its own (same lights)."""
    out = dict(scene)
    for key in ("normal", "view_dir", "position"):
        if key in scene:
            out[key] = np.ascontiguousarray(scene[key][:, y0:y1, x0:x1])
    for key in ("depth", "roughness", "albedo", "vis"):
        out[key] = np.ascontiguousarray(scene[key][y0:y1, x0:x1])
    out["width"], out["height"] = x1 - x0, y1 - y0
    return out


# Workloads of the hot path, named by what they are.
CONFIGS = {
    "64x64_spp1_8f_fp32_static": dict(width=64, height=64, spp=1, frames=8, moving=False,
                                      gamma_dtype="f32", seed=SEED_BASE + 1),
    "1080p_spp1_64f_fp32_pan": dict(width=1920, height=1080, spp=1, frames=64, moving=True,
                                    gamma_dtype="f32", seed=SEED_BASE + 2,
                                    crop=(832, 412, 1088, 668)),
    "1080p_4k_spp1_64f_fp16_bf16": dict(sizes=((1920, 1080), (3840, 2160)), spp=1, frames=64,
                                        moving=True, gamma_dtype=("f16", "bf16"),
                                        seed=SEED_BASE + 3),
    "4k_spp4_gradient_fit": dict(width=3840, height=2160, spp=4, frames=1, moving=False,
                                 gamma_dtype="f32", seed=SEED_BASE + 4,
                                 fd_crop=(1904, 1064, 1936, 1096)),
    "batched_16_views": dict(n_views=16, sizes=((640, 360), (1280, 720), (1920, 1080),
                                                (2560, 1440), (3840, 2160)),
                             spp_range=(1, 8), frames=64, moving=True, gamma_dtype="f16",
                             seed=SEED_BASE + 5),
}
