"""Pins of the oracle's positional reuse of virtual point lights and of the
near-field workload it is measured on (CPU only).

A pixel trains on its neighbours' samples along the direction from its own
position to each sample's next surface interaction y = x_q + t w_q (Fig. 2
caption): for a point light every such direction is exactly the direction
to the light, so positional reuse learns the lobe of each pixel without the
offset of its neighbours, which reusing the neighbours' directions cannot."""
import numpy as np
import pytest

import oracle as O
from paper_2112_09728_amd import workload as wl
from test_oracle_frame import _flat_scene, _hemisphere_grid


def _grid_positions(W, H, z=0.0):
    X, Y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    return np.stack([X, Y, np.full_like(X, z)]).astype(np.float32)


def _point_light_records(W, H, spp, light, rough=0.6):
    """Flat scene whose every sample is a BRDF draw aimed at one point light
    (its direction, distance and a unit radiance)."""
    sc = _flat_scene(W, H, rough=rough)
    pos = _grid_positions(W, H)
    d = np.asarray(light, float)[:, None, None] - pos.astype(float)
    t = np.sqrt((d * d).sum(0))
    w = d / t
    wo = sc["view_dir"][:, 0, 0].astype(float)
    pb = O.brdf_pdf(wo, w.reshape(3, -1).T, rough ** 2).reshape(H, W)
    rec = dict(dir=np.repeat(w[:, None], spp, 1), pdf_brdf=np.repeat(pb[None], spp, 0),
               strategy=np.ones((spp, H, W), np.uint8), radiance=np.ones((spp, H, W)),
               hit_dist=np.repeat(t[None], spp, 0))
    return sc, pos, rec


def _target_mu(sc, pos, light):
    """M^-1 of the local direction from each pixel to the light (normal +z)."""
    d = np.asarray(light, float)[:, None, None] - pos.astype(float)
    d /= np.sqrt((d * d).sum(0))
    return O.hemi2sq(d.reshape(3, -1).T).T.reshape(2, *pos.shape[1:])


def test_positional_reuse_learns_each_pixels_own_direction():
    """From a new model (one EM step, no clamp), every pixel's lobe mean is
    exactly M^-1 of its own direction to the light with positional reuse; with
    the neighbours' directions reused as they are it is off by the spread of
    the 7x7 window's directions (> 1e-3 near the light)."""
    W, H, spp, K = 21, 17, 2, 1
    light = (10.5, 8.5, 6.0)
    sc, pos, rec = _point_light_records(W, H, spp, light)
    v = O.OView(sc)
    P = O.params(31, frame=0, flags=1)
    g0, _ = O.reproject_k(P, K, v, None, None)
    g_pos = O.em_vpl(P, K, v, pos, rec, g0)
    g_dir = O.em_k(P, K, v, rec, g0)
    mu = _target_mu(sc, pos, light)
    assert (g_pos[7] == 1).all()
    assert np.abs(g_pos[:2] - mu).max() < 1e-9
    near = np.zeros((H, W), bool)
    near[4:13, 6:15] = True
    err_dir = np.abs(g_dir[:2] - mu).max(0)
    assert err_dir[near].min() > 1e-3, err_dir[near].min()
    # the collapsed batch has no scatter: Sigma is the regulariser's alone
    assert np.abs(g_pos[2:5]).max() < 1e-12


def test_infinite_hit_distance_is_the_directional_update():
    """t = +inf everywhere (every light at infinity) gives the update that
    reuses the neighbours' directions, bit for bit, for K = 1 and 2."""
    W, H, spp = 23, 19, 2
    sc, pos, rec = _point_light_records(W, H, spp, (11.5, 9.5, 6.0))
    rng = np.random.default_rng(3)
    rec["radiance"] = rng.uniform(0.5, 2.0, rec["radiance"].shape)
    rec["hit_dist"] = np.full(rec["hit_dist"].shape, np.inf)
    v = O.OView(sc)
    for K in (1, 2):
        P = O.params(32, frame=2)
        g0, _ = O.reproject_k(P, K, v, None, None)
        g0[6 * K + 1] = 2.0
        g0[6 * K] = 1.5
        np.testing.assert_array_equal(O.em_vpl(P, K, v, pos, rec, g0), O.em_k(P, K, v, rec, g0))


def test_own_samples_train_along_their_own_direction():
    """With every neighbour's sample guided (never trains), only own samples
    remain, and y - x_p = t w: positional and directional reuse agree."""
    W, H, spp = 15, 13, 3
    sc, pos, rec = _point_light_records(W, H, spp, (7.5, 6.5, 5.0))
    rec["strategy"][:] = 2
    rec["strategy"][:, 6, 7] = 1
    v = O.OView(sc)
    P = O.params(33, frame=1)
    g0, _ = O.reproject_k(P, 2, v, None, None)
    a, b = O.em_vpl(P, 2, v, pos, rec, g0), O.em_k(P, 2, v, rec, g0)
    assert a[13, 6, 7] == 1
    np.testing.assert_allclose(a[:, 6, 7], b[:, 6, 7], rtol=1e-12, atol=1e-14)
    # its neighbours that picked its samples train along other directions
    nb = (a[13] == 1)
    nb[6, 7] = False
    assert nb.sum() >= 5 and (np.abs(a[:2] - b[:2]).max(0)[nb] > 1e-3).all()


def test_ceiling_light_field():
    """Hit points lie on the plane; a direction at a lamp's centre sees the
    lamp's intensity plus the tails of the others (summed here over every lamp
    of the table); rays at or below the horizontal leave the scene with the
    ambient term; null samples carry nothing."""
    W, H = 40, 30
    sc = wl.make_scene(W, H, 77, margin=16)
    sc = wl.crop_scene(sc, 0, 0, W, H)
    ceil = sc["ceiling"]
    pos = sc["position"].astype(float)
    v = O.OView(sc)
    lamps = ceil["lamps"].reshape(-1, 4).astype(float)
    rng = np.random.default_rng(5)
    # a direction from each pixel at a random lamp's centre, one random direction
    pick = rng.integers(0, lamps.shape[0], (H, W))
    tgt = np.stack([lamps[pick, 0], lamps[pick, 1], np.full((H, W), ceil["z"])])
    d0 = tgt - pos
    d0 /= np.sqrt((d0 * d0).sum(0))
    d1 = rng.normal(size=(3, H, W))
    d1 /= np.sqrt((d1 * d1).sum(0))
    dirs = np.stack([d0, d1], 1)
    strat = np.ones((2, H, W), np.uint8)
    strat[1, ::3] = 3
    L, t = O.light_ceiling(ceil, v, sc["position"], dirs, strat)
    up = (dirs[2] > 0) & (strat == 1)
    y = pos[:, None] + t[None] * dirs
    assert np.abs(y[2][up] - ceil["z"]).max() < 1e-9
    full = ceil["ambient"] + sum(c * np.exp(-((y[0] - sx) ** 2 + (y[1] - sy) ** 2) / (2 * r * r))
                                 for sx, sy, r, c in lamps)
    # (the lamps beyond the 3x3 cells around y add less than 1e-9 relative)
    np.testing.assert_allclose(L[up], full[up], rtol=1e-9)
    assert (L[0] >= lamps[pick, 3] + ceil["ambient"] - 1e-9).all()
    down = (dirs[2] <= 0) & (strat == 1)
    assert down.any() and np.isinf(t[down]).all() and (L[down] == np.float64(ceil["ambient"])).all()
    assert (L[strat == 3] == 0).all() and (t[strat == 3] == 0).all()


@pytest.mark.parametrize("rough", [0.7, 0.4])
def test_ceiling_reference_against_quadrature(rough):
    """The BRDF-sampling reference of int f_r E cos under the ceiling equals a
    hemisphere quadrature of the same integrand within 5 standard errors."""
    sc = _flat_scene(1, 1, rough=rough)
    pos = np.array([24.0, 24.0, 0.0], np.float32)[:, None, None]
    ceil = dict(z=32.0, period=48.0, x0=-48.0, y0=-48.0, ambient=0.05,
                lamps=np.array([[[10.0, 20.0, 6.0, 20.0], [60.0, 16.0, 5.0, 10.0], [110.0, 30.0, 7.0, 15.0]],
                                [[14.0, 70.0, 4.0, 25.0], [70.0, 80.0, 8.0, 5.0], [100.0, 60.0, 3.0, 30.0]],
                                [[20.0, 120.0, 6.0, 20.0], [60.0, 110.0, 5.0, 12.0], [120.0, 110.0, 7.0, 8.0]]],
                               np.float32))
    v = O.OView(sc)
    m, se = O.reference_ceiling(O.params(9, frame=0), v, pos, ceil, [0], 65536)
    dirs, wts = _hemisphere_grid(400, 400)
    st = np.ones((dirs.shape[0], 1, 1), np.uint8)
    L, _ = O.light_ceiling(ceil, v, pos, dirs.T.reshape(3, -1, 1, 1), st)
    wo = sc["view_dir"][:, 0, 0].astype(float)
    truth = (O.brdf_f(wo, dirs, rough ** 2, float(np.float32(0.6))) * L.reshape(-1) * dirs[:, 2] * wts).sum()
    assert abs(m[0] - truth) < 5 * se[0], (m[0], truth, se[0])
    assert se[0] < 0.02 * truth
