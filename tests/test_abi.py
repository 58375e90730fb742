"""C ABI contract checks that need no GPU: the library loads, exports every
entry point its header declares, and rejects bad arguments on the host with
the documented status before any launch."""
import ctypes as C
import os
import re

import pytest
import torch

import paper_2112_09728_amd as pg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmmguide.h")

# With a live device a call that passed validation would launch on the fake
# pointers below; these checks therefore run only where no GPU is present.
no_device = pytest.mark.skipif(torch.cuda.is_available(),
                               reason="error-path probes use fake pointers; CPU-only")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:pg_status|const char \*|size_t)\s*(pg_\w+)\(", src, re.M)))


def test_header_declarations_are_exported():
    names = declared_functions()
    assert len(names) >= 10
    L = pg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(pg.EXPORTS) == set(names)


def test_params_default_matches_paper_constants():
    p = pg.params(9)
    assert p.k_max == 16 and p.radius == 3
    assert p.pi_init == pytest.approx(0.05) and p.pi_lo == pytest.approx(0.05)
    assert p.pi_hi == pytest.approx(0.95)


FAKE = 0x10000  # never dereferenced: every call below fails validation first


def _view(w=8, h=4, pitch=None, albedo=True):
    return pg.PgView(w, h, w if pitch is None else pitch, FAKE, FAKE, FAKE, FAKE,
                     FAKE if albedo else None, None, None)


def _samples(spp=1, radiance=True):
    return pg.PgSamples(spp, FAKE, FAKE, FAKE, FAKE, FAKE if radiance else None)


def _status(fn, *args):
    st = fn(*args)
    return st, pg.lib().pg_last_error().decode()


@no_device
def test_argument_errors_before_launch():
    L = pg.lib()
    P = pg.params(1, frame=1)
    v = _view()
    g = pg.PgGamma(pg.PG_F32, FAKE)
    g2 = pg.PgGamma(pg.PG_F32, FAKE + 4096)
    s = _samples()
    cases = [
        (L.pg_reproject, (None, C.byref(v), C.byref(v), g, g2, None, None), pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(v), C.byref(v), g, g, None, None), pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(v), None, g, g2, None, None), pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(_view(pitch=4)), C.byref(v), g, g2, None, None),
         pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(_view(w=0)), C.byref(v), g, g2, None, None),
         pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(v), C.byref(v), g, pg.PgGamma(7, FAKE), None, None),
         pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(v), C.byref(v), pg.PgGamma(pg.PG_F16, FAKE), g2, None,
                          None), pg.PG_ERR_ARG),
        (L.pg_reproject, (C.byref(P), C.byref(_view(w=20000)), C.byref(v), g, g2, None, None),
         pg.PG_ERR_UNSUPPORTED),
        # row offsets are 24-bit products: a pitch of 2^24 is refused
        (L.pg_reproject, (C.byref(P), C.byref(_view(h=1, pitch=1 << 24)), C.byref(_view(h=1, pitch=1 << 24)), g, g2,
                          None, None), pg.PG_ERR_UNSUPPORTED),
        (L.pg_sample_mis, (C.byref(P), C.byref(v), g, C.byref(_samples(spp=0)), None), pg.PG_ERR_ARG),
        (L.pg_sample_mis, (C.byref(P), C.byref(v), g, C.byref(_samples(spp=9)), None), pg.PG_ERR_ARG),
        (L.pg_sample_mis, (C.byref(P), C.byref(v), pg.PgGamma(0, None), C.byref(s), None),
         pg.PG_ERR_ARG),
        (L.pg_pdf, (C.byref(P), C.byref(v), g, 0, FAKE, FAKE, None, None, None), pg.PG_ERR_ARG),
        (L.pg_pdf, (C.byref(P), C.byref(v), g, 1, None, FAKE, None, None, None), pg.PG_ERR_ARG),
        (L.pg_em_update, (C.byref(P), C.byref(v), C.byref(s), g, 2, None), pg.PG_ERR_ARG),
        (L.pg_em_update, (C.byref(P), C.byref(_view(albedo=False)), C.byref(s), g, 1, None),
         pg.PG_ERR_ARG),
        (L.pg_em_update, (C.byref(P), C.byref(v), C.byref(_samples(radiance=False)), g, 1, None),
         pg.PG_ERR_ARG),
        (L.pg_nll_backward, (C.byref(P), C.byref(v), C.byref(s), None, None, FAKE, FAKE, None),
         pg.PG_ERR_ARG),
        (L.pg_nll_backward, (C.byref(P), C.byref(v), C.byref(s), FAKE, None, None, None, None),
         pg.PG_ERR_ARG),
        (L.pg_estimate, (C.byref(P), C.byref(v), C.byref(s), None, None), pg.PG_ERR_ARG),
        (L.pg_estimate, (C.byref(P), C.byref(_view(albedo=False)), C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_estimate, (C.byref(P), C.byref(v), C.byref(_samples(radiance=False)), FAKE, None),
         pg.PG_ERR_ARG),
        (L.pg_philox, (-1, None, 0, None, None), pg.PG_ERR_ARG),
    ]
    for fn, args, want in cases:
        st, msg = _status(fn, *args)
        assert st == want, (fn.__name__, st, msg)
        assert msg, fn.__name__
    Pr = pg.params(1, frame=1, radius=2)
    assert _status(L.pg_reproject, C.byref(Pr), C.byref(v), C.byref(v), g, g2, None, None)[0] == \
        pg.PG_ERR_UNSUPPORTED
    Pt = pg.params(1, frame=1, tile_w=24, tile_h=24)
    assert _status(L.pg_em_update, C.byref(Pt), C.byref(v), C.byref(s), g, 1, None)[0] == \
        pg.PG_ERR_UNSUPPORTED
    Pb = pg.params(1, frame=1, flags=pg.PG_EM_BATCH)
    assert _status(L.pg_em_update, C.byref(Pb), C.byref(v), C.byref(s), g, 0, None)[0] == pg.PG_ERR_ARG
    lights = pg.PgLights()
    lights.count = 9
    assert _status(L.pg_light_field, C.byref(lights), C.byref(v), FAKE, C.byref(s), None)[0] == \
        pg.PG_ERR_ARG
    # the zero-size diagnostic call succeeds without touching a device
    assert L.pg_philox(0, None, 0, None, None) == pg.PG_OK
    assert pg.lib().pg_last_error().decode() == ""


@no_device
def test_lobes_argument_errors_before_launch():
    L = pg.lib()
    P = pg.params(1, frame=1)
    v = _view()
    s = _samples()
    big = _view(w=16384, h=5100)   # 26 planes pass 2^31 at K = 4 (24 do not)
    other = _view(w=9)
    cases = [
        (L.pg_em_update_lobes, (C.byref(P), 0, C.byref(v), C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_em_update_lobes, (C.byref(P), 5, C.byref(v), C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_em_update_lobes, (C.byref(P), 2, C.byref(v), C.byref(s), None, None), pg.PG_ERR_ARG),
        (L.pg_em_update_lobes, (C.byref(P), 2, C.byref(_view(albedo=False)), C.byref(s), FAKE, None),
         pg.PG_ERR_ARG),
        (L.pg_em_update_lobes, (C.byref(pg.params(1, flags=pg.PG_EM_BATCH)), 2, C.byref(v), C.byref(s), FAKE,
                                None), pg.PG_ERR_UNSUPPORTED),
        (L.pg_em_update_lobes, (C.byref(pg.params(1, flags=pg.PG_STALE_RESET)), 2, C.byref(v), C.byref(s),
                                FAKE, None), pg.PG_ERR_UNSUPPORTED),
        (L.pg_em_update_lobes, (C.byref(P), 4, C.byref(big), C.byref(s), FAKE, None), pg.PG_ERR_UNSUPPORTED),
        (L.pg_reproject_sample_lobes, (C.byref(P), 2, C.byref(v), C.byref(v), FAKE, FAKE, C.byref(s), None),
         pg.PG_ERR_ARG),
        (L.pg_reproject_sample_lobes, (C.byref(P), 2, C.byref(v), None, FAKE, FAKE + 4096, C.byref(s), None),
         pg.PG_ERR_ARG),
        (L.pg_reproject_sample_lobes, (C.byref(P), 2, C.byref(v), C.byref(v), None, FAKE, C.byref(s), None),
         pg.PG_ERR_ARG),
        (L.pg_reproject_sample_lobes, (C.byref(P), 2, C.byref(v), C.byref(other), FAKE, FAKE + 4096,
                                       C.byref(s), None), pg.PG_ERR_UNSUPPORTED),
        (L.pg_reproject_sample_lobes, (C.byref(P), 2, C.byref(v), C.byref(v), FAKE, None, C.byref(s), None),
         pg.PG_ERR_ARG),
        (L.pg_pdf_lobes, (C.byref(P), 2, C.byref(v), FAKE, 0, FAKE, FAKE, None), pg.PG_ERR_ARG),
        (L.pg_pdf_lobes, (C.byref(P), 2, C.byref(v), FAKE, 1, None, FAKE, None), pg.PG_ERR_ARG),
        (L.pg_pdf_lobes, (C.byref(P), 2, C.byref(v), None, 1, FAKE, FAKE, None), pg.PG_ERR_ARG),
        (L.pg_pdf_lobes, (C.byref(P), -1, C.byref(v), FAKE, 1, FAKE, FAKE, None), pg.PG_ERR_ARG),
    ]
    for fn, args, want in cases:
        st, msg = _status(fn, *args)
        assert st == want, (fn.__name__, st, msg)
        assert msg, fn.__name__


@no_device
def test_vpl_argument_errors_before_launch():
    L = pg.lib()
    P = pg.params(1, frame=1)
    v = _view()
    s = _samples()
    c = pg.PgCeiling(32.0, 48.0, -48.0, -48.0, 0.05, 4, 3, FAKE)
    cases = [
        (L.pg_em_update_vpl, (C.byref(P), 1, C.byref(v), None, C.byref(s), FAKE, FAKE, None), pg.PG_ERR_ARG),
        (L.pg_em_update_vpl, (C.byref(P), 1, C.byref(v), FAKE, C.byref(s), None, FAKE, None), pg.PG_ERR_ARG),
        (L.pg_em_update_vpl, (C.byref(P), 0, C.byref(v), FAKE, C.byref(s), FAKE, FAKE, None), pg.PG_ERR_ARG),
        (L.pg_em_update_vpl, (C.byref(P), 1, C.byref(v), FAKE, C.byref(s), FAKE, None, None), pg.PG_ERR_ARG),
        (L.pg_em_update_vpl, (C.byref(pg.params(1, flags=pg.PG_EM_BATCH)), 1, C.byref(v), FAKE, C.byref(s), FAKE,
                              FAKE, None), pg.PG_ERR_UNSUPPORTED),
        (L.pg_light_ceiling, (None, C.byref(v), FAKE, C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_light_ceiling, (C.byref(pg.PgCeiling(32.0, 48.0, 0, 0, 0.05, 0, 3, FAKE)), C.byref(v), FAKE,
                              C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_light_ceiling, (C.byref(pg.PgCeiling(32.0, 0.0, 0, 0, 0.05, 4, 3, FAKE)), C.byref(v), FAKE,
                              C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_light_ceiling, (C.byref(pg.PgCeiling(32.0, 48.0, 0, 0, 0.05, 4, 3, FAKE + 4)), C.byref(v), FAKE,
                              C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_light_ceiling, (C.byref(c), C.byref(v), None, C.byref(s), FAKE, None), pg.PG_ERR_ARG),
        (L.pg_light_ceiling, (C.byref(c), C.byref(v), FAKE, C.byref(s), None, None), pg.PG_ERR_ARG),
        (L.pg_light_ceiling, (C.byref(c), C.byref(v), FAKE, C.byref(_samples(radiance=False)), FAKE, None),
         pg.PG_ERR_ARG),
    ]
    for fn, args, want in cases:
        st, msg = _status(fn, *args)
        assert st == want, (fn.__name__, st, msg)
        assert msg, fn.__name__


def test_pick_division_identity():
    """The training kernel divides a pick code c < 48 spp by spp as
    (c * ceil(2^16/spp)) >> 16; exact for every code it can meet."""
    for spp in range(1, 9):
        m = (65536 + spp - 1) // spp
        for c in range(48 * spp):
            assert (c * m) >> 16 == c // spp


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(pg, "_lib", None)
    monkeypatch.setattr(pg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(pg.LibraryMissing):
        pg.lib()


def _bview(w=8, h=4, spp=1, frame=1, dtype=pg.PG_F32, base=0, **params):
    """A batch view on fake pointers (pg_batch_pack only validates and packs)."""
    b = pg.PgBatchView()
    b.params = pg.params(3, frame=frame, **params)
    b.cur = _view(w, h)
    b.prev = _view(w, h)
    b.gamma_in = pg.PgGamma(dtype, FAKE + base + 1024)
    b.gamma_out = pg.PgGamma(dtype, FAKE + base + 2048)
    b.samples = pg.PgSamples(spp, FAKE + base + 4096, FAKE, FAKE, FAKE, FAKE)
    b.vis = FAKE
    b.lights.count = 1
    return b


def _pack(views, nbytes=None):
    n = len(views)
    nbytes = pg.batch_table_bytes(n) if nbytes is None else nbytes
    table = torch.zeros(max(nbytes, 1), dtype=torch.uint8)
    arr = (pg.PgBatchView * n)(*views) if n else None
    st = pg.lib().pg_batch_pack(arr, n, C.c_void_p(table.data_ptr()), nbytes)
    return st, pg.lib().pg_last_error().decode(), table


def test_batch_pack_layout_and_tile_counts():
    """Host-only packing: the header counts the 64x4 sampling tiles and the
    training tiles of every view (the requested tile where it fits the view's
    spp) and groups the views by spp."""
    sizes = [(70, 37, 1), (129, 64, 3), (33, 95, 8), (640, 360, 2), (40, 40, 3)]
    views = [_bview(w, h, spp, base=i << 16, tile_w=32, tile_h=8) for i, (w, h, spp) in enumerate(sizes)]
    st, msg, table = _pack(views)
    assert st == pg.PG_OK, msg
    n, rs, em, dtype, n_classes, magic = table[:24].view(torch.int32).tolist()
    assert (n, dtype, n_classes, magic) == (5, pg.PG_F32, 4, 0x31424750)
    assert rs == sum(-(-w // 64) * -(-h // 4) for w, h, _ in sizes)

    def tiles(w, h, spp):  # the requested 32x8 fits every spp in the batched frame's two-pass tile
        tw, th = 32, 8
        return -(-w // tw) * -(-h // th)
    assert em == sum(tiles(*v) for v in sizes)
    assert pg.batch_table_bytes(0) == 0
    assert pg.batch_table_bytes(2) - pg.batch_table_bytes(1) == pg.batch_table_bytes(3) - pg.batch_table_bytes(2)


def test_batch_pack_rejects_bad_batches():
    ok = [_bview(base=0), _bview(base=1 << 16)]
    assert _pack(ok)[0] == pg.PG_OK
    bad_dtype = [_bview(base=0), _bview(base=1 << 16, dtype=pg.PG_F16)]
    shared_out = [_bview(base=0), _bview(base=0)]
    alias = [_bview()]
    alias[0].gamma_in = alias[0].gamma_out
    params_differ = [_bview(base=0), _bview(base=1 << 16, pi_hi=0.9)]
    spp9 = [_bview(spp=9)]
    no_albedo = [_bview()]
    no_albedo[0].cur = _view(albedo=False)
    prev_size = [_bview()]
    prev_size[0].prev = _view(w=9)
    cases = [
        (bad_dtype, pg.PG_ERR_ARG, "view 1"),
        (shared_out, pg.PG_ERR_ARG, "view 1"),
        (alias, pg.PG_ERR_ARG, "view 0"),
        (params_differ, pg.PG_ERR_ARG, "view 1"),
        (spp9, pg.PG_ERR_ARG, "view 0"),
        (no_albedo, pg.PG_ERR_ARG, "view 0"),
        (prev_size, pg.PG_ERR_UNSUPPORTED, "view 0"),
        ([_bview(flags=pg.PG_EM_BATCH)], pg.PG_ERR_UNSUPPORTED, "view 0"),
        # a tile shape that is not built
        ([_bview(tile_w=24, tile_h=24)], pg.PG_ERR_UNSUPPORTED, "not built"),
    ]
    for views, want, where in cases:
        st, msg, _ = _pack(views)
        assert st == want and where in msg, (st, msg)
    # frame 0 needs no history
    first = [_bview(frame=0)]
    first[0].gamma_in = pg.PgGamma(pg.PG_F32, None)
    first[0].prev = pg.PgView()
    assert _pack(first)[0] == pg.PG_OK
    # too small a table, and no views
    assert _pack(ok, nbytes=pg.batch_table_bytes(2) - 1)[0] == pg.PG_ERR_ARG
    assert _pack([])[0] == pg.PG_ERR_ARG


@no_device
def test_low_precision_state_limits_the_epoch():
    """k is stored in the state's type: BF16 holds every integer up to 256 and
    FP16 up to 2048, so larger k_max values are rejected by every call that
    takes such a state (pg_batch_pack included); FP32 accepts them."""
    L = pg.lib()
    v = _view()
    s = _samples()
    for dtype, limit in ((pg.PG_BF16, 256), (pg.PG_F16, 2048)):
        g = pg.PgGamma(dtype, FAKE)
        g2 = pg.PgGamma(dtype, FAKE + 4096)
        for k_max, ok in ((limit, True), (limit + 1, False)):
            P = pg.params(1, frame=1, k_max=k_max)
            calls = [
                (L.pg_reproject, (C.byref(P), C.byref(v), C.byref(v), g, g2, None, None)),
                (L.pg_sample_mis, (C.byref(P), C.byref(v), g, C.byref(s), None)),
                (L.pg_reproject_sample, (C.byref(P), C.byref(v), C.byref(v), g, g2, C.byref(s), None)),
                (L.pg_pdf, (C.byref(P), C.byref(v), g, 1, None, None, None, None, None)),
                (L.pg_em_update, (C.byref(P), C.byref(_view(albedo=True)), C.byref(s), g, 0, None)),
            ]
            for fn, args in calls:
                st, msg = _status(fn, *args)
                if ok:
                    # the epoch check passes; a later check (NULL dir, zero
                    # iterations) is what fails here
                    assert "k_max" not in msg, (fn.__name__, msg)
                else:
                    assert st == pg.PG_ERR_ARG and f"k_max {k_max}" in msg, (fn.__name__, st, msg)
        st, msg, _ = _pack([_bview(dtype=dtype, k_max=limit + 1)])
        assert st == pg.PG_ERR_ARG and "k_max" in msg, msg
        assert _pack([_bview(dtype=dtype, k_max=limit)])[0] == pg.PG_OK
    P = pg.params(1, frame=1, k_max=100000)
    st, msg = _status(L.pg_em_update, C.byref(P), C.byref(v), C.byref(s), pg.PgGamma(pg.PG_F32, FAKE), 0, None)
    assert "k_max" not in msg


def test_batch_pack_tile_per_spp_group():
    """Each spp group is trained with the tile its views request; views of
    one spp that request different tiles are rejected."""
    views = [_bview(w=70, h=37, spp=1, base=0, tile_w=16, tile_h=16),
             _bview(w=70, h=37, spp=2, base=1 << 16, tile_w=64, tile_h=4),
             _bview(w=70, h=37, spp=1, base=2 << 16, tile_w=16, tile_h=16)]
    st, msg, table = _pack(views)
    assert st == pg.PG_OK, msg
    hdr = table[:32].view(torch.int32).tolist()
    assert hdr[4] == 2  # two groups
    # BatchClass entries follow the header and ParamsK: find them by their spp
    ints = table.view(torch.int32).tolist()
    groups = [ints[i:i + 3] for i in range(8, 200) if ints[i] in (1, 2) and ints[i + 1] in (16, 64)
              and ints[i + 2] in (16, 4)]
    assert [1, 16, 16] in groups and [2, 64, 4] in groups, groups
    bad = [_bview(spp=1, base=0, tile_w=16, tile_h=16), _bview(spp=1, base=1 << 16, tile_w=32, tile_h=8)]
    st, msg, _ = _pack(bad)
    assert st == pg.PG_ERR_ARG and "different training tiles" in msg and "view 1" in msg, msg
