"""pg_frame_batched_noalloc, the entry point for callers that cannot
allocate: the device copy of the packed table lives in the library's own
fixed array.  Through the C ABI it must give pg_frame_batched's results bit
for bit, on consecutive calls whose second batch is smaller than the first
(the array keeps the last call's table), eagerly and from a captured graph."""
import sys

import pytest
import torch

import paper_2112_09728_amd as pg
from paper_2112_09728_amd import workload as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

BIG = [(70, 37, 1), (129, 64, 3), (33, 95, 8), (200, 17, 2)]
SMALL = [(40, 30, 2), (17, 9, 1)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _specs(sizes, seed0):
    specs, seqs = [], []
    for i, (w, h, spp) in enumerate(sizes):
        seed = seed0 + 31 * i
        seq = wl.Sequence(w, h, seed)
        fr0 = seq.frame(0)
        specs.append(dict(width=w, height=h, spp=spp, seed=seed, lights=fr0["lights"],
                          ambient=float(fr0["ambient"]), view=i))
        seqs.append((seq, fr0))
    return specs, seqs


def _frames(seqs, t, prev):
    out = []
    for i, (seq, fr0) in enumerate(seqs):
        cur = pg.DeviceFrame(fr0 if t == 0 else seq.frame(t))
        out.append((cur, prev[i][0] if prev else None))
    return out


def _same(a, b):
    return torch.equal(a.view(torch.int16) if a.dtype != torch.float32 else a.view(torch.int32),
                       b.view(torch.int16) if b.dtype != torch.float32 else b.view(torch.int32))


@pytest.mark.parametrize("graph", [False, True])
def test_noalloc_frame_matches_frame_batched(graph):
    for name, sizes, seed0, dtype in (("big", BIG, wl.SEED_BASE + 90, torch.float16),
                                      ("small", SMALL, wl.SEED_BASE + 95, torch.float32)):
        say(f"case: no-alloc batched frame, {name} batch of {len(sizes)} views, graph={graph}")
        specs, seqs = _specs(sizes, seed0)
        ref = pg.BatchedGuide(specs, gamma_dtype=dtype)
        mine = pg.BatchedGuide(specs, gamma_dtype=dtype, noalloc=True)
        assert mine.dev_table is None
        prev = None
        for t in range(2):
            frames = _frames(seqs, t, prev)
            ref.step(frames, t)
            mine.step(frames, t, graph=graph)
            torch.cuda.synchronize()
            for i in range(len(sizes)):
                assert _same(mine.state(i), ref.state(i)), f"{name}: Gamma of view {i} differs at frame {t}"
                for f in ("dir", "pdf_mix", "pdf_brdf", "radiance"):
                    assert torch.equal(getattr(mine.samples[i], f).view(torch.int32),
                                       getattr(ref.samples[i], f).view(torch.int32)), (name, f, i, t)
                assert torch.equal(mine.samples[i].strategy, ref.samples[i].strategy), (name, i, t)
            prev = frames
        say(f"  {name}: 2 frames bit-identical to pg_frame_batched")


def test_noalloc_rejects_tables_beyond_its_array():
    n = 1
    while pg.batch_table_bytes(n) <= pg.NOALLOC_TABLE_BYTES:
        n += 1
    table = torch.zeros(pg.batch_table_bytes(n), dtype=torch.uint8).pin_memory()
    # a header that claims n views (the size check comes before any work)
    hdr = table[:24].view(torch.int32)
    hdr[0] = n
    hdr[4] = 1
    hdr[5] = 0x31424750
    with pytest.raises(RuntimeError, match="status 2"):
        pg.frame_batched_noalloc(table)
