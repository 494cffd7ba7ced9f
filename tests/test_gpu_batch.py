"""Batched multi-volume rendering: the persistent launch, the per-volume
launches and the replays of the captured graph all give images bit-identical
to one vdbc_render call per volume (same random keys)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2504_04564_amd import _build, autotune, vdbc
from synth import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib():
    _build.ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return vdbc.load()


def _items(count=10, seed=3):
    specs = synth.batch_sizes(count, seed=seed, lo=24, hi=96)
    grids, items = [], []
    for i, (side, q, spp) in enumerate(specs):
        v = synth.cloud_volume((side, side + 3 * (i % 3), side), seed=100 + i)
        buf, _ = vdbc.encode(v, q)
        g = vdbc.Grid(buf)
        grids.append(g)
        w, h = 40 + 8 * (i % 4), 36 + 5 * (i % 3)
        items.append(dict(grid=g, camera=scenes.orbit_camera(g.dims, w, h, azimuth_deg=20 * i),
                          medium=scenes.pt_medium(48.0), spp=min(spp, 4), max_bounces=6,
                          seed=0x1234 + i, frame=i, host=buf))
    return items


def _coloured_tf(i):
    # the five-point transfer function with its colour channels rotated by i
    # and its alpha scaled: every volume of the batch has its own colours
    sc = 1.0 - 0.1 * (i % 4)
    return [(c[i % 3], c[(i + 1) % 3], c[(i + 2) % 3], a * sc) for *c, a in scenes.TF5]


def _single(it, macrocell, tile_w=8):
    prm = dict(spp=it["spp"], max_bounces=it["max_bounces"], seed=it["seed"], frame=it["frame"],
               macrocell=macrocell, tile_w=tile_w)
    return vdbc.render(it["grid"], it["camera"], it["medium"], prm, vdbc.MODE_PT).clone()


def _same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


# chunk_spp splits the tiles of every volume with more samples than that into
# work items (the items' spp are 1..4: chunk 3 leaves a ragged last item and
# some volumes whole, so one batch mixes split and whole volumes)
@pytest.mark.parametrize("tuning", [dict(macrocell=16, tile_w=8, blocks_per_cu=4, persistent=1),
                                    dict(macrocell=8, tile_w=16, blocks_per_cu=2, persistent=1),
                                    dict(macrocell=16, tile_w=32, blocks_per_cu=1, persistent=0),
                                    dict(macrocell=16, tile_w=8, blocks_per_cu=4, persistent=1, chunk_spp=1),
                                    dict(macrocell=8, tile_w=16, blocks_per_cu=2, persistent=1, chunk_spp=3),
                                    dict(macrocell=16, tile_w=32, blocks_per_cu=1, persistent=0, chunk_spp=2)])
def test_batch_equals_single_launches(tuning):
    items = _items()
    ref = [_single(it, tuning["macrocell"]) for it in items]
    b = vdbc.Batch(items, tuning)
    b.launch()
    torch.cuda.synchronize()
    for img, r in zip(b.images, ref):
        assert _same(img, r)
    b.close()


def test_batch_images_match_oracle_with_coloured_tfs():
    # the persistent batched launch against the oracle, volume by volume:
    # uneven sizes, rates, images and spp, a different coloured transfer
    # function, extinction and frame per volume
    items = _items(6, seed=13)
    for i, it in enumerate(items):
        it["medium"] = dict(scenes.pt_medium_tf5(32.0 + 8.0 * i), tf=_coloured_tf(i))
    C = 16
    b = vdbc.Batch(items, dict(macrocell=C, tile_w=8, blocks_per_cu=4, persistent=1))
    b.launch()
    torch.cuda.synchronize()
    lit = 0
    for i, (it, img) in enumerate(zip(items, b.images)):
        prm = dict(spp=it["spp"], max_bounces=it["max_bounces"], seed=it["seed"], frame=it["frame"],
                   macrocell=C)
        want = oracle.render_pt(oracle.VdbField(it["host"]), it["camera"], it["medium"], prm)
        got = img.cpu().numpy().reshape(-1, 4).astype(np.float64)
        rel = float(np.mean((got - want) ** 2 / (want * want + 0.01)))
        assert rel <= 1e-4, (i, rel)
        lit += np.count_nonzero(want[:, 3] > 0) >= 16
    # a small volume at 1:20 may keep no brick at all (K = round(q N) = 0) and
    # render as empty space; most volumes of the batch must show the medium
    assert lit >= 4, lit
    b.close()


@pytest.mark.parametrize("chunk_spp", [0, 2])
def test_graph_replays_match_eager(chunk_spp):
    # with chunk_spp 2 every replay also clears and resolves the pixel sums
    items = _items(8, seed=5)
    ref = [_single(it, 16) for it in items]
    b = vdbc.Batch(items, dict(macrocell=16, chunk_spp=chunk_spp))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    b.capture(s)
    for rep in range(3):
        for img in b.images:
            img.zero_()
        # eager work in between replays
        _ = _single(items[rep], 16)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.replay()
        s.synchronize()
        for img, r in zip(b.images, ref):
            assert _same(img, r), rep
    b.close()


def test_autotuner_picks_a_measured_candidate(tmp_path):
    items = _items(4, seed=9)
    best, allr = autotune.tune_batch(items, dict(macrocell=(16,), tile_w=(8, 16),
                                                 blocks_per_cu=(2, 4), persistent=(0, 1)), reps=2)
    assert best in allr and len(allr) == 8
    assert best["ms"] == min(r["ms"] for r in allr)
    # the item sizes are a second stage at the fastest whole-tile candidate
    best2, allr2 = autotune.tune_batch(items, dict(macrocell=(16,), tile_w=(8,), blocks_per_cu=(4,),
                                                   persistent=(1,), chunk_spp=(0, 1, 2)), reps=2)
    assert [r["chunk_spp"] for r in allr2] == [0, 1, 2]
    assert best2["ms"] == min(r["ms"] for r in allr2)
    it = items[0]
    prm = dict(spp=it["spp"], max_bounces=it["max_bounces"], seed=it["seed"])
    path = str(tmp_path / "tune.json")
    key = autotune.workload_key("vdb", it["grid"].dims, 0.1, it["spp"])
    choice = autotune.cached_render_tuning(
        path, key, lambda: autotune.tune_render(it["grid"], it["camera"], it["medium"], prm,
                                                space=dict(macrocell=(8, 16), tile_w=(8, 32)),
                                                reps=2))
    assert autotune.load(path)[key] == choice


def test_cache_policies_give_identical_images():
    # the accessor's cache policy changes the work of a lookup, never its value
    items = _items(1, seed=21)
    it = items[0]
    base = dict(spp=3, max_bounces=6, seed=it["seed"], macrocell=8)
    imgs = []
    for flag in (0, vdbc.RENDER_CACHE_LEAF, vdbc.RENDER_CACHE_NONE):
        img = vdbc.render(it["grid"], it["camera"], it["medium"], dict(base, flags=flag),
                          vdbc.MODE_PT).clone()
        imgs.append(img)
    assert _same(imgs[0], imgs[1]) and _same(imgs[0], imgs[2])
    with pytest.raises(vdbc.VdbcError):
        vdbc.render(it["grid"], it["camera"], it["medium"],
                    dict(base, flags=vdbc.RENDER_CACHE_LEAF | vdbc.RENDER_CACHE_NONE), vdbc.MODE_PT)
