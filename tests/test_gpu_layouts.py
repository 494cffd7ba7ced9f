"""Node layouts on the GPU (Morton child-slot order, SoA node words, both):
lookups of every voxel equal the oracle's reconstruction bit for bit, and
samples, majorants, error statistics, EA / ISO / PT images and batched images
are bit-identical to those of the layout-0 buffer (the accessor returns the
same values, so every later step is the same arithmetic)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2504_04564_amd import _build, vdbc
from synth import scenes

# Device support for node layouts 1..3 is switched off (vdbc_grid_init
# rejects them): the first GPU run that rendered them ended in a memory fault
# whose cause has not been shown, so these tests stay skipped until it is.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="device kernels for node layouts 1..3 are switched off after an "
                                      "unexplained GPU memory fault; the host converter is tested on the CPU")]

LAYOUTS = [1, 2, 3]


@pytest.fixture(scope="module", autouse=True)
def lib():
    _build.ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return vdbc.load()


def _rand(shape, seed, zero=0.6):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < zero] = 0.0
    return v


def _same(a, b):
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def _grids(v, q, metric=2, flags=0):
    buf, st = vdbc.encode(v, q, metric, flags)
    return buf, {L: vdbc.Grid(vdbc.relayout(buf, L)) for L in (0, 1, 2, 3)}


def _all_ijk(shape, pad=2):
    nz, ny, nx = shape
    g = np.stack(np.meshgrid(np.arange(-pad, nx + pad), np.arange(-pad, ny + pad),
                             np.arange(-pad, nz + pad), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(np.int32)


def _upper_tile_volume():
    v = _rand((130, 131, 133), 7, zero=0.9)
    v[:128, :128, :128] = np.float32(0.25)
    return v


@pytest.mark.parametrize("case", ["tiles", "upper_tile", "ragged"])
def test_lookup_every_voxel_every_layout(case):
    if case == "tiles":
        v, q = _rand((64, 72, 80), 6), 0.6
        v[:40, :48, :56] = np.float32(0.75)
    elif case == "upper_tile":
        v, q = _upper_tile_volume(), 1.0
    else:
        v, q = _rand((129, 33, 257), 8), 0.07
    buf, grids = _grids(v, q)
    ijk = _all_ijk(v.shape)
    R = oracle.reconstruct(v, q)
    inside = np.all((ijk >= 0) & (ijk < [v.shape[2], v.shape[1], v.shape[0]]), axis=1)
    want = np.full(len(ijk), np.float32(vdbc.validate(buf)["background"]), np.float32)
    want[inside] = R[ijk[inside, 2], ijk[inside, 1], ijk[inside, 0]]
    q_t = torch.from_numpy(ijk).cuda()
    for L in LAYOUTS:
        got = vdbc.lookup(grids[L], q_t).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), L


def test_samples_majorant_and_statistics_every_layout():
    v = synth.mid_volume(n=160)
    buf, grids = _grids(v, 0.1)
    rng = np.random.default_rng(3)
    pos = torch.from_numpy((rng.random((1 << 18, 3)) * 164 - 2).astype(np.float32)).cuda()
    med = scenes.pt_medium(64.0)
    dense = torch.from_numpy(v).cuda()
    ref_tri = vdbc.sample(grids[0], pos, 1).clone()
    ref_nn = vdbc.sample(grids[0], pos, 0).clone()
    ref_maj = {C: vdbc.majorant(grids[0], med, C).clone() for C in (8, 16)}
    ref_cmp = vdbc.compare_dense(grids[0], dense)
    for L in LAYOUTS:
        assert _same(vdbc.sample(grids[L], pos, 1), ref_tri), L
        assert _same(vdbc.sample(grids[L], pos, 0), ref_nn), L
        for C in (8, 16):
            assert _same(vdbc.majorant(grids[L], med, C), ref_maj[C]), (L, C)
        assert vdbc.compare_dense(grids[L], dense) == ref_cmp, L


def test_ea_and_iso_every_layout():
    v = synth.mid_volume(n=128)
    buf, grids = _grids(v, 0.05)
    cam = scenes.orbit_camera((128, 128, 128), 96, 72)
    med = scenes.ea_medium(8.0)
    for flags in (0, vdbc.RENDER_HDDA):
        ea = vdbc.render(grids[0], cam, med, dict(step=0.5, flags=flags), vdbc.MODE_EA).clone()
        iso = vdbc.render(grids[0], cam, None, dict(step=0.5, iso=0.3, refine=8, flags=flags),
                          vdbc.MODE_ISO).clone()
        for L in LAYOUTS:
            assert _same(vdbc.render(grids[L], cam, med, dict(step=0.5, flags=flags), vdbc.MODE_EA), ea)
            assert _same(vdbc.render(grids[L], cam, None, dict(step=0.5, iso=0.3, refine=8, flags=flags),
                                     vdbc.MODE_ISO), iso)


@pytest.mark.parametrize("cache", [0, 1, 2])
def test_pt_every_layout_and_cache_policy(cache):
    v = synth.mid_volume(n=128)
    buf, grids = _grids(v, 0.1)
    cam = scenes.orbit_camera((128, 128, 128), 80, 64)
    med = scenes.pt_medium(64.0)
    prm = dict(spp=4, max_bounces=8, seed=0x77, macrocell=16, flags=vdbc.CACHE_FLAGS[cache])
    ref, ref_aov = vdbc.render(grids[0], cam, med, dict(prm, flags=0), vdbc.MODE_PT, aov=True)
    for L in LAYOUTS:
        img, aov = vdbc.render(grids[L], cam, med, prm, vdbc.MODE_PT, aov=True)
        assert _same(img, ref) and _same(aov, ref_aov), (L, cache)
    if cache == 2:
        # roulette and the sample counters through a non-default layout
        rr = dict(prm, flags=vdbc.RENDER_RR | vdbc.RENDER_COUNT)
        r0 = vdbc.Renderer(grids[0], cam, med, rr, vdbc.MODE_PT)
        r3 = vdbc.Renderer(grids[3], cam, med, rr, vdbc.MODE_PT)
        a, b = r0.launch().clone(), r3.launch()
        torch.cuda.synchronize()
        assert _same(a, b) and r0.sample_count() == r3.sample_count() > 0


def test_batch_every_layout_and_mixed_layouts_rejected():
    items = []
    for i, side in enumerate((40, 56, 72)):
        vol = synth.cloud_volume((side, side + 4, side), seed=200 + i)
        buf, _ = vdbc.encode(vol, 0.15)
        items.append((buf, dict(camera=scenes.orbit_camera((side, side + 4, side), 48, 40, azimuth_deg=30 * i),
                                medium=scenes.pt_medium(48.0), spp=2, max_bounces=6, seed=0x99 + i, frame=i)))
    outs = {}
    for L in (0, 1, 2, 3):
        its = [dict(it, grid=vdbc.Grid(vdbc.relayout(buf, L))) for buf, it in items]
        b = vdbc.Batch(its, dict(macrocell=16))
        b.launch()
        torch.cuda.synchronize()
        outs[L] = [img.clone() for img in b.images]
        b.close()
    for L in LAYOUTS:
        for a, r in zip(outs[L], outs[0]):
            assert _same(a, r), L
    mixed = [dict(it, grid=vdbc.Grid(vdbc.relayout(buf, k % 2))) for k, (buf, it) in enumerate(items)]
    with pytest.raises(vdbc.VdbcError) as e:
        vdbc.Batch(mixed, dict(macrocell=16))
    assert e.value.status == vdbc.E_UNSUPPORTED
