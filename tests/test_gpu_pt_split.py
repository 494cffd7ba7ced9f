"""Path tracer with its tiles split into several work items (chunk_spp): the
image, the AOV and the counters are bit-identical to those of the launch with
one work item per tile (per pixel the work items add integer fixed-point
sums, so the order in which they finish cannot change the total), on VDB and
dense volumes, with Russian roulette and an image-based light, on a
workspace holding stale bytes, and within relMSE 1e-4 of the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2504_04564_amd import _build, vdbc
from synth import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib():
    _build.ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return vdbc.load()


def relmse(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean((x - y) ** 2 / (y * y + 0.01)))


def _scene(n, w, h, spp, bounces=8, seed=0x5EED):
    cam = scenes.orbit_camera((n, n, n), w, h)
    med = scenes.pt_medium(64.0)
    prm = dict(spp=spp, max_bounces=bounces, seed=seed, macrocell=8)
    return cam, med, prm


def _bits(t):
    return t.view(torch.int32).cpu().numpy()


def _launch(field, cam, med, prm, stale=False, background=None):
    r = vdbc.Renderer(field, cam, med, prm, vdbc.MODE_PT, aov=True, background=background)
    if stale:
        r.ws.fill_(0xA5)   # whatever the caller's workspace held before
    r.launch()
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("tw", [8, 64])
def test_split_tiles_bit_identical_to_one_item_per_tile(tw):
    # 70 x 33 pixels: ragged tiles at both tile widths; 13 spp: chunks that do
    # not divide the sample count, a chunk of one sample, chunks >= spp
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.25)
    g = vdbc.Grid(buf)
    cam, med, prm = _scene(64, 70, 33, 13)
    prm.update(tile_w=tw, flags=vdbc.RENDER_COUNT)
    r0 = _launch(g, cam, med, dict(prm, chunk_spp=0))
    img0, aov0 = _bits(r0.image), _bits(r0.aov)
    n0, s0 = r0.sample_count(), r0.segment_count()
    assert n0 > 0 and np.count_nonzero(r0.image[..., 3].cpu().numpy()) > 0
    for chunk in (1, 2, 3, 4, 6, 12, 13, 14):
        r = _launch(g, cam, med, dict(prm, chunk_spp=chunk), stale=True)
        assert np.array_equal(_bits(r.image), img0), chunk
        assert np.array_equal(_bits(r.aov), aov0), chunk
        assert (r.sample_count(), r.segment_count()) == (n0, s0), chunk
        # the same workspace again: the call clears its own sums
        r.launch()
        torch.cuda.synchronize()
        assert np.array_equal(_bits(r.image), img0), chunk


def test_split_tiles_roulette_and_image_based_light_bit_identical():
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.10)
    g = vdbc.Grid(buf)
    cam, med, prm = _scene(64, 48, 40, 8, bounces=16)
    rng = np.random.default_rng(8)
    env = torch.from_numpy((0.2 + rng.random((16, 32, 3))).astype(np.float32)).cuda()
    med = dict(med, albedo=0.9, env=env)
    prm["flags"] = vdbc.RENDER_RR
    r0 = _launch(g, cam, med, dict(prm, chunk_spp=0))
    r1 = _launch(g, cam, med, dict(prm, chunk_spp=3), stale=True)
    assert np.array_equal(_bits(r1.image), _bits(r0.image))
    assert np.array_equal(_bits(r1.aov), _bits(r0.aov))


def test_split_tiles_vs_oracle_vdb_and_dense():
    v = synth.mid_volume(n=96)
    buf, _ = vdbc.encode(v, 0.10)
    cam, med, prm = _scene(96, 52, 44, 4)
    prm["chunk_spp"] = 1
    want, want_aov = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, aov=True)
    r = _launch(vdbc.Grid(buf), cam, med, prm, stale=True)
    assert relmse(r.image.cpu().numpy().reshape(-1, 4), want) <= 1e-4
    assert relmse(r.aov.cpu().numpy().reshape(-1, 2), want_aov) <= 1e-4
    d = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    want_d = oracle.render_pt(oracle.DenseField(v, 0.0), cam, med, prm)
    rd = _launch(d, cam, med, prm, stale=True, background=0.0)
    assert relmse(rd.image.cpu().numpy().reshape(-1, 4), want_d) <= 1e-4
    rd0 = _launch(d, cam, med, dict(prm, chunk_spp=0), background=0.0)
    assert np.array_equal(_bits(rd.image), _bits(rd0.image))


def test_split_paper_launch_sampled_pixels():
    # the paper-scale launch (1920x1080, 64 spp, <= 16 bounces, 1:10, macrocell
    # 64, 64-wide wave rows) split into work items of 8 samples, on the billowed
    # recipe at 1/8 of the edge lengths: bit-identical to the unsplit launch,
    # and a sample of the pixels against the oracle
    P = scenes.PAPER
    dims = tuple(d // 8 for d in P["dims"])
    v = synth.paper_volume(dims=dims)
    buf, _ = vdbc.encode(v, 0.10)
    g = vdbc.Grid(buf)
    cam = scenes.orbit_camera(dims, P["width"], P["height"])
    med = scenes.pt_medium(64.0)
    prm = dict(spp=P["spp"], max_bounces=P["max_bounces"], seed=P["seed"], macrocell=64, tile_w=64)
    a = vdbc.render(g, cam, med, dict(prm, chunk_spp=8), vdbc.MODE_PT).clone()
    b = vdbc.render(g, cam, med, prm, vdbc.MODE_PT)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    img = a.cpu().numpy().reshape(-1, 4)
    rng = np.random.default_rng(54)
    pix = np.sort(rng.choice(P["width"] * P["height"], 512, replace=False)).astype(np.uint32)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, pixels=pix)
    assert relmse(img[pix], want) <= 1e-4
    assert np.count_nonzero(want[:, 3] > 0) >= 16


@pytest.mark.parametrize("tw,chunk", [(8, 0), (8, 3), (64, 4)])
def test_cost_order_bit_identical(tw, chunk):
    # tiles handed out in decreasing estimated cost instead of raster order:
    # the same image, AOV and counts, on VDB and dense volumes
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.10)
    cam, med, prm = _scene(64, 70, 33, 12)
    prm.update(tile_w=tw, chunk_spp=chunk)
    d = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    for field, bg in ((vdbc.Grid(buf), None), (d, 0.0)):
        r0 = _launch(field, cam, med, dict(prm, flags=vdbc.RENDER_COUNT), background=bg)
        r1 = _launch(field, cam, med, dict(prm, flags=vdbc.RENDER_COUNT | vdbc.RENDER_COST_ORDER),
                     stale=True, background=bg)
        assert np.array_equal(_bits(r1.image), _bits(r0.image))
        assert np.array_equal(_bits(r1.aov), _bits(r0.aov))
        assert (r1.sample_count(), r1.segment_count()) == (r0.sample_count(), r0.segment_count())


def test_noalloc_split_and_cost_order_equal_the_workspace_render():
    # the allocation-free entry point keeps the pixel sums and the cost order
    # in its fixed scratch: same bits as the render with a workspace, on two
    # calls in a row (the second smaller), image and AOV
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.10)
    g = vdbc.Grid(buf)
    for w, h, spp, chunk in ((96, 80, 12, 5), (40, 24, 6, 1)):
        cam, med, prm = _scene(64, w, h, spp)
        prm.update(tile_w=16, chunk_spp=chunk, flags=vdbc.RENDER_COST_ORDER)
        ref = _launch(g, cam, med, prm)
        aov = torch.empty((h, w, 2), dtype=torch.float32, device="cuda")
        img = vdbc.render_noalloc(g, cam, med, prm, vdbc.MODE_PT, aov=aov)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(img), _bits(ref.image)), (w, h)
        assert np.array_equal(_bits(aov), _bits(ref.aov)), (w, h)
