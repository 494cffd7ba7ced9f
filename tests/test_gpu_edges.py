"""Degenerate inputs of the renderers against the oracle: one-voxel and
one-voxel-thick volumes, ragged edge bricks, a 1x1 image, the largest
macrocell over a volume smaller than one cell, and the same volumes as
dense arrays (with the encoder's background outside the volume: with two
distinct values it is the smaller one).  Bars as in the parity tests: EA
within 1e-5, PT relMSE 1e-4 at matched seeds, lossless VDB == dense
bitwise."""
import numpy as np
import pytest
import torch

import oracle
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


def _vol(shape, seed):
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.2, 1.0, size=shape).astype(np.float32)
    v[rng.random(shape) < 0.3] = 0.0
    return v


SHAPES = [(1, 1, 1), (1, 1, 2), (3, 40, 1), (1, 33, 70), (9, 2, 37)]


@pytest.mark.parametrize("shape", SHAPES)
def test_ea_degenerate_volumes(shape):
    v = _vol(shape, 3)
    nz, ny, nx = shape
    buf, st = vdbc.encode(v, 1.0)
    med = scenes.ea_medium(8.0)
    for w, h in ((1, 1), (9, 7)):
        cam = scenes.orbit_camera((nx, ny, nz), w, h)
        for flags in (0, vdbc.RENDER_HDDA):
            prm = dict(step=0.25, flags=flags)
            want = oracle.render_ea(oracle.VdbField(buf), cam, med, prm).reshape(-1, 4)
            got = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_EA).cpu().numpy().reshape(-1, 4)
            assert np.max(np.abs(got - want)) <= 1e-5, (shape, w, flags)
            dense = vdbc.render(torch.from_numpy(v).cuda(), cam, med, prm, vdbc.MODE_EA,
                                background=st["background"])
            assert np.array_equal(dense.cpu().numpy().reshape(-1, 4).view(np.uint32), got.view(np.uint32))


@pytest.mark.parametrize("shape", SHAPES)
def test_pt_degenerate_volumes(shape):
    v = _vol(shape, 5)
    nz, ny, nx = shape
    for q in (1.0, 0.5):
        buf, st = vdbc.encode(v, q)
        g = vdbc.Grid(buf)
        med = scenes.pt_medium(64.0)
        for (w, h), C in (((1, 1), 4), ((9, 7), 64)):
            cam = scenes.orbit_camera((nx, ny, nz), w, h)
            prm = dict(spp=16, max_bounces=8, seed=0x1D, macrocell=C)
            want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm)
            got = vdbc.render(g, cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
            assert relmse(got, want) <= 1e-4, (shape, q, w, C)
            if q == 1.0:
                dense = vdbc.render(torch.from_numpy(v).cuda(), cam, med, prm, vdbc.MODE_PT,
                                    background=st["background"])
                assert np.array_equal(dense.cpu().numpy().reshape(-1, 4).view(np.uint32), got.view(np.uint32))


def test_majorant_of_volume_smaller_than_one_cell():
    v = _vol((1, 33, 70), 9)
    buf, _ = vdbc.encode(v, 0.5)
    med = scenes.pt_medium(64.0)
    for C in (4, 64):
        got = vdbc.majorant(vdbc.Grid(buf), med, C).cpu().numpy()
        want = oracle.majorant(oracle.VdbField(buf), med, C)
        assert got.shape == want.shape
        np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-12)
