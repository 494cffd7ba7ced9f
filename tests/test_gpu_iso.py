"""GPU parity of the iso-surface marcher (Section 5.4's interval-based
implicit iso-surface ray marcher, reading R22) against the oracle.  Where
float rounding decides which lattice interval crosses the iso value, both
sides can be right; pixels whose lattice samples all stay 1e-4 away from the
iso value must agree on hit or miss, and on hits the hit parameter agrees to
step / 2^refine + 1e-3 and the normal colour to 2e-3 where the bisection
midpoints also keep 1e-5 away.  The VDB at 1:1 equals the dense array
bitwise, and empty-node skipping leaves the image bitwise unchanged."""
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


def _gpu(field, cam, prm, background=None):
    r = vdbc.Renderer(field, cam, None, prm, vdbc.MODE_ISO, background=background, aov=True)
    r.launch()
    return r.image.cpu().numpy().astype(np.float64), r.aov.cpu().numpy().astype(np.float64)


def _check(img, aov, want, aux, step, refine):
    robust = aux[..., 1] >= 1e-4
    assert robust.mean() > 0.9
    hit_g = img[..., 3] == 1.0
    hit_o = want[..., 3] == 1.0
    assert np.array_equal(hit_g[robust], hit_o[robust])
    both = robust & hit_o
    assert both.sum() > 50
    assert np.max(np.abs(aov[..., 0][both] - aux[..., 0][both])) <= step / 2 ** refine + 1e-3
    fine = both & (aux[..., 2] >= 1e-5)
    assert np.max(np.abs(img[fine][:, :3] - want[fine][:, :3])) <= 2e-3
    assert np.all(img[~hit_g] == 0.0) and np.all(aov[..., 0][~hit_g] == -1.0)


@pytest.mark.parametrize("shape,q,iso", [((48, 40, 56), 0.25, 0.5), ((33, 47, 29), 0.5, 0.3),
                                         ((64, 64, 64), 1.0, 0.5)])
def test_iso_vdb_vs_oracle(shape, q, iso):
    v = synth.cloud_volume(shape, seed=7 + shape[0])
    buf, _ = vdbc.encode(v, q)
    nz, ny, nx = shape
    cam = scenes.orbit_camera((nx, ny, nz), 96, 80)
    step, refine = 0.5, 12
    prm = dict(step=step, iso=iso, refine=refine)
    img, aov = _gpu(vdbc.Grid(buf), cam, prm)
    want, aux = oracle.render_iso(oracle.VdbField(buf), cam, iso, step, refine, aux=True)
    _check(img, aov, want, aux, step, refine)


def test_iso_dense_vs_oracle_and_lossless_vdb_bitwise():
    v = synth.cloud_volume((40, 44, 52), seed=3)
    nz, ny, nx = v.shape
    cam = scenes.orbit_camera((nx, ny, nz), 72, 64, azimuth_deg=-50)
    prm = dict(step=0.4, iso=0.5, refine=10)
    img_d, aov_d = _gpu(torch.from_numpy(v).cuda(), cam, prm, background=0.0)
    want, aux = oracle.render_iso(oracle.DenseField(v, 0.0), cam, 0.5, 0.4, 10, aux=True)
    _check(img_d, aov_d, want, aux, 0.4, 10)
    img_v, aov_v = _gpu(vdbc.Grid(vdbc.encode(v, 1.0)[0]), cam, prm)
    assert np.array_equal(img_v.view(np.uint64), img_d.view(np.uint64))
    assert np.array_equal(aov_v.view(np.uint64), aov_d.view(np.uint64))


def test_iso_empty_node_skipping_is_bitwise_neutral_and_counts_fewer_samples():
    v = synth.cloud_volume((96, 80, 112), seed=11)
    buf, _ = vdbc.encode(v, 0.10)
    g = vdbc.Grid(buf)
    cam = scenes.orbit_camera((112, 80, 96), 128, 96)
    base = dict(step=0.5, iso=0.5, refine=12)
    a = vdbc.Renderer(g, cam, None, dict(base, flags=vdbc.RENDER_COUNT), vdbc.MODE_ISO, aov=True)
    b = vdbc.Renderer(g, cam, None, dict(base, flags=vdbc.RENDER_COUNT | vdbc.RENDER_HDDA),
                      vdbc.MODE_ISO, aov=True)
    a.launch()
    b.launch()
    assert torch.equal(a.image.view(torch.int32), b.image.view(torch.int32))
    assert torch.equal(a.aov.view(torch.int32), b.aov.view(torch.int32))
    assert b.sample_count() < a.sample_count()


def test_iso_ramp_plane_closed_form():
    # linear field: trilinear is exact, the plane z = (nz-1)/2 is hit at
    # t = nz/2 with normal -z, colour (0.5, 0.5, 0)
    nx, ny, nz = 24, 20, 40
    v = np.broadcast_to((np.arange(nz, dtype=np.float32) / (nz - 1))[:, None, None],
                        (nz, ny, nx)).copy()
    cam = scenes.ortho_z_camera(nx, ny, nx, ny)
    img, aov = _gpu(vdbc.Grid(vdbc.encode(v, 1.0)[0]), cam, dict(step=0.37, iso=0.5, refine=16))
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    assert np.all(img[inner][..., 3] == 1.0)
    assert np.max(np.abs(aov[inner][..., 0] - nz / 2.0)) <= 2e-5
    assert np.max(np.abs(img[inner][..., :3] - [0.5, 0.5, 0.0])) <= 1e-5
