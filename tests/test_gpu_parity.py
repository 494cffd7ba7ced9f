"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Bars: bit-exact for lookups, nearest samples and Philox;
trilinear |d| <= 1e-6 * max|corner|; emission-absorption pixels within 1e-5;
path-traced images within relMSE 1e-4 at matched seeds."""
import math

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


def _rand(shape, seed, zero=0.6):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < zero] = 0.0
    return v


def _dense_t(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _cuda(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda() if dtype is None else t.to(dtype).cuda()


# ---------------------------------------------------------------- Philox

def test_philox_bit_exact():
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(65536 + 17, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(65536 + 17, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0], key[0] = 0, 0
    ctr[1], key[1] = 0xFFFFFFFF, 0xFFFFFFFF
    got = vdbc.philox(_cuda(ctr.view(np.int32)), _cuda(key.view(np.int32)))
    got = got.cpu().numpy().view(np.uint32).reshape(-1, 4)
    for i in range(len(ctr)):
        assert np.array_equal(got[i], oracle.philox(ctr[i], key[i])), i


def test_philox_bit_exact_1e8_counters():
    # 12 chunks of 2^23 seeded (counter, key) pairs: 100,663,296 counters
    n = 1 << 23
    for c in range(12):
        rng = np.random.default_rng([11, c])
        ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint32)
        key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint32)
        got = vdbc.philox(_cuda(ctr.view(np.int32)), _cuda(key.view(np.int32)))
        got = got.cpu().numpy().view(np.uint32).reshape(-1, 4)
        assert np.array_equal(got, oracle.philox_many(ctr, key)), c


# ---------------------------------------------------------------- lookups

LOOKUP_CASES = [((64, 64, 64), 0.25, 2, 0), ((37, 50, 70), 0.3, 1, 0),
                ((37, 50, 70), 0.3, 3, vdbc.NO_PRUNE), ((130, 20, 140), 0.5, 2, vdbc.NO_CORNERS),
                ((1, 1, 1), 1.0, 2, 0), ((200, 9, 3), 0.6, 2, 0), ((129, 257, 33), 0.07, 2, 0)]


def _all_ijk(shape, pad=2):
    nz, ny, nx = shape
    g = np.stack(np.meshgrid(np.arange(-pad, nx + pad), np.arange(-pad, ny + pad),
                             np.arange(-pad, nz + pad), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(np.int32)


@pytest.mark.parametrize("shape,q,metric,flags", LOOKUP_CASES)
def test_lookup_every_voxel_bit_exact(shape, q, metric, flags):
    v = _rand(shape, 41)
    v[: shape[0] // 2, : shape[1] // 2, : shape[2] // 2] = np.float32(0.75)
    buf, st = vdbc.encode(v, q, metric, flags)
    g = vdbc.Grid(buf)
    ijk = _all_ijk(shape)
    got = vdbc.lookup(g, _cuda(ijk)).cpu().numpy()
    want = oracle.lookup(oracle.VdbField(buf), ijk.astype(np.int64))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    R = oracle.reconstruct(v, q, metric, flags)
    inside = np.all((ijk >= 0) & (ijk < [shape[2], shape[1], shape[0]]), axis=1)
    assert np.array_equal(got[inside], R[ijk[inside, 2], ijk[inside, 1], ijk[inside, 0]])
    assert np.all(got[~inside] == np.float32(st["background"]))


PARTIAL_LOOKUP_CASES = [((64, 96, 128), 0.25, 0, (0.5, 1e30)), ((37, 50, 70), 0.3, 0, (0.3, 0.6)),
                        ((45, 70, 90), 0.4, vdbc.NO_PRUNE, (0.1, 1e30)),
                        ((129, 257, 33), 0.07, 0, (0.5, 0.99))]


@pytest.mark.parametrize("shape,q,flags,part", PARTIAL_LOOKUP_CASES)
def test_partial_bricks_lookup_every_voxel_bit_exact(shape, q, flags, part):
    # partial-brick activation: leaves with scattered active voxels, every
    # voxel (and two voxels of padding) against the oracle's reconstruction
    v = _rand(shape, 43)
    v[: shape[0] // 2, : shape[1] // 2, : shape[2] // 2] = np.float32(0.75)
    buf, st = vdbc.encode(v, q, 2, flags, partial=part)
    g = vdbc.Grid(buf)
    ijk = _all_ijk(shape)
    got = vdbc.lookup(g, _cuda(ijk)).cpu().numpy()
    R = oracle.reconstruct(v, q, 2, flags, partial=part)
    inside = np.all((ijk >= 0) & (ijk < [shape[2], shape[1], shape[0]]), axis=1)
    assert np.array_equal(got[inside].view(np.uint32),
                          R[ijk[inside, 2], ijk[inside, 1], ijk[inside, 0]].view(np.uint32))
    assert np.all(got[~inside] == np.float32(st["background"]))
    m = oracle.active_mask(v, q, 2, flags, partial=part)
    assert 0 < m.sum() < m.size


def test_partial_bricks_pt_vs_oracle():
    # the path tracer over a partially activated cloud (1:10, half the voxels
    # of twice the bricks) against the oracle at matched seeds
    v = synth.mid_volume(n=96)
    buf, _ = vdbc.encode(v, 0.10, partial=(0.5, 1e30))
    cam = scenes.orbit_camera((96, 96, 96), 48, 40)
    med = scenes.pt_medium_tf5(64.0)
    prm = dict(spp=4, max_bounces=8, seed=0x5EED, macrocell=8)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm)
    got = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
    assert relmse(got, want) <= 1e-4
    assert np.count_nonzero(want[:, 3] > 0) >= 64


# ---------------------------------------------------------------- sampling

def _positions(shape, n, seed, margin=2.0):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    p = rng.uniform([-margin] * 3, [nx + margin, ny + margin, nz + margin], size=(n, 3))
    p = p.astype(np.float32)
    # exact lattice points, half points, leaf and brick boundaries
    k = min(n // 4, 4096)
    p[:k] = np.floor(p[:k])
    p[k:2 * k] = np.floor(p[k:2 * k]) + 0.5
    p[2 * k:2 * k + 64, 0] = np.float32(7.0) + np.arange(64, dtype=np.float32) / 64
    return p


def _corner_scale(fld, p):
    i0 = np.floor(p.astype(np.float64)).astype(np.int64)
    m = np.zeros(len(p))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c = oracle.lookup(fld, i0 + [dx, dy, dz])
                m = np.maximum(m, np.abs(c))
    return m


@pytest.mark.parametrize("shape,q", [((64, 64, 64), 0.25), ((37, 50, 70), 0.5),
                                     ((130, 20, 140), 0.1)])
def test_trilinear_vdb_and_dense_within_1e6(shape, q):
    v = _rand(shape, 43, zero=0.4)
    buf, st = vdbc.encode(v, q)
    g = vdbc.Grid(buf)
    p = _positions(shape, 200_003, 44)
    fv = oracle.VdbField(buf)
    want = oracle.sample(fv, p)
    got = vdbc.sample(g, _cuda(p)).cpu().numpy().astype(np.float64)
    tol = 1e-6 * _corner_scale(fv, p) + 1e-30
    assert np.all(np.abs(got - want) <= tol)
    # dense baseline on the original grid
    fd = oracle.DenseField(v, st["background"])
    want_d = oracle.sample(fd, p)
    got_d = vdbc.sample_dense(_dense_t(v), st["background"], _cuda(p)).cpu().numpy()
    tol_d = 1e-6 * _corner_scale(fd, p) + 1e-30
    assert np.all(np.abs(got_d.astype(np.float64) - want_d) <= tol_d)


def test_nearest_bit_exact():
    shape = (37, 50, 70)
    v = _rand(shape, 45)
    buf, st = vdbc.encode(v, 0.4)
    g = vdbc.Grid(buf)
    p = _positions(shape, 50_001, 46)
    got = vdbc.sample(g, _cuda(p), filter=0).cpu().numpy()
    want = oracle.sample(oracle.VdbField(buf), p, filter=0).astype(np.float32)
    assert np.array_equal(got, want)
    got_d = vdbc.sample_dense(_dense_t(v), st["background"], _cuda(p), filter=0).cpu().numpy()
    want_d = oracle.sample(oracle.DenseField(v, st["background"]), p, filter=0).astype(np.float32)
    assert np.array_equal(got_d, want_d)


def test_lossless_vdb_sample_equals_dense_bitwise():
    shape = (70, 33, 45)
    v = _rand(shape, 47, zero=0.5)
    buf, st = vdbc.encode(v, 1.0)
    g = vdbc.Grid(buf)
    p = _positions(shape, 100_000, 48)
    a = vdbc.sample(g, _cuda(p)).cpu().numpy()
    b = vdbc.sample_dense(_dense_t(v), st["background"], _cuda(p)).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_sample_edge_cases():
    # empty input, a single voxel volume, one position
    v = np.full((1, 1, 1), 0.5, np.float32)
    buf, st = vdbc.encode(v, 1.0)
    g = vdbc.Grid(buf)
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    assert vdbc.sample(g, empty).numel() == 0
    p = np.array([[0, 0, 0], [0.25, 0, 0], [-1, 0, 0], [5, 5, 5]], np.float32)
    got = vdbc.sample(g, _cuda(p)).cpu().numpy()
    want = oracle.sample(oracle.VdbField(buf), p)
    assert np.allclose(got, want, atol=1e-7, rtol=0)
    # far away positions read the background
    far = np.array([[1e9, -1e9, 3e7], [-5e5, 0, 0]], np.float32)
    assert np.all(vdbc.sample(g, _cuda(far)).cpu().numpy() == st["background"])


def test_full_size_lookup_and_sample_mid_volume():
    # the 512^3 cloud at 1:10 that the benchmark renders: sampled lookups,
    # every voxel on brick/leaf boundary planes of a slab, random samples
    v = synth.mid_volume()
    buf, st = vdbc.encode(v, 0.10)
    g = vdbc.Grid(buf)
    fld = oracle.VdbField(buf)
    rng = np.random.default_rng(49)
    ijk = rng.integers(-1, 513, size=(1_000_000, 3)).astype(np.int32)
    yy, zz = np.meshgrid(np.arange(512), np.arange(0, 512, 31), indexing="ij")
    for x in (7, 8, 31, 32, 127, 128, 255, 256, 511):
        ijk = np.concatenate([ijk, np.stack([np.full(yy.size, x), yy.ravel(), zz.ravel()],
                                            1).astype(np.int32)])
    got = vdbc.lookup(g, _cuda(ijk)).cpu().numpy()
    want = oracle.lookup(fld, ijk.astype(np.int64))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    p = _positions(v.shape, 500_000, 50)
    got = vdbc.sample(g, _cuda(p)).cpu().numpy().astype(np.float64)
    want = oracle.sample(fld, p)
    assert np.all(np.abs(got - want) <= 1e-6 * _corner_scale(fld, p) + 1e-30)


# ---------------------------------------------------------------- majorant

TF5 = dict(tf=[(0.2, 0.3, 0.9, 0.0), (0.9, 0.1, 0.2, 0.8), (0.4, 0.4, 0.4, 0.3),
               (1.0, 1.0, 0.0, 1.0), (0.0, 1.0, 1.0, 0.5)], tf_range=(0.1, 0.9))


@pytest.mark.parametrize("C", [4, 8, 16, 64])
def test_majorant_vs_oracle(C):
    shape = (45, 37, 70)
    v = _rand(shape, 51, zero=0.5)
    buf, st = vdbc.encode(v, 0.4)
    med = dict(sigma_scale=6.0, **TF5)
    got = vdbc.majorant(vdbc.Grid(buf), med, C).cpu().numpy()
    want = oracle.majorant(oracle.VdbField(buf), med, C)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-12)
    got_d = vdbc.majorant(_dense_t(v), med, C, background=st["background"]).cpu().numpy()
    want_d = oracle.majorant(oracle.DenseField(v, st["background"]), med, C)
    np.testing.assert_allclose(got_d, want_d, rtol=2e-6, atol=1e-12)


@pytest.mark.parametrize("C", [4, 8, 16, 32, 64])
def test_majorant_of_tree_equals_majorant_of_its_reconstruction(C):
    # the VDB majorant reads leaf regions (one value for a tile or empty
    # region), the dense one every voxel: on the reconstructed grid the two
    # must agree bit for bit, with tiles, empty regions, ragged edge bricks
    # and footprints reaching outside the volume; lossless and 1:5, plus the
    # partial-brick encoding
    shape = (70, 45, 133)
    v = _rand(shape, 52, zero=0.7)
    v[:40, :32, :64] = np.float32(0.5)      # uniform region: tiles after pruning
    med = dict(sigma_scale=6.0, **TF5)
    for q, part in ((1.0, None), (0.2, None), (0.2, (0.5, 1e30))):
        buf, st = vdbc.encode(v, q, partial=part)
        R = oracle.reconstruct(v, q, partial=part)
        got = vdbc.majorant(vdbc.Grid(buf), med, C).cpu().numpy()
        want = vdbc.majorant(_dense_t(R), med, C, background=st["background"]).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (q, part)


# ---------------------------------------------------------------- EA

def _tiny():
    v = synth.tiny_volume()
    buf, st = vdbc.encode(v, synth.scenes.TINY["rate"])
    return v, buf, st


def test_ea_tiny_config_within_1e5():
    # 64^3 sphere cloud at 1:4, 128x128 orthographic, step 0.5, sigma_t = 8 density
    v, buf, st = _tiny()
    cam = scenes.ortho_z_camera(64, 64, 128, 128)
    med = scenes.ea_medium(8.0)
    prm = dict(step=0.5)
    want = oracle.render_ea(oracle.VdbField(buf), cam, med, prm)
    got = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_EA).cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-5
    want_d = oracle.render_ea(oracle.DenseField(v, 0.0), cam, med, prm)
    got_d = vdbc.render(_dense_t(v), cam, med, prm, vdbc.MODE_EA, background=0.0).cpu().numpy()
    assert np.max(np.abs(got_d - want_d)) <= 1e-5


def test_ea_pinhole_and_hdda_bitwise():
    v, buf, st = _tiny()
    g = vdbc.Grid(buf)
    cam = scenes.orbit_camera((64, 64, 64), 96, 80)
    med = scenes.ea_medium(8.0)
    prm = dict(step=0.5)
    want = oracle.render_ea(oracle.VdbField(buf), cam, med, prm)
    off = vdbc.render(g, cam, med, prm, vdbc.MODE_EA).cpu().numpy()
    on = vdbc.render(g, cam, med, dict(step=0.5, flags=vdbc.RENDER_HDDA), vdbc.MODE_EA)
    on = on.cpu().numpy()
    assert np.max(np.abs(off - want)) <= 1e-5
    assert np.array_equal(on.view(np.uint32), off.view(np.uint32))
    # HDDA also skips on a sparse 1:20 grid with big empty nodes
    big = synth.mid_volume(n=256)
    b2, _ = vdbc.encode(big, 0.05)
    g2 = vdbc.Grid(b2)
    cam2 = scenes.orbit_camera((256, 256, 256), 64, 64)
    a = vdbc.render(g2, cam2, med, prm, vdbc.MODE_EA).cpu().numpy()
    b = vdbc.render(g2, cam2, med, dict(step=0.5, flags=vdbc.RENDER_HDDA), vdbc.MODE_EA)
    assert np.array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32))


def test_ea_lossless_vdb_equals_dense_bitwise():
    v = synth.tiny_volume()
    buf, st = vdbc.encode(v, 1.0)
    cam = scenes.orbit_camera((64, 64, 64), 64, 48)
    med = scenes.ea_medium(8.0)
    a = vdbc.render(vdbc.Grid(buf), cam, med, dict(step=0.5), vdbc.MODE_EA).cpu().numpy()
    b = vdbc.render(_dense_t(v), cam, med, dict(step=0.5), vdbc.MODE_EA, background=0.0)
    assert np.array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32))


def test_ea_sample_count():
    v, buf, st = _tiny()
    cam = scenes.ortho_z_camera(64, 64, 128, 128)
    med = scenes.ea_medium(8.0)
    r = vdbc.Renderer(vdbc.Grid(buf), cam, med, dict(step=0.5, flags=vdbc.RENDER_COUNT),
                      vdbc.MODE_EA)
    r.launch()
    torch.cuda.synchronize()
    assert r.sample_count() == 128 * 128 * 128   # 64 voxels / 0.5 per ray


# ---------------------------------------------------------------- PT

def _pt_scene(n, w, h, spp, seed=0x5EED, bounces=8):
    cam = scenes.orbit_camera((n, n, n), w, h)
    med = scenes.pt_medium(64.0)
    prm = dict(spp=spp, max_bounces=bounces, seed=seed, macrocell=8)
    return cam, med, prm


@pytest.mark.parametrize("q", [0.25, 0.10, 0.05])
def test_pt_small_relmse(q):
    v = synth.mid_volume(n=96)
    buf, st = vdbc.encode(v, q)
    cam, med, prm = _pt_scene(96, 52, 44, 4)
    want, want_aov = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, aov=True)
    img, aov = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT, aov=True)
    got = img.cpu().numpy().reshape(-1, 4)
    assert relmse(got, want) <= 1e-4
    assert relmse(aov.cpu().numpy().reshape(-1, 2), want_aov) <= 1e-4
    want_d = oracle.render_pt(oracle.DenseField(v, 0.0), cam, med, prm)
    got_d = vdbc.render(_dense_t(v), cam, med, prm, vdbc.MODE_PT, background=0.0)
    assert relmse(got_d.cpu().numpy().reshape(-1, 4), want_d) <= 1e-4


@pytest.mark.parametrize("q,C", [(0.25, 8), (0.10, 8), (0.05, 8), (0.10, 16)])
def test_pt_coloured_five_point_tf_vs_oracle(q, C):
    # the coloured five-point transfer function: alpha interval search in the
    # LDS copy of the control points, throughput weighted by the interpolated
    # colour per channel; 1:4, 1:10 and 1:20
    v = synth.mid_volume(n=96)
    buf, _ = vdbc.encode(v, q)
    cam = scenes.orbit_camera((96, 96, 96), 52, 44)
    med = scenes.pt_medium_tf5(64.0)
    prm = dict(spp=4, max_bounces=8, seed=0x5EED, macrocell=C)
    want, want_aov = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, aov=True)
    img, aov = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT, aov=True)
    got = img.cpu().numpy().reshape(-1, 4)
    assert relmse(got, want) <= 1e-4
    assert relmse(aov.cpu().numpy().reshape(-1, 2), want_aov) <= 1e-4
    # the image is coloured: red and blue differ by much more than the noise
    assert np.abs(want[:, 0] - want[:, 2]).max() > 0.05
    want_d = oracle.render_pt(oracle.DenseField(v, 0.0), cam, med, prm)
    got_d = vdbc.render(_dense_t(v), cam, med, prm, vdbc.MODE_PT, background=0.0)
    assert relmse(got_d.cpu().numpy().reshape(-1, 4), want_d) <= 1e-4


def test_pt_mid_config_coloured_1to20_sampled_pixels():
    # the mid configuration at 1:20 (512^3, 1024x1024, 16 spp, 8 bounces) with
    # the coloured five-point transfer function, on sampled pixels
    v = synth.mid_volume()
    buf, _ = vdbc.encode(v, 0.05)
    M = scenes.MID
    cam = scenes.orbit_camera((512, 512, 512), M["width"], M["height"])
    med = scenes.pt_medium_tf5(64.0)
    prm = dict(spp=M["spp"], max_bounces=M["max_bounces"], seed=M["seed"], macrocell=16)
    img = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
    rng = np.random.default_rng(54)
    pix = np.sort(rng.choice(M["width"] * M["height"], 192, replace=False)).astype(np.uint32)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, pixels=pix)
    assert relmse(img[pix], want) <= 1e-4
    assert np.all(np.isfinite(img)) and np.count_nonzero(want[:, 3] > 0) >= 32


@pytest.mark.parametrize("kind", ["vdb", "dense"])
def test_pt_pinhole_camera_rays_see_their_texels(kind):
    # the pinhole camera's ray directions through the image-based light:
    # every pixel whose whole footprint (and a 10 % margin) sees one texel of
    # the map returns exactly that texel (texels from the camera definition
    # in float64 on the host)
    from tests.test_oracle_render import pinhole_texel_cases
    n, env, cam, want = pinhole_texel_cases()
    z = np.zeros((n, n, n), np.float32)
    med = dict(scenes.pt_medium(16.0), env=_cuda(env))
    prm = dict(spp=5, max_bounces=2, seed=2)
    if kind == "vdb":
        img = vdbc.render(vdbc.Grid(vdbc.encode(z, 0.5)[0]), cam, med, prm, vdbc.MODE_PT)
    else:
        img = vdbc.render(_dense_t(z), cam, med, prm, vdbc.MODE_PT, background=0.0)
    ok = want >= 0
    got = img.cpu().numpy()[..., :3]
    assert np.array_equal(got[ok], env.reshape(-1, 3)[want[ok]])


def test_pt_lossless_vdb_equals_dense_bitwise_and_deterministic():
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 1.0)
    cam, med, prm = _pt_scene(64, 40, 36, 3)
    g = vdbc.Grid(buf)
    a = vdbc.render(g, cam, med, prm, vdbc.MODE_PT).cpu().numpy()
    a2 = vdbc.render(g, cam, med, prm, vdbc.MODE_PT).cpu().numpy()
    b = vdbc.render(_dense_t(v), cam, med, prm, vdbc.MODE_PT, background=0.0).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), a2.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_pt_white_furnace_and_zero_density():
    n = 32
    v = np.full((n, n, n), 1.0, np.float32)
    buf, _ = vdbc.encode(v, 1.0)
    cam = scenes.orbit_camera((n, n, n), 24, 24)
    med = dict(sigma_scale=40.0, albedo=1.0, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 1, 0), light_E=(0, 0, 0), ambient=(0.25, 0.5, 1.0))
    img = vdbc.render(vdbc.Grid(buf), cam, med, dict(spp=4, max_bounces=65535, seed=3),
                      vdbc.MODE_PT).cpu().numpy()
    np.testing.assert_allclose(img[..., :3], np.broadcast_to([0.25, 0.5, 1.0], img[..., :3].shape),
                               rtol=1e-6)
    z = np.zeros((n, n, n), np.float32)
    img = vdbc.render(_dense_t(z), cam, scenes.pt_medium(), dict(spp=2, seed=3), vdbc.MODE_PT,
                      background=0.0).cpu().numpy()
    amb = np.asarray(scenes.pt_medium()["ambient"], np.float32)
    assert np.all(img[..., :3] == amb) and np.all(img[..., 3] == 0)


def test_pt_sample_count_and_ragged_image():
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.25)
    cam, med, prm = _pt_scene(64, 17, 5, 2)
    prm["flags"] = vdbc.RENDER_COUNT
    r = vdbc.Renderer(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT)
    img = r.launch().cpu().numpy()
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm)
    assert relmse(img.reshape(-1, 4), want) <= 1e-4
    assert r.sample_count() > 17 * 5 * 2


def test_pt_segment_count():
    # one bounce: every path has its camera segment and, where that segment
    # ends in a real collision, one shadow ray; the image's alpha is the
    # fraction of such paths (exact for 4 spp), so segments = paths + hits
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.25)
    g = vdbc.Grid(buf)
    w, h, spp = 37, 29, 4
    cam, med, prm = _pt_scene(64, w, h, spp, bounces=1)
    prm["flags"] = vdbc.RENDER_COUNT
    r = vdbc.Renderer(g, cam, med, prm, vdbc.MODE_PT)
    img = r.launch().cpu().numpy().reshape(-1, 4)
    hits = int(np.rint(img[:, 3] * spp).sum())
    assert 0 < hits < w * h * spp
    assert r.segment_count() == w * h * spp + hits
    # more bounces: between one and 2 * bounces segments per path, the same
    # count on a second launch
    cam, med, prm = _pt_scene(64, w, h, spp, bounces=8)
    prm["flags"] = vdbc.RENDER_COUNT
    r = vdbc.Renderer(g, cam, med, prm, vdbc.MODE_PT)
    r.launch()
    n1 = r.segment_count()
    r.launch()
    assert r.segment_count() == n1
    assert w * h * spp + hits <= n1 <= w * h * spp * 16


def test_pt_mid_config_sampled_pixels():
    # the benchmark's launch: 512^3 cloud at 1:10, 1024x1024, 16 spp, 8 bounces;
    # the oracle renders a sample of the pixels one by one
    v = synth.mid_volume()
    buf, st = vdbc.encode(v, 0.10)
    M = scenes.MID
    cam = scenes.orbit_camera((512, 512, 512), M["width"], M["height"])
    med = scenes.pt_medium(64.0)
    prm = dict(spp=M["spp"], max_bounces=M["max_bounces"], seed=M["seed"], macrocell=16)
    img = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
    rng = np.random.default_rng(52)
    pix = np.sort(rng.choice(M["width"] * M["height"], 192, replace=False)).astype(np.uint32)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, pixels=pix)
    assert relmse(img[pix], want) <= 1e-4
    assert np.all(np.isfinite(img))


@pytest.mark.parametrize("C,tw", [(16, 8), (64, 32), (64, 64)])
def test_pt_paper_launch_configuration_sampled_pixels(C, tw):
    # the paper-scale launch (1920x1080, 64 spp, <= 16 bounces, 1:10; the
    # benchmark's macrocell 64 with 64-wide wave tiles, the same cells with
    # 32-wide tiles, and macrocell 16) on
    # the same billowed recipe at 1/8 of the edge lengths; the oracle renders
    # a sample of the pixels one by one
    P = scenes.PAPER
    dims = tuple(d // 8 for d in P["dims"])
    v = synth.paper_volume(dims=dims)
    buf, _ = vdbc.encode(v, 0.10)
    cam = scenes.orbit_camera(dims, P["width"], P["height"])
    med = scenes.pt_medium(64.0)
    prm = dict(spp=P["spp"], max_bounces=P["max_bounces"], seed=P["seed"], macrocell=C, tile_w=tw)
    img = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
    rng = np.random.default_rng(53)
    pix = np.sort(rng.choice(P["width"] * P["height"], 1024, replace=False)).astype(np.uint32)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm, pixels=pix)
    assert relmse(img[pix], want) <= 1e-4
    assert np.all(np.isfinite(img)) and np.count_nonzero(want[:, 3] > 0) >= 32


def test_pt_image_independent_of_wave_tile_shape():
    v = synth.mid_volume(n=64)
    buf, _ = vdbc.encode(v, 0.25)
    g = vdbc.Grid(buf)
    cam, med, prm = _pt_scene(64, 70, 33, 2)
    imgs = []
    for tw in (8, 16, 32, 64):
        p = dict(prm, tile_w=tw)
        imgs.append(vdbc.render(g, cam, med, p, vdbc.MODE_PT).cpu().numpy())
    for im in imgs[1:]:
        assert np.array_equal(im.view(np.uint32), imgs[0].view(np.uint32))


def test_pt_russian_roulette_vs_oracle():
    # albedo 0.9 and 16 bounces: roulette from bounce 2 changes the draws and
    # ends paths early; the GPU must follow the oracle path by path
    v = synth.mid_volume(n=96)
    buf, _ = vdbc.encode(v, 0.25)
    cam, med, prm = _pt_scene(96, 48, 40, 4)
    prm = dict(prm, max_bounces=16, flags=vdbc.RENDER_RR, rr=True)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm)
    got = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
    assert relmse(got, want) <= 1e-4
    plain = vdbc.render(vdbc.Grid(buf), cam, med, dict(prm, flags=0), vdbc.MODE_PT)
    assert not np.array_equal(plain.cpu().numpy().reshape(-1, 4), got)
    want_d = oracle.render_pt(oracle.DenseField(v, 0.0), cam, med, prm)
    got_d = vdbc.render(_dense_t(v), cam, med, prm, vdbc.MODE_PT, background=0.0)
    assert relmse(got_d.cpu().numpy().reshape(-1, 4), want_d) <= 1e-4


def test_pt_russian_roulette_white_furnace():
    n = 32
    v = np.full((n, n, n), 1.0, np.float32)
    buf, _ = vdbc.encode(v, 1.0)
    cam = scenes.orbit_camera((n, n, n), 24, 24)
    med = dict(sigma_scale=40.0, albedo=1.0, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 1, 0), light_E=(0, 0, 0), ambient=(0.25, 0.5, 1.0))
    img = vdbc.render(vdbc.Grid(buf), cam, med,
                      dict(spp=4, max_bounces=65535, seed=3, flags=vdbc.RENDER_RR),
                      vdbc.MODE_PT).cpu().numpy()
    np.testing.assert_allclose(img[..., :3], np.broadcast_to([0.25, 0.5, 1.0], img[..., :3].shape),
                               rtol=1e-6)


def _env_map(w=64, h=32, seed=4):
    # smooth sky: brighter towards +y, with a warm patch and mild noise
    rng = np.random.default_rng(seed)
    v = (np.arange(h) + 0.5)[:, None] / h
    u = (np.arange(w) + 0.5)[None, :] / w
    sky = np.stack([0.3 + 0.7 * (1 - v) + 0 * u, 0.35 + 0.6 * (1 - v) + 0 * u,
                    0.5 + 0.5 * (1 - v) + 0 * u], -1)
    sky += 1.5 * np.exp(-((u - 0.3) ** 2 + (v - 0.35) ** 2) / 0.01)[..., None] * [1.0, 0.7, 0.3]
    sky += 0.02 * rng.random(sky.shape)
    return sky.astype(np.float32)


def test_pt_image_based_light_vs_oracle():
    v = synth.mid_volume(n=96)
    buf, _ = vdbc.encode(v, 0.25)
    cam, med, prm = _pt_scene(96, 48, 40, 4)
    env = _env_map()
    want = oracle.render_pt(oracle.VdbField(buf), cam, dict(med, env=env), prm)
    got = vdbc.render(vdbc.Grid(buf), cam, dict(med, env=_cuda(env)), prm, vdbc.MODE_PT)
    assert relmse(got.cpu().numpy().reshape(-1, 4), want) <= 1e-4
    want_d = oracle.render_pt(oracle.DenseField(v, 0.0), cam, dict(med, env=env), prm)
    got_d = vdbc.render(_dense_t(v), cam, dict(med, env=_cuda(env)), prm, vdbc.MODE_PT,
                        background=0.0)
    assert relmse(got_d.cpu().numpy().reshape(-1, 4), want_d) <= 1e-4
    # a constant map is the ambient term, bit for bit
    const = np.broadcast_to(np.asarray(med["ambient"], np.float32), (8, 16, 3)).copy()
    a = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).clone()
    b = vdbc.render(vdbc.Grid(buf), cam, dict(med, env=_cuda(const)), prm, vdbc.MODE_PT)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("direction,texel", [((1, 0, 0), (4, 2)), ((-1, 0, 0), (7, 2)),
                                             ((0, 1, 0), (4, 0)), ((0, -1, 0), (4, 3)),
                                             ((0, 0, 1), (6, 2)), ((0, 0, -1), (2, 2))])
def test_pt_env_map_axis_directions(direction, texel):
    n = 8
    env = np.zeros((4, 8, 3), np.float32)
    for y in range(4):
        for x in range(8):
            env[y, x] = (x, y, 100 + x + 8 * y)
    d = np.asarray(direction, np.float64)
    a = np.roll(d, 1)
    b = np.cross(d, a)
    cam = dict(kind=0, width=4, height=4, lower_left=tuple(-20.0 * d - a - b),
               du=tuple(0.5 * a), dv=tuple(0.5 * b), dir=tuple(d))
    med = dict(scenes.pt_medium(16.0), env=_cuda(env))
    img = vdbc.render(_dense_t(np.zeros((n, n, n), np.float32)), cam, med,
                      dict(spp=3, max_bounces=2, seed=1), vdbc.MODE_PT, background=0.0)
    assert np.array_equal(img.cpu().numpy()[..., :3].reshape(-1, 3),
                          np.tile(env[texel[1], texel[0]], (16, 1)))


@pytest.mark.parametrize("C", [4, 32, 64])
def test_pt_macrocell_sizes_vs_oracle(C):
    # the coarse-block skip covers 2^lf macrocells, blocks of at least 4 cells
    # and 64 voxels per axis: lf = 4 at C = 4, lf = 2 at C = 32 and 64; each
    # must follow the oracle's uniform walk
    v = synth.mid_volume(n=80)
    buf, _ = vdbc.encode(v, 0.25)
    cam, med, prm = _pt_scene(80, 40, 36, 3)
    prm = dict(prm, macrocell=C)
    want = oracle.render_pt(oracle.VdbField(buf), cam, med, prm)
    got = vdbc.render(vdbc.Grid(buf), cam, med, prm, vdbc.MODE_PT).cpu().numpy().reshape(-1, 4)
    assert relmse(got, want) <= 1e-4
