"""Pins for the oracle's level-0 reconstruction (Section 3.2.2: nearest and
trilinear interpolation, background where no voxel exists)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def _vol(shape, seed):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < 0.5] = 0.0
    return v


def test_trilinear_matches_library_interpolation():
    # scipy's order-1 spline with a constant outside the grid is trilinear
    # interpolation with B substituted for missing corners.
    v = _vol((20, 23, 26), 1)
    B = 0.0
    buf, _ = oracle.encode(v, 1.0)
    fv = oracle.VdbField(buf)
    fd = oracle.DenseField(v, B)
    rng = np.random.default_rng(2)
    p = rng.uniform(-1.5, 27.5, size=(20000, 3)).astype(np.float32)
    want = ndimage.map_coordinates(v.astype(np.float64), p[:, ::-1].T.astype(np.float64),
                                   order=1, mode="grid-constant", cval=B)
    for f in (fv, fd):
        got = oracle.sample(f, p)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_trilinear_on_lossy_grid_matches_reconstruction():
    v = _vol((40, 40, 40), 3)
    buf, st = oracle.encode(v, 0.4)
    R = oracle.reconstruct(v, 0.4)
    f = oracle.VdbField(buf)
    rng = np.random.default_rng(4)
    p = rng.uniform(-1, 41, size=(20000, 3)).astype(np.float32)
    want = ndimage.map_coordinates(R.astype(np.float64), p[:, ::-1].T.astype(np.float64),
                                   order=1, mode="grid-constant", cval=st["background"])
    np.testing.assert_allclose(oracle.sample(f, p), want, rtol=0, atol=1e-12)


def test_integer_positions_are_lookups():
    v = _vol((17, 18, 19), 5)
    buf, _ = oracle.encode(v, 0.5)
    f = oracle.VdbField(buf)
    rng = np.random.default_rng(6)
    ijk = rng.integers(-2, 21, size=(5000, 3))
    got = oracle.sample(f, ijk.astype(np.float32))
    want = oracle.lookup(f, ijk).astype(np.float64)
    assert np.array_equal(got, want)
    got0 = oracle.sample(f, ijk.astype(np.float32), filter=0)
    assert np.array_equal(got0, want)


def test_affine_field_is_reproduced():
    # trilinear interpolation reproduces affine functions exactly (up to
    # rounding) wherever all 8 corners are inside the grid
    n = 24
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    v = (0.25 * x - 0.125 * y + 0.0625 * z + 1.0).astype(np.float32)
    buf, _ = oracle.encode(v, 1.0)
    f = oracle.VdbField(buf)
    rng = np.random.default_rng(7)
    p = rng.uniform(0, n - 1, size=(5000, 3)).astype(np.float32)
    p64 = p.astype(np.float64)
    want = 0.25 * p64[:, 0] - 0.125 * p64[:, 1] + 0.0625 * p64[:, 2] + 1.0
    np.testing.assert_allclose(oracle.sample(f, p), want, rtol=0, atol=1e-12)


def test_constant_field_is_constant_everywhere():
    v = np.full((30, 31, 32), 0.375, np.float32)
    buf, st = oracle.encode(v, 1.0)
    assert st["background"] == 0.375
    f = oracle.VdbField(buf)
    rng = np.random.default_rng(8)
    p = rng.uniform(-50, 80, size=(3000, 3)).astype(np.float32)
    assert np.all(oracle.sample(f, p) == 0.375)


def test_nearest_rounds_half_up():
    v = np.arange(4 * 4 * 4, dtype=np.float32).reshape(4, 4, 4) + 1
    f = oracle.DenseField(v, 0.0)
    p = np.array([[1.5, 1.0, 1.0], [1.49, 1.0, 1.0], [2.0, 2.5, 0.5], [-0.5, 0, 0],
                  [-0.51, 0, 0]], np.float32)
    got = oracle.sample(f, p, filter=0)
    assert list(got) == [v[1, 1, 2], v[1, 1, 1], v[1, 3, 2], v[0, 0, 0], 0.0]


def test_dense_and_lossless_vdb_agree_bitwise():
    v = _vol((33, 34, 35), 9)
    buf, st = oracle.encode(v, 1.0)
    fv = oracle.VdbField(buf)
    fd = oracle.DenseField(v, st["background"])
    rng = np.random.default_rng(10)
    p = rng.uniform(-2, 37, size=(20000, 3)).astype(np.float32)
    assert np.array_equal(oracle.sample(fv, p), oracle.sample(fd, p))
