"""Pins for the oracle's partial-brick activation, the variant Section 3.2.1
leaves as future work (past a similarity threshold, a share of each brick's
voxels in proportionally more bricks, e.g. half of them in twice as many
bricks).  The paper gives no rule for which voxels to keep; the
oracle's rule (fraction p, similarity threshold tau, voxels by |value - B|
inside a brick) is checked here by what must hold for it whatever its code:
the paper's own half/twice example, the exact voxel budget of plain Alg. 1,
reduction to Alg. 1, losslessness at 1:1, nesting in the rate, and that a
partially kept brick keeps its most dissimilar voxels."""
import numpy as np
import pytest

import oracle
import synth
from tests import fmt


def _cloud(shape, seed, frac_zero=0.5):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < frac_zero] = 0.0
    return v


def _bricks(shape):
    nz, ny, nx = shape
    nbx, nby, nbz = -(-nx // 32), -(-ny // 32), -(-nz // 32)
    out = []
    for b in range(nbx * nby * nbz):
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        out.append(np.s_[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32])
    return out


def _similarity(v, metric=2):
    # Eq. (1)-(3) per brick from numpy ranges (the oracle's are pinned against
    # brute force elsewhere)
    B = oracle.background(v)
    f = []
    for sl in _bricks(v.shape):
        lo, hi = float(v[sl].min()), float(v[sl].max())
        dl, dh = abs(lo - B), abs(hi - B)
        f.append({1: min(dl, dh), 2: max(dl, dh), 3: abs((lo + hi) / 2 - B)}[metric])
    return np.array(f), B


SHAPES = [(64, 96, 128), (45, 70, 37), (33, 64, 100)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fraction_one_or_low_threshold_is_alg1(shape):
    v = _cloud(shape, 3)
    for q in (0.1, 0.3, 0.6):
        plain = oracle.reconstruct(v, q)
        for part in ((1.0, 1e30), (1.0, 0.0), (0.5, -1.0), (0.25, -1.0)):
            R = oracle.reconstruct(v, q, partial=part)
            assert np.array_equal(R.view(np.uint32), plain.view(np.uint32)), (q, part)
        # the buffers differ only in the header's flag and the recorded p, tau
        b0, _ = oracle.encode(v, q)
        b1, _ = oracle.encode(v, q, partial=(0.5, -1.0))
        d = np.nonzero(b0 != b1)[0]
        assert set(d.tolist()) <= set(range(32, 36)) | set(range(160, 168))
        h = fmt.header(b1)
        assert h["flags"] == oracle.PARTIAL


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("q", [0.05, 0.2, 0.5])
@pytest.mark.parametrize("p", [0.5, 0.3, 0.1])
def test_active_count_is_the_plain_budget(shape, q, p):
    # the voxels of the K bricks plain Alg. 1 keeps, to the voxel, whatever
    # the threshold (no corners, so nothing else is active)
    v = _cloud(shape, 5)
    order, K = oracle.brick_order(v, q)
    bricks = _bricks(shape)
    budget = sum(v[bricks[b]].size for b in order[:K])
    f, _ = _similarity(v)
    for tau in (1e30, float(np.median(f)), -1.0):
        m = oracle.active_mask(v, q, flags=oracle.REF_NO_CORNERS, partial=(p, tau))
        assert int(m.sum()) == budget, tau


def test_half_the_voxels_of_twice_the_bricks():
    # the paper's example: with a threshold above every brick, half of each
    # brick's voxels in twice as many bricks (no edge bricks here)
    v = _cloud((64, 128, 128), 8)
    order, K = oracle.brick_order(v, 0.25)
    m = oracle.active_mask(v, 0.25, flags=oracle.REF_NO_CORNERS, partial=(0.5, 1e30))
    counts = np.array([int(m[sl].sum()) for sl in _bricks(v.shape)])
    assert K == 8 and np.count_nonzero(counts) == 2 * K
    assert set(counts[counts > 0].tolist()) == {32 ** 3 // 2}
    # ... and they are the 2K most dissimilar bricks
    assert set(np.nonzero(counts)[0].tolist()) == set(order[:2 * K].tolist())


@pytest.mark.parametrize("shape", SHAPES)
def test_bricks_above_threshold_kept_whole(shape):
    v = _cloud(shape, 9)
    f, _ = _similarity(v)
    q = 0.3
    order, K = oracle.brick_order(v, q)
    tau = float(np.sort(f[order[:K]])[K // 2])   # about half of the K bricks reach it
    m = oracle.active_mask(v, q, flags=oracle.REF_NO_CORNERS, partial=(0.5, tau))
    bricks = _bricks(shape)
    F = int(np.sum(f[order[:K]] >= tau))
    assert 0 < F < K
    for r, b in enumerate(order):
        n = int(m[bricks[b]].sum())
        if r < F:
            assert n == v[bricks[b]].size, r          # whole
        else:
            assert n < v[bricks[b]].size or f[b] == f[order[F]], r


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("p,tau", [(0.5, 1e30), (0.2, 1e30), (0.35, "mid-rank")])
def test_kept_voxels_are_the_most_dissimilar_of_their_brick(shape, p, tau):
    # inside every brick, no inactive voxel is farther from B than an active
    # one; among equal distances the active ones have the smaller index
    v = _cloud(shape, 12, frac_zero=0.3)
    v[v > 0.9] = np.float32(0.95)            # ties in |v - B|
    bricks = _bricks(shape)
    for b, sl in enumerate(bricks):          # bricks of different similarity
        v[sl] *= np.float32(0.3 + 0.7 * b / len(bricks))
    B = oracle.background(v)
    if tau == "mid-rank":                    # about half the K bricks stay whole
        order, K = oracle.brick_order(v, 0.2)
        tau = float(np.nextafter(np.float32(_similarity(v)[0][order[K // 2]]), np.float32(2)))
    m = oracle.active_mask(v, 0.2, flags=oracle.REF_NO_CORNERS, partial=(p, tau))
    idx = np.arange(v.size).reshape(v.shape)
    partial_seen = 0
    for sl in _bricks(shape):
        a, d, i = m[sl].ravel(), np.abs(v[sl].astype(np.float64).ravel() - B), idx[sl].ravel()
        if a.all() or not a.any():
            continue
        partial_seen += 1
        assert d[a].min() >= d[~a].max()
        t = d[a].min()
        if t == d[~a].max():
            assert i[a & (d == t)].max() < i[~a & (d == t)].min()
    assert partial_seen >= 1


@pytest.mark.parametrize("p,tau", [(0.5, 1e30), (0.25, 0.6)])
def test_nested_in_rate_and_error_non_increasing(p, tau):
    v = synth.mid_volume(n=128)
    prev_m, prev_mse = None, None
    for q in (0.02, 0.05, 0.1, 0.2, 0.4, 0.7, 1.0):
        m = oracle.active_mask(v, q, partial=(p, tau))
        R = oracle.reconstruct(v, q, partial=(p, tau))
        mse = float(((R.astype(np.float64) - v) ** 2).mean())
        if prev_m is not None:
            assert np.all(m[prev_m]), q
            assert mse <= prev_mse, q
        prev_m, prev_mse = m, mse
    assert prev_mse == 0.0


@pytest.mark.parametrize("shape", SHAPES + [(1, 1, 1), (8, 200, 9)])
@pytest.mark.parametrize("p", [0.5, 0.01])
def test_rate_one_is_lossless(shape, p):
    v = _cloud(shape, 14)
    R = oracle.reconstruct(v, 1.0, partial=(p, 1e30))
    assert np.array_equal(R.view(np.uint32), v.view(np.uint32))


def test_reconstruction_and_buffer_lookup_agree_with_the_mask():
    v = _cloud((45, 70, 90), 17, frac_zero=0.6)
    v[:20, :30, :40] = np.float32(0.75)       # uniform regions: tiles after pruning
    for part, flags in (((0.5, 1e30), 0), ((0.3, 0.5), oracle.REF_NO_PRUNE), ((0.7, 0.2), 0)):
        m = oracle.active_mask(v, 0.3, flags=flags, partial=part)
        R = oracle.reconstruct(v, 0.3, flags=flags, partial=part)
        B = oracle.background(v)
        assert np.array_equal(R, np.where(m, v, np.float32(B)))
        buf, st = oracle.encode(v, 0.3, flags=flags, partial=part)
        assert st["active_voxels"] == int(m.sum())
        h = fmt.header(buf)
        assert h["total_bytes"] == len(buf) == fmt.expected_size(h)
        nz, ny, nx = v.shape
        g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
        ijk = g.reshape(-1, 3)
        got = oracle.lookup(oracle.VdbField(buf), ijk)
        assert np.array_equal(got.view(np.uint32), R[ijk[:, 2], ijk[:, 1], ijk[:, 0]].view(np.uint32))
        masks = np.frombuffer(bytes(buf[h["off_leaf_masks"]:h["off_leaf_masks"] + 64 * h["n_leaf"]]),
                              "<u8")
        in_tiles = 512 * h["n_lower_tiles"] + 512 * 4096 * h["n_upper_tiles"]
        assert int(fmt.popcount64(masks).sum()) + in_tiles == int(m.sum())


def test_rejects_bad_partial_parameters():
    v = _cloud((32, 32, 32), 1)
    for part in ((0.0, 1.0), (1.5, 1.0), (float("nan"), 1.0), (0.5, float("nan"))):
        with pytest.raises(Exception):
            oracle.reconstruct(v, 0.5, partial=part)
