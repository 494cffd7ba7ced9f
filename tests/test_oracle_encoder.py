"""Pins for the oracle encoder (Alg. 1 "Compress", Section 3.1; tree and
linearisation, Section 3.2).  Each test checks the oracle against something
other than itself: brute force, closed forms, or a statement of the paper."""
from collections import Counter

import numpy as np
import pytest

import oracle
import synth
from tests import fmt


def _rand_cloud(shape, seed, frac_zero=0.6):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < frac_zero] = 0.0
    return v


def _mode_bruteforce(v):
    c = Counter(float(x) + 0.0 for x in v.ravel())  # -0 + 0 -> +0
    best = max(c.values())
    return min(x for x, n in c.items() if n == best)


# ---------------------------- background (Alg. 1 histogram/argmax) ----------

def test_background_exact_mode_bruteforce():
    rng = np.random.default_rng(3)
    for trial in range(20):
        v = rng.integers(-3, 4, size=(5, 6, 7)).astype(np.float32) * np.float32(0.25)
        assert oracle.background(v) == _mode_bruteforce(v)


def test_background_negative_zero_and_ties():
    v = np.array([-0.0, -0.0, 0.0, 1.0, 1.0, 1.0, 2.0], np.float32).reshape(1, 1, 7)
    b = oracle.background(v)
    assert b == 0.0 and not np.signbit(b)  # 3 zeros tie with 3 ones -> smaller
    v = np.array([5.0, 5.0, -1.0, -1.0], np.float32).reshape(1, 1, 4)
    assert oracle.background(v) == -1.0


def test_background_sparse_volume_is_empty_space():
    # Section 3.1: the background is the value most voxels hold (empty space)
    assert oracle.background(synth.tiny_volume()) == 0.0


# ---------------------------- bricks and similarity -------------------------

def test_brick_ranges_bruteforce_with_partial_bricks():
    v = _rand_cloud((45, 33, 70), 1)
    lo, hi = oracle.brick_ranges(v)
    nz, ny, nx = v.shape
    nbx, nby, nbz = -(-nx // 32), -(-ny // 32), -(-nz // 32)
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                blk = v[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32]
                b = bx + nbx * (by + nby * bz)
                assert lo[b] == blk.min() and hi[b] == blk.max()


def test_similarity_equations():
    # Eq. (1)-(3) at lo=0.25, hi=1.0, B=0.5: closest 0.25, farthest 0.5,
    # median |0.625-0.5| = 0.125
    assert oracle.similarity(1, 0.25, 1.0, 0.5) == 0.25
    assert oracle.similarity(2, 0.25, 1.0, 0.5) == 0.5
    assert oracle.similarity(3, 0.25, 1.0, 0.5) == 0.125
    # a range [B:B] is most similar under every metric
    for m in (1, 2, 3):
        assert oracle.similarity(m, 0.5, 0.5, 0.5) == 0.0


@pytest.mark.parametrize("metric", [1, 2, 3])
@pytest.mark.parametrize("rate", [0.05, 0.1, 0.25, 0.5, 0.7, 1.0])
def test_brick_order_bruteforce(metric, rate):
    v = _rand_cloud((64, 96, 100), 5 + metric)
    v[:, :, :40] = 0.0     # many exact ties (f = 0)
    B = oracle.background(v)
    order, K = oracle.brick_order(v, rate, metric)
    lo, hi = oracle.brick_ranges(v)
    f = []
    for b in range(len(lo)):
        dl, dh = abs(float(lo[b]) - B), abs(float(hi[b]) - B)
        f.append({1: min(dl, dh), 2: max(dl, dh),
                  3: abs((float(lo[b]) + float(hi[b])) / 2 - B)}[metric])
    want = sorted(range(len(lo)), key=lambda b: (-f[b], b))
    assert list(order) == want
    N = len(lo)
    assert K == min(N, int(np.floor(np.float64(np.float32(rate)) * N + 0.5)))


def test_k_closed_form_float_rates():
    v = _rand_cloud((32, 32, 320), 2)  # 10 bricks
    for q, k in [(0.7, 7), (0.1, 1), (0.05, 1), (0.04, 0), (1.0, 10), (0.25, 3)]:
        _, K = oracle.brick_order(v, q)
        assert K == k, (q, K)


# ---------------------------- reconstruction -------------------------------

@pytest.mark.parametrize("shape", [(64, 64, 64), (37, 50, 70), (1, 1, 1), (8, 8, 200)])
def test_rate_one_is_lossless(shape):
    # Section 5.1: at 1:1 the encoding loses nothing
    v = _rand_cloud(shape, 11)
    R = oracle.reconstruct(v, 1.0)
    assert np.array_equal(R.view(np.uint32), v.view(np.uint32))


def test_reconstruction_is_selection():
    v = _rand_cloud((64, 64, 96), 4)
    for metric in (1, 2, 3):
        order, K = oracle.brick_order(v, 0.25, metric)
        R = oracle.reconstruct(v, 0.25, metric)
        B = oracle.background(v)
        want = np.full_like(v, B)
        for b in order[:K]:
            bx, by, bz = b % 3, (b // 3) % 2, b // 6
            sl = np.s_[bz * 32:(bz + 1) * 32, by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32]
            want[sl] = v[sl]
        want[0, 0, 0] = v[0, 0, 0]
        want[-1, -1, -1] = v[-1, -1, -1]
        assert np.array_equal(R, want)


def test_mse_non_increasing_and_prefix_nesting():
    # Table tab:stats: error falls as the rate rises and reaches 0.
    v = synth.mid_volume(n=128)
    prev = None
    prev_sel = None
    for q in (0.05, 0.1, 0.2, 0.3, 0.5, 1.0):
        R = oracle.reconstruct(v, q)
        mse = float(((R.astype(np.float64) - v) ** 2).mean())
        sel = R != oracle.background(v)
        if prev is not None:
            assert mse <= prev
            assert np.all(sel[prev_sel])   # earlier selection is kept
        prev, prev_sel = mse, sel
    assert prev == 0.0


def test_farthest_and_median_beat_closest():
    # Section 5.2: farthest / median point-in-range beat closest (PSNR).
    v = synth.mid_volume(n=128)
    mse = {}
    for m in (1, 2, 3):
        R = oracle.reconstruct(v, 0.1, m)
        mse[m] = float(((R.astype(np.float64) - v) ** 2).mean())
    assert mse[2] < mse[1] and mse[3] < mse[1]


def test_corners_and_explicit_background():
    v = np.full((40, 40, 40), 0.5, np.float32)
    v[0, 0, 0] = 0.9
    v[-1, -1, -1] = 0.1
    R = oracle.reconstruct(v, 0.01, flags=oracle.REF_BG_EXPLICIT, bg=0.5)
    assert R[0, 0, 0] == np.float32(0.9) and R[-1, -1, -1] == np.float32(0.1)
    R = oracle.reconstruct(v, 0.01, flags=oracle.REF_BG_EXPLICIT | oracle.REF_NO_CORNERS,
                           bg=0.25)
    # q=0.01 of 8 bricks -> K=0: everything background, corners dropped
    assert np.all(R == np.float32(0.25))


def test_rejects_bad_input():
    v = np.zeros((4, 4, 4), np.float32)
    for q in (0.0, -0.1, 1.5, float("nan")):
        with pytest.raises(oracle.OracleError):
            oracle.encode(v, q)
    w = v.copy()
    w[1, 2, 3] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.encode(w, 0.5)
    w[1, 2, 3] = np.inf
    with pytest.raises(oracle.OracleError):
        oracle.encode(w, 0.5)
    with pytest.raises(oracle.OracleError):
        oracle.encode(v, 0.5, metric=4)


# ---------------------------- buffer ---------------------------------------

def _all_ijk(shape):
    nz, ny, nx = shape
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    return g.reshape(-1, 3)


CASES = [((64, 64, 64), 0.25, 2, 0), ((37, 50, 70), 0.3, 1, 0), ((37, 50, 70), 0.3, 3,
         oracle.REF_NO_PRUNE), ((130, 20, 140), 0.5, 2, oracle.REF_NO_CORNERS),
         ((8, 8, 8), 1.0, 2, 0), ((200, 9, 3), 0.6, 2, 0)]


@pytest.mark.parametrize("shape,q,metric,flags", CASES)
def test_lookup_equals_reconstruction_every_voxel(shape, q, metric, flags):
    v = _rand_cloud(shape, 21)
    # flat regions so that pruning produces tiles
    v[: shape[0] // 2, : shape[1] // 2, : shape[2] // 2] = np.float32(0.75)
    buf, st = oracle.encode(v, q, metric, flags)
    R = oracle.reconstruct(v, q, metric, flags)
    f = oracle.VdbField(buf)
    ijk = _all_ijk(shape)
    got = oracle.lookup(f, ijk)
    want = R[ijk[:, 2], ijk[:, 1], ijk[:, 0]]
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # outside the volume: background
    B = st["background"]
    out = np.array([[-1, 0, 0], [0, -1, 0], [0, 0, -1], [shape[2], 0, 0],
                    [0, shape[1], 0], [0, 0, shape[0]], [10 ** 6, 3, 3]])
    assert np.all(oracle.lookup(f, out) == np.float32(B))


@pytest.mark.parametrize("shape,q,metric,flags", CASES)
def test_buffer_structure(shape, q, metric, flags):
    v = _rand_cloud(shape, 22)
    v[: shape[0] // 2, : shape[1] // 2, : shape[2] // 2] = np.float32(0.75)
    buf, st = oracle.encode(v, q, metric, flags)
    h = fmt.header(buf)
    assert h["magic"] == b"VDBC" and h["version"] == 1 and h["layout"] == 0
    assert (h["nx"], h["ny"], h["nz"]) == (shape[2], shape[1], shape[0])
    assert h["total_bytes"] == len(buf) == fmt.expected_size(h) == st["bytes"]
    for k in ("off_root", "off_upper", "off_lower", "off_upper_tiles", "off_lower_tiles",
              "off_leaf_masks", "off_leaf_values", "total_bytes"):
        assert h[k] % 256 == 0
    assert h["n_leaf"] == st["n_leaf"] and h["n_lower"] == st["n_lower"]
    # prefix fields are running popcounts; totals match the counts
    up = fmt.words(buf, h["off_upper"], h["n_upper"], 512)
    lo = fmt.words(buf, h["off_lower"], h["n_lower"], 64)
    for recs, nchild, ntile in ((up, h["n_lower"], h["n_upper_tiles"]),
                                (lo, h["n_leaf"], h["n_lower_tiles"])):
        if recs.size == 0:
            continue
        pc = fmt.popcount64(recs["child"]).ravel()
        pt = fmt.popcount64(recs["tile"]).ravel()
        assert np.array_equal(recs["cidx"].ravel(), np.concatenate([[0], np.cumsum(pc)[:-1]]))
        assert np.array_equal(recs["tidx"].ravel(), np.concatenate([[0], np.cumsum(pt)[:-1]]))
        assert pc.sum() == nchild and pt.sum() == ntile
        assert not np.any(recs["child"] & recs["tile"])
        assert not np.any(recs["pad"])
    # leaf value masks count the active voxels held in leaves
    masks = np.frombuffer(bytes(buf[h["off_leaf_masks"]:h["off_leaf_masks"] + 64 * h["n_leaf"]]),
                          "<u8")
    in_leaves = int(fmt.popcount64(masks).sum())
    in_tiles = 512 * h["n_lower_tiles"] + 512 * 4096 * h["n_upper_tiles"]
    assert in_leaves + in_tiles == st["active_voxels"] == h["active_voxels"]


def test_constant_grid():
    v = np.full((64, 64, 64), 0.3, np.float32)
    buf, st = oracle.encode(v, 1.0)
    assert st["background"] == np.float32(0.3)
    assert st["n_leaf"] == 0            # every leaf pruned to a tile
    f = oracle.VdbField(buf)
    ijk = _all_ijk(v.shape)[::97]
    assert np.all(oracle.lookup(f, ijk) == np.float32(0.3))


def test_dense_noise_overhead_within_ten_percent():
    # Table tab:worstcase: losslessly encoded dense noise stays within 10 %
    # of the dense size for large grids.
    for n in (128, 160):
        v = synth.dense_noise(n)
        buf, st = oracle.encode(v, 1.0)
        assert st["n_leaf"] == (-(-n // 8)) ** 3
        assert len(buf) <= 1.10 * v.nbytes


def test_achieved_rate_matches_target():
    # Section 3.2.1: output size grows one to one with the activated voxels
    v = synth.mid_volume(n=128)   # 64 bricks, ~45 non-background
    n = v.size
    for q in (0.05, 0.1, 0.25, 0.5):
        buf, st = oracle.encode(v, q)
        K = st["k_bricks"]
        assert K == min(64, int(np.floor(np.float64(np.float32(q)) * 64 + 0.5)))
        assert abs(st["achieved_rate"] - K / 64) <= 2.0 / n
        assert abs(st["achieved_rate"] - q) <= 0.5 / 64 + 2.0 / n
        # bytes ~ activated voxels * 4 B * (1 + leaf-mask overhead) + nodes;
        # uniform leaves pruned to tiles only make it smaller
        payload = st["active_voxels"] * 4
        assert st["n_leaf"] * 2112 <= len(buf) <= payload * 1.04 + 64 * 1024


def test_size_saturates():
    # Table tab:rates: once every non-background brick is active the size
    # stops growing (only constant tiles are added).
    v = synth.tiny_volume()
    lo, hi = oracle.brick_ranges(v)
    nonbg = int(np.sum((lo != 0) | (hi != 0)))
    sizes, leaves = [], []
    for q in (nonbg / 8, 1.0):
        buf, st = oracle.encode(v, q)
        sizes.append(len(buf))
        leaves.append(st["n_leaf"])
    assert leaves[0] == leaves[1]
    assert sizes[1] - sizes[0] <= 4 * 64 * 8 + 512
