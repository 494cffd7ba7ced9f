"""Test-side reader of the canonical buffer (format v1, every node layout),
used to check the structural invariants of buffers written by either encoder
and to decode voxels of the layout variants independently of both."""
import struct

import numpy as np

HEADER_FIELDS = [
    ("magic", 0, "4s"), ("version", 4, "I"), ("nx", 8, "I"), ("ny", 12, "I"),
    ("nz", 16, "I"), ("background", 20, "f"), ("rate", 24, "f"), ("metric", 28, "I"),
    ("flags", 32, "I"), ("layout", 36, "I"), ("n_bricks", 40, "Q"),
    ("k_bricks", 48, "Q"), ("active_voxels", 56, "Q"), ("n_upper", 64, "I"),
    ("n_lower", 68, "I"), ("n_leaf", 72, "I"), ("n_upper_tiles", 76, "I"),
    ("n_lower_tiles", 80, "I"), ("root_nx", 84, "I"), ("root_ny", 88, "I"),
    ("root_nz", 92, "I"), ("off_root", 96, "Q"), ("off_upper", 104, "Q"),
    ("off_lower", 112, "Q"), ("off_upper_tiles", 120, "Q"),
    ("off_lower_tiles", 128, "Q"), ("off_leaf_masks", 136, "Q"),
    ("off_leaf_values", 144, "Q"), ("total_bytes", 152, "Q"),
]


def header(buf: np.ndarray) -> dict:
    b = bytes(buf[:256])
    return {name: struct.unpack_from("<" + fmt, b, off)[0] for name, off, fmt in HEADER_FIELDS}


def words(buf: np.ndarray, off: int, count: int, per_node: int):
    """Word records of `count` nodes: dict of arrays child, cidx, tidx, tile,
    each shaped (count, per_node)."""
    rec = np.dtype([("child", "<u8"), ("cidx", "<u4"), ("tidx", "<u4"), ("tile", "<u8"),
                    ("pad", "<u8")])
    n = count * per_node
    a = np.frombuffer(bytes(buf[off:off + 32 * n]), dtype=rec).reshape(count, per_node)
    return a


def popcount64(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    c = np.zeros(x.shape, np.int64)
    for s in range(0, 64, 8):
        byte = ((x >> np.uint64(s)) & np.uint64(0xFF)).astype(np.int64)
        c += np.array([bin(i).count("1") for i in range(256)])[byte]
    return c


def expected_size(h: dict) -> int:
    def a(x):
        return (x + 255) // 256 * 256
    rn = h["root_nx"] * h["root_ny"] * h["root_nz"]
    off = 256
    off = a(off + 4 * rn)
    wb = 24 if h["layout"] & 2 else 32
    off = a(off + h["n_upper"] * 512 * wb)
    off = a(off + h["n_lower"] * 64 * wb)
    off = a(off + 4 * h["n_upper_tiles"])
    off = a(off + 4 * h["n_lower_tiles"])
    off = a(off + 64 * h["n_leaf"])
    off = a(off + 2048 * h["n_leaf"])
    return off


def node_words(buf: np.ndarray, off: int, count: int, per_node: int, layout: int) -> dict:
    """child / tile masks and child / tile index prefixes of `count` nodes of
    `per_node` words, each shaped (count, per_node): 32-byte records, or with
    layout bit 2 the four arrays u64 child | u64 tile | u32 cidx | u32 tidx."""
    if not layout & 2:
        a = words(buf, off, count, per_node)
        return {"child": a["child"], "tile": a["tile"], "cidx": a["cidx"], "tidx": a["tidx"]}
    W = per_node
    raw = np.frombuffer(bytes(buf[off:off + 24 * W * count]), np.uint8).reshape(count, 24 * W)
    return {"child": raw[:, :8 * W].copy().view("<u8"), "tile": raw[:, 8 * W:16 * W].copy().view("<u8"),
            "cidx": raw[:, 16 * W:20 * W].copy().view("<u4"), "tidx": raw[:, 20 * W:].copy().view("<u4")}


def slot(layout: int, log2: int, x, y, z):
    """Child-slot number: x-fastest, or with layout bit 1 a Morton number whose
    bit 3b+a is bit b of coordinate a (x = 0, y = 1, z = 2)."""
    x, y, z = (np.asarray(c, np.int64) for c in (x, y, z))
    if not layout & 1:
        return x + ((y + (z << log2)) << log2)
    n = np.zeros_like(x)
    for b in range(log2):
        n |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return n


def read_voxels(buf: np.ndarray, ijk: np.ndarray) -> np.ndarray:
    """Values of integer voxels (rows i, j, k) by a vectorised descent of the
    buffer in any node layout; outside the volume or the tree: background."""
    h = header(buf)
    L = h["layout"]
    q = np.asarray(ijk, np.int64).reshape(-1, 3)
    i, j, k = q[:, 0], q[:, 1], q[:, 2]
    f32 = lambda off, n: np.frombuffer(bytes(buf[off:off + 4 * n]), "<f4")
    out = np.full(len(q), h["background"], np.float32)
    ok = (i >= 0) & (j >= 0) & (k >= 0) & (i < h["nx"]) & (j < h["ny"]) & (k < h["nz"])
    rn = h["root_nx"] * h["root_ny"] * h["root_nz"]
    root = np.frombuffer(bytes(buf[h["off_root"]:h["off_root"] + 4 * rn]), "<u4")
    r = (i >> 12) + h["root_nx"] * ((j >> 12) + h["root_ny"] * (k >> 12))
    u = np.where(ok, root[np.where(ok, r, 0)], 0xFFFFFFFF).astype(np.int64)
    ok &= u != 0xFFFFFFFF
    one = np.uint64(1)

    def step(nodes, node_idx, n, tiles, ok):
        w, b = n >> 6, (n & 63).astype(np.uint64)
        below = (one << b) - one
        cm = nodes["child"][node_idx, w]
        tm = nodes["tile"][node_idx, w]
        is_child = ok & (((cm >> b) & one) == one)
        is_tile = ok & ~is_child & (((tm >> b) & one) == one)
        child = nodes["cidx"][node_idx, w].astype(np.int64) + popcount64(cm & below)
        tix = nodes["tidx"][node_idx, w].astype(np.int64) + popcount64(tm & below)
        out[is_tile] = tiles[tix[is_tile]]
        return is_child, child

    U = node_words(buf, h["off_upper"], h["n_upper"], 512, L)
    n1 = slot(L, 5, (i >> 7) & 31, (j >> 7) & 31, (k >> 7) & 31)
    ok, lower = step(U, np.where(ok, u, 0), n1, f32(h["off_upper_tiles"], h["n_upper_tiles"]), ok)
    Lw = node_words(buf, h["off_lower"], h["n_lower"], 64, L)
    n2 = slot(L, 4, (i >> 3) & 15, (j >> 3) & 15, (k >> 3) & 15)
    ok, leaf = step(Lw, np.where(ok, lower, 0), n2, f32(h["off_lower_tiles"], h["n_lower_tiles"]), ok)
    vals = f32(h["off_leaf_values"], 512 * h["n_leaf"])
    n3 = (i & 7) + 8 * (j & 7) + 64 * (k & 7)
    out[ok] = vals[leaf[ok] * 512 + n3[ok]]
    return out


def all_voxels(shape) -> np.ndarray:
    """(i, j, k) rows of every voxel of a (nz, ny, nx) volume, x fastest."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
