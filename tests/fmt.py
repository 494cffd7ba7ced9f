"""Test-side reader of the canonical buffer (format v1), used to check the
structural invariants of buffers written by either encoder."""
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
    off = a(off + h["n_upper"] * 512 * 32)
    off = a(off + h["n_lower"] * 64 * 32)
    off = a(off + 4 * h["n_upper_tiles"])
    off = a(off + 4 * h["n_lower_tiles"])
    off = a(off + 64 * h["n_leaf"])
    off = a(off + 2048 * h["n_leaf"])
    return off
