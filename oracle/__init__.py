"""Python access to the CPU oracle (``liboracle.so``, plain C in this folder).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only users.  The product library never
imports this package.  The oracle is single-threaded, double precision, and
shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["philox.c", "encode.c", "field.c", "render.c"]

REF_BG_EXPLICIT = 1
REF_NO_CORNERS = 2
REF_NO_PRUNE = 4


_HASH_PATH = _LIB_PATH + ".hash"


def _source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for s in sorted(_SOURCES + ["oracle.h"]):
        with open(os.path.join(_HERE, s), "rb") as fh:
            h.update(s.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, IEEE arithmetic, no contraction);
    without `force`, only when it is missing or was built from other
    sources (the hash of the sources is kept beside the library)."""
    want = _source_hash()
    have = None
    if os.path.exists(_HASH_PATH):
        with open(_HASH_PATH) as fh:
            have = fh.read().strip()
    if force or not os.path.exists(_LIB_PATH) or have != want:
        srcs = [os.path.join(_HERE, s) for s in _SOURCES]
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
        with open(_HASH_PATH + ".tmp%d" % os.getpid(), "w") as fh:
            fh.write(want + "\n")
        os.replace(_HASH_PATH + ".tmp%d" % os.getpid(), _HASH_PATH)
    return _LIB_PATH


class Stats(C.Structure):
    _fields_ = [("background", C.c_float), ("n_bricks", C.c_uint64),
                ("k_bricks", C.c_uint64), ("n_leaf", C.c_uint64),
                ("n_lower", C.c_uint64), ("n_upper", C.c_uint64),
                ("n_lower_tiles", C.c_uint64), ("n_upper_tiles", C.c_uint64),
                ("active_voxels", C.c_uint64), ("bytes", C.c_uint64),
                ("achieved_rate", C.c_double)]


class Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("buf", C.c_void_p), ("bytes", C.c_uint64),
                ("dense", C.c_void_p), ("nx", C.c_uint32), ("ny", C.c_uint32),
                ("nz", C.c_uint32), ("background", C.c_float)]


class Camera(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("width", C.c_uint32), ("height", C.c_uint32),
                ("origin", C.c_float * 3), ("lower_left", C.c_float * 3),
                ("du", C.c_float * 3), ("dv", C.c_float * 3), ("dir", C.c_float * 3)]


class Medium(C.Structure):
    _fields_ = [("sigma_scale", C.c_float), ("albedo", C.c_float), ("tf_n", C.c_uint32),
                ("tf", (C.c_float * 4) * 64), ("tf_lo", C.c_float), ("tf_hi", C.c_float),
                ("light_dir", C.c_float * 3), ("light_E", C.c_float * 3),
                ("ambient", C.c_float * 3), ("env", C.c_void_p), ("env_w", C.c_uint32),
                ("env_h", C.c_uint32)]


class Params(C.Structure):
    _fields_ = [("spp", C.c_uint32), ("max_bounces", C.c_uint32),
                ("macrocell", C.c_uint32), ("step", C.c_float),
                ("t_terminate", C.c_float), ("seed", C.c_uint64), ("frame", C.c_uint32),
                ("rr", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.c_void_p
        u32, u64, f32 = C.c_uint32, C.c_uint64, C.c_float
        L.ref_philox4x32_10.argtypes = [P, P, P]
        L.ref_philox_many.argtypes = [P, P, u64, P]
        L.ref_philox_many.restype = None
        L.ref_u01.argtypes = [u32]
        L.ref_u01.restype = C.c_double
        L.ref_background.argtypes = [P, u64]
        L.ref_background.restype = f32
        L.ref_brick_ranges.argtypes = [P, u32, u32, u32, P, P]
        L.ref_similarity.argtypes = [u32, f32, f32, f32]
        L.ref_similarity.restype = C.c_double
        L.ref_brick_order.argtypes = [P, u32, u32, u32, f32, u32, f32, P, P]
        L.ref_reconstruct.argtypes = [P, u32, u32, u32, f32, u32, u32, f32, P]
        L.ref_encode.argtypes = [P, u32, u32, u32, f32, u32, u32, f32,
                                 C.POINTER(C.POINTER(C.c_uint8)), C.POINTER(u64),
                                 C.POINTER(Stats)]
        L.ref_reconstruct_partial.argtypes = [P, u32, u32, u32, f32, u32, u32, f32, f32, f32, P]
        L.ref_encode_partial.argtypes = [P, u32, u32, u32, f32, u32, u32, f32, f32, f32,
                                         C.POINTER(C.POINTER(C.c_uint8)), C.POINTER(u64),
                                         C.POINTER(Stats)]
        L.ref_active_mask.argtypes = [P, u32, u32, u32, f32, u32, u32, f32, f32, f32, P]
        L.ref_free.argtypes = [P]
        L.ref_field_vdb.argtypes = [C.POINTER(Field), P, u64]
        L.ref_field_dense.argtypes = [C.POINTER(Field), P, u32, u32, u32, f32]
        L.ref_field_dense.restype = None
        L.ref_lookup.argtypes = [C.POINTER(Field), C.c_int64, C.c_int64, C.c_int64]
        L.ref_lookup.restype = f32
        L.ref_lookup_many.argtypes = [C.POINTER(Field), P, u64, P]
        L.ref_lookup_many.restype = None
        L.ref_sample_many.argtypes = [C.POINTER(Field), P, u64, u32, P]
        L.ref_sample_many.restype = None
        L.ref_majorant.argtypes = [C.POINTER(Field), C.POINTER(Medium), u32, P]
        L.ref_majorant_cells.argtypes = [C.POINTER(Field), C.POINTER(Medium), u32, u64, u64, P]
        L.ref_render_pt_majorant.argtypes = [C.POINTER(Field), C.POINTER(Camera), C.POINTER(Medium),
                                             C.POINTER(Params), P, P, u64, P, P]
        L.ref_render_ea.argtypes = [C.POINTER(Field), C.POINTER(Camera), C.POINTER(Medium),
                                    C.POINTER(Params), P]
        L.ref_render_pt.argtypes = [C.POINTER(Field), C.POINTER(Camera), C.POINTER(Medium),
                                    C.POINTER(Params), P, u64, P, P]
        L.ref_transmittance.argtypes = [C.POINTER(Field), C.POINTER(Medium), u32, P, P,
                                        u64, u64]
        L.ref_transmittance.restype = C.c_double
        L.ref_render_iso.argtypes = [C.POINTER(Field), C.POINTER(Camera), C.c_double, C.c_double,
                                     u32, P, P]
        L.ref_isotropic.argtypes = [C.c_double, C.c_double, P]
        L.ref_isotropic.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


# ------------------------------ Philox ------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_many(ctr, key) -> np.ndarray:
    """Philox4x32-10 of n counters (n x 4) under n keys (n x 2)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    if len(c) != len(k):
        raise ValueError("one key per counter")
    out = np.zeros_like(c)
    lib().ref_philox_many(_ptr(c), _ptr(k), len(c), _ptr(out))
    return out


def u01(x: int) -> float:
    return lib().ref_u01(int(x))


# ------------------------------ encoder ------------------------------

def _dims(dense: np.ndarray):
    nz, ny, nx = dense.shape
    return nx, ny, nz


def background(dense: np.ndarray) -> float:
    d = np.ascontiguousarray(dense, dtype=np.float32)
    return float(lib().ref_background(_ptr(d), d.size))


def brick_ranges(dense: np.ndarray):
    d = np.ascontiguousarray(dense, dtype=np.float32)
    nx, ny, nz = _dims(d)
    nb = (-(-nx // 32)) * (-(-ny // 32)) * (-(-nz // 32))
    lo = np.zeros(nb, np.float32)
    hi = np.zeros(nb, np.float32)
    lib().ref_brick_ranges(_ptr(d), nx, ny, nz, _ptr(lo), _ptr(hi))
    return lo, hi


def similarity(metric: int, lo: float, hi: float, B: float) -> float:
    return lib().ref_similarity(metric, lo, hi, B)


def brick_order(dense: np.ndarray, rate: float, metric: int = 2, B: float | None = None):
    d = np.ascontiguousarray(dense, dtype=np.float32)
    nx, ny, nz = _dims(d)
    if B is None:
        B = background(d)
    nb = (-(-nx // 32)) * (-(-ny // 32)) * (-(-nz // 32))
    order = np.zeros(nb, np.uint32)
    k = C.c_uint64(0)
    _check(lib().ref_brick_order(_ptr(d), nx, ny, nz, rate, metric, B, _ptr(order),
                                 C.byref(k)), "ref_brick_order")
    return order, int(k.value)


PARTIAL = 8   # REF_PARTIAL


def reconstruct(dense: np.ndarray, rate: float, metric: int = 2, flags: int = 0,
                bg: float = 0.0, partial=None) -> np.ndarray:
    """Reconstructed grid; `partial` = (fraction, threshold) selects the
    partial-brick activation (sets REF_PARTIAL)."""
    d = np.ascontiguousarray(dense, dtype=np.float32)
    nx, ny, nz = _dims(d)
    R = np.empty_like(d)
    if partial is None:
        _check(lib().ref_reconstruct(_ptr(d), nx, ny, nz, rate, metric, flags, bg, _ptr(R)),
               "ref_reconstruct")
    else:
        _check(lib().ref_reconstruct_partial(_ptr(d), nx, ny, nz, rate, metric, flags | PARTIAL,
                                             bg, partial[0], partial[1], _ptr(R)),
               "ref_reconstruct_partial")
    return R


def active_mask(dense: np.ndarray, rate: float, metric: int = 2, flags: int = 0,
                bg: float = 0.0, partial=None) -> np.ndarray:
    """Boolean activation mask of the encoder's selection (shape of dense)."""
    d = np.ascontiguousarray(dense, dtype=np.float32)
    nx, ny, nz = _dims(d)
    m = np.zeros(d.shape, np.uint8)
    pf, pt = (1.0, 0.0) if partial is None else partial
    fl = flags | (PARTIAL if partial is not None else 0)
    _check(lib().ref_active_mask(_ptr(d), nx, ny, nz, rate, metric, fl, bg, pf, pt, _ptr(m)),
           "ref_active_mask")
    return m.astype(bool)


def encode(dense: np.ndarray, rate: float, metric: int = 2, flags: int = 0,
           bg: float = 0.0, partial=None):
    """Canonical buffer (numpy uint8) and encoder statistics (dict);
    `partial` = (fraction, threshold) as in reconstruct()."""
    d = np.ascontiguousarray(dense, dtype=np.float32)
    nx, ny, nz = _dims(d)
    out = C.POINTER(C.c_uint8)()
    nbytes = C.c_uint64(0)
    st = Stats()
    if partial is None:
        rc = lib().ref_encode(_ptr(d), nx, ny, nz, rate, metric, flags, bg, C.byref(out),
                              C.byref(nbytes), C.byref(st))
    else:
        rc = lib().ref_encode_partial(_ptr(d), nx, ny, nz, rate, metric, flags | PARTIAL, bg,
                                      partial[0], partial[1], C.byref(out), C.byref(nbytes),
                                      C.byref(st))
    _check(rc, "ref_encode")
    try:
        buf = np.ctypeslib.as_array(out, shape=(nbytes.value,)).copy()
    finally:
        lib().ref_free(out)
    stats = {name: getattr(st, name) for name, _ in Stats._fields_}
    return buf, stats


# ------------------------------ fields ------------------------------

class VdbField:
    """Oracle view of a canonical buffer (keeps the bytes alive)."""

    def __init__(self, buf: np.ndarray):
        self.buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self.f = Field()
        _check(lib().ref_field_vdb(C.byref(self.f), _ptr(self.buf), self.buf.size),
               "ref_field_vdb")


class DenseField:
    def __init__(self, dense: np.ndarray, background: float):
        self.dense = np.ascontiguousarray(dense, dtype=np.float32)
        nx, ny, nz = _dims(self.dense)
        self.f = Field()
        lib().ref_field_dense(C.byref(self.f), _ptr(self.dense), nx, ny, nz, background)


def lookup(fld, ijk: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(ijk, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(len(q), np.float32)
    lib().ref_lookup_many(C.byref(fld.f), _ptr(q), len(q), _ptr(out))
    return out


def sample(fld, pos: np.ndarray, filter: int = 1) -> np.ndarray:
    p = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    out = np.zeros(len(p), np.float64)
    lib().ref_sample_many(C.byref(fld.f), _ptr(p), len(p), filter, _ptr(out))
    return out


# ------------------------------ rendering ------------------------------

def make_camera(cam: dict) -> Camera:
    c = Camera()
    c.kind = cam["kind"]
    c.width, c.height = cam["width"], cam["height"]
    for name in ("origin", "lower_left", "du", "dv", "dir"):
        v = cam.get(name, (0.0, 0.0, 0.0))
        getattr(c, name)[:] = [float(x) for x in v]
    return c


def make_medium(med: dict) -> Medium:
    m = Medium()
    m.sigma_scale = med["sigma_scale"]
    m.albedo = med.get("albedo", 1.0)
    tf = np.asarray(med["tf"], dtype=np.float32).reshape(-1, 4)
    m.tf_n = len(tf)
    for i, row in enumerate(tf):
        m.tf[i][:] = [float(x) for x in row]
    m.tf_lo, m.tf_hi = med.get("tf_range", (0.0, 1.0))
    m.light_dir[:] = [float(x) for x in med.get("light_dir", (0.0, 0.0, 1.0))]
    m.light_E[:] = [float(x) for x in med.get("light_E", (0.0, 0.0, 0.0))]
    m.ambient[:] = [float(x) for x in med.get("ambient", (0.0, 0.0, 0.0))]
    env = med.get("env")
    if env is not None:
        # host float32 [h][w][3]; the array is kept alive on the struct
        e = np.ascontiguousarray(env, dtype=np.float32)
        if e.ndim != 3 or e.shape[2] != 3:
            raise ValueError("env must be [h][w][3]")
        m._env = e
        m.env = e.ctypes.data
        m.env_h, m.env_w = e.shape[0], e.shape[1]
    return m


def make_params(p: dict) -> Params:
    r = Params()
    r.spp = p.get("spp", 1)
    r.max_bounces = p.get("max_bounces", 8)
    r.macrocell = p.get("macrocell", 8)
    r.step = p.get("step", 0.5)
    r.t_terminate = p.get("t_terminate", 0.0)
    r.seed = p.get("seed", 0)
    r.frame = p.get("frame", 0)
    r.rr = 1 if p.get("rr", False) else 0
    return r


def majorant(fld, medium: dict, C_: int = 8, cells=None, out=None) -> np.ndarray:
    """Majorant grid (nz/C, ny/C, nx/C); with cells=(begin, end) only the
    cells of that flat-index range are computed (into `out` if given)."""
    f = fld.f
    g = [(-(-n // C_)) for n in (f.nz, f.ny, f.nx)]
    if out is None:
        out = np.zeros(g, np.float64)
    assert out.shape == tuple(g) and out.dtype == np.float64 and out.flags.c_contiguous
    m = make_medium(medium)
    if cells is None:
        _check(lib().ref_majorant(C.byref(f), C.byref(m), C_, _ptr(out)), "ref_majorant")
    else:
        _check(lib().ref_majorant_cells(C.byref(f), C.byref(m), C_, int(cells[0]), int(cells[1]),
                                        _ptr(out)), "ref_majorant_cells")
    return out


def majorant_threads(fld, medium: dict, C_: int, threads: int) -> np.ndarray:
    """The same majorant grid computed by `threads` concurrent calls of the
    single-threaded oracle on disjoint cell ranges (ctypes releases the GIL
    during each call)."""
    from concurrent.futures import ThreadPoolExecutor
    f = fld.f
    g = [(-(-n // C_)) for n in (f.nz, f.ny, f.nx)]
    out = np.zeros(g, np.float64)
    n = out.size
    cuts = np.linspace(0, n, 8 * threads + 1).astype(np.int64)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda i: majorant(fld, medium, C_, (cuts[i], cuts[i + 1]), out), range(len(cuts) - 1)))
    return out


def render_ea(fld, camera: dict, medium: dict, params: dict) -> np.ndarray:
    c, m, r = make_camera(camera), make_medium(medium), make_params(params)
    img = np.zeros((c.height, c.width, 4), np.float64)
    _check(lib().ref_render_ea(C.byref(fld.f), C.byref(c), C.byref(m), C.byref(r), _ptr(img)),
           "ref_render_ea")
    return img


def render_iso(fld, camera: dict, iso: float, step: float, refine: int = 12, aux=False):
    """Iso-surface normals: RGBA [h][w][4]; with aux=True also [h][w][3] =
    (hit ray parameter or -1, lattice margin, bisection margin)."""
    c = make_camera(camera)
    img = np.zeros((c.height, c.width, 4), np.float64)
    ax = np.zeros((c.height, c.width, 3), np.float64) if aux else None
    _check(lib().ref_render_iso(C.byref(fld.f), C.byref(c), float(iso), float(step), int(refine),
                                _ptr(img), _ptr(ax) if aux else None), "ref_render_iso")
    return (img, ax) if aux else img


def render_pt(fld, camera: dict, medium: dict, params: dict, pixels=None, aov=False, majorant=None):
    """Path-traced RGBA for `pixels` (flat indices py*W+px; default all);
    `majorant`: a grid from majorant() at params' macrocell, used instead of
    building one."""
    c, m, r = make_camera(camera), make_medium(medium), make_params(params)
    if pixels is None:
        pixels = np.arange(c.width * c.height, dtype=np.uint32)
    pix = np.ascontiguousarray(pixels, dtype=np.uint32)
    rgba = np.zeros((len(pix), 4), np.float64)
    a = np.zeros((len(pix), 2), np.float64) if aov else None
    if majorant is None:
        _check(lib().ref_render_pt(C.byref(fld.f), C.byref(c), C.byref(m), C.byref(r), _ptr(pix),
                                   len(pix), _ptr(rgba), _ptr(a) if aov else None),
               "ref_render_pt")
    else:
        f = fld.f
        g = tuple(-(-n // r.macrocell) for n in (f.nz, f.ny, f.nx))
        mj = np.ascontiguousarray(majorant, dtype=np.float64)
        if mj.shape != g:
            raise ValueError(f"majorant grid {mj.shape} does not match macrocell {r.macrocell}: {g}")
        _check(lib().ref_render_pt_majorant(C.byref(fld.f), C.byref(c), C.byref(m), C.byref(r),
                                            _ptr(mj), _ptr(pix), len(pix), _ptr(rgba),
                                            _ptr(a) if aov else None), "ref_render_pt_majorant")
    return (rgba, a) if aov else rgba


def isotropic(u1: float, u2: float) -> np.ndarray:
    d = np.zeros(3, np.float64)
    lib().ref_isotropic(float(u1), float(u2), _ptr(d))
    return d


def transmittance(fld, medium: dict, o, d, trials: int, seed: int = 1, C_: int = 8) -> float:
    m = make_medium(medium)
    oo = np.asarray(o, np.float32)
    dd = np.asarray(d, np.float32)
    return float(lib().ref_transmittance(C.byref(fld.f), C.byref(m), C_, _ptr(oo), _ptr(dd),
                                         trials, seed))
