"""Thin ctypes binding of libvdbc.so (include/vdbc.h).

Argument marshalling only: every step runs in the library (host encoder in
C++, everything else in HIP kernels).  PyTorch supplies device memory and the
current stream.  There is no fallback: if the library is missing, loading
fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvdbc.so")

OK, E_INVALID, E_NOMEM, E_BUFFER_TOO_SMALL, E_FORMAT, E_DEVICE, E_UNSUPPORTED = range(7)
BG_EXPLICIT, NO_CORNERS, NO_PRUNE = 1, 2, 4
MODE_EA, MODE_PT = 0, 1
RENDER_HDDA, RENDER_COUNT, RENDER_KEEP_MAJORANT = 1, 2, 4


class VdbcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vdbc status {status}: {msg}")
        self.status = status


class Dims(C.Structure):
    _fields_ = [("nx", C.c_uint32), ("ny", C.c_uint32), ("nz", C.c_uint32)]


class EncodeParams(C.Structure):
    _fields_ = [("rate", C.c_float), ("metric", C.c_uint32), ("flags", C.c_uint32),
                ("background", C.c_float), ("threads", C.c_uint32)]


class EncodeStats(C.Structure):
    _fields_ = [("background", C.c_float), ("n_bricks", C.c_uint64),
                ("k_bricks", C.c_uint64), ("n_leaf", C.c_uint64),
                ("n_lower", C.c_uint64), ("n_upper", C.c_uint64),
                ("n_lower_tiles", C.c_uint64), ("n_upper_tiles", C.c_uint64),
                ("active_voxels", C.c_uint64), ("bytes", C.c_uint64),
                ("achieved_rate", C.c_double)]


class GridC(C.Structure):
    _fields_ = [("device", C.c_void_p), ("bytes", C.c_uint64), ("header", C.c_uint8 * 256)]


class CameraC(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("width", C.c_uint32), ("height", C.c_uint32),
                ("origin", C.c_float * 3), ("lower_left", C.c_float * 3),
                ("du", C.c_float * 3), ("dv", C.c_float * 3), ("dir", C.c_float * 3)]


class MediumC(C.Structure):
    _fields_ = [("sigma_scale", C.c_float), ("albedo", C.c_float), ("tf_n", C.c_uint32),
                ("tf", (C.c_float * 4) * 64), ("tf_lo", C.c_float), ("tf_hi", C.c_float),
                ("light_dir", C.c_float * 3), ("light_E", C.c_float * 3),
                ("ambient", C.c_float * 3)]


class RenderParamsC(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("spp", C.c_uint32), ("max_bounces", C.c_uint32),
                ("macrocell", C.c_uint32), ("flags", C.c_uint32), ("step", C.c_float),
                ("t_terminate", C.c_float), ("seed", C.c_uint64), ("frame", C.c_uint32),
                ("reserved", C.c_uint32 * 3)]


SYMBOLS = [
    "vdbc_status_string", "vdbc_last_error", "vdbc_abi_version", "vdbc_encode_begin",
    "vdbc_encode_finish", "vdbc_encode_abort", "vdbc_encode", "vdbc_validate",
    "vdbc_grid_init", "vdbc_sample", "vdbc_sample_dense", "vdbc_lookup",
    "vdbc_render_workspace", "vdbc_render", "vdbc_render_dense", "vdbc_majorant",
    "vdbc_majorant_dense", "vdbc_philox",
]

_lib = None


def load():
    """Loads libvdbc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2504_04564_amd._build`")
    L = C.CDLL(LIB_PATH)
    P, u32, u64, f32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_float
    st = C.c_int
    L.vdbc_status_string.argtypes = [st]
    L.vdbc_status_string.restype = C.c_char_p
    L.vdbc_last_error.argtypes = []
    L.vdbc_last_error.restype = C.c_char_p
    L.vdbc_abi_version.restype = u32
    L.vdbc_encode_begin.argtypes = [P, Dims, C.POINTER(EncodeParams), C.POINTER(P),
                                    C.POINTER(u64), C.POINTER(EncodeStats)]
    L.vdbc_encode_finish.argtypes = [P, P, u64]
    L.vdbc_encode_abort.argtypes = [P]
    L.vdbc_encode_abort.restype = None
    L.vdbc_encode.argtypes = [P, Dims, C.POINTER(EncodeParams), P, u64, C.POINTER(u64),
                              C.POINTER(EncodeStats)]
    L.vdbc_validate.argtypes = [P, u64, C.POINTER(EncodeStats)]
    L.vdbc_grid_init.argtypes = [C.POINTER(GridC), P, u64, P]
    L.vdbc_sample.argtypes = [C.POINTER(GridC), P, u64, u32, P, P]
    L.vdbc_sample_dense.argtypes = [P, Dims, f32, P, u64, u32, P, P]
    L.vdbc_lookup.argtypes = [C.POINTER(GridC), P, u64, P, P]
    L.vdbc_render_workspace.argtypes = [C.POINTER(RenderParamsC), Dims, C.POINTER(u64)]
    L.vdbc_render.argtypes = [C.POINTER(GridC), C.POINTER(CameraC), C.POINTER(MediumC),
                              C.POINTER(RenderParamsC), P, P, P, u64, P]
    L.vdbc_render_dense.argtypes = [P, Dims, f32, C.POINTER(CameraC), C.POINTER(MediumC),
                                    C.POINTER(RenderParamsC), P, P, P, u64, P]
    L.vdbc_majorant.argtypes = [C.POINTER(GridC), C.POINTER(MediumC), u32, P, P]
    L.vdbc_majorant_dense.argtypes = [P, Dims, f32, C.POINTER(MediumC), u32, P, P]
    L.vdbc_philox.argtypes = [P, P, u64, P, P]
    for name in ["vdbc_encode_begin", "vdbc_encode_finish", "vdbc_encode", "vdbc_validate",
                 "vdbc_grid_init", "vdbc_sample", "vdbc_sample_dense", "vdbc_lookup",
                 "vdbc_render_workspace", "vdbc_render", "vdbc_render_dense", "vdbc_majorant",
                 "vdbc_majorant_dense", "vdbc_philox"]:
        getattr(L, name).restype = st
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        L = load()
        raise VdbcError(status, (L.vdbc_last_error() or b"").decode())


def _dims_of(shape) -> Dims:
    nz, ny, nx = shape
    return Dims(nx, ny, nz)


# ------------------------------------------------------------------ encoder

def encode(dense: np.ndarray, rate: float, metric: int = 2, flags: int = 0,
           background: float = 0.0, threads: int = 0):
    """Encode a host float32 volume (nz, ny, nx) -> (uint8 buffer, stats)."""
    L = load()
    d = np.ascontiguousarray(dense, dtype=np.float32)
    if d.ndim != 3:
        raise ValueError("dense must be 3-D (nz, ny, nx)")
    p = EncodeParams(rate, metric, flags, background, threads)
    h = C.c_void_p()
    nbytes = C.c_uint64(0)
    st = EncodeStats()
    _check(L.vdbc_encode_begin(d.ctypes.data, _dims_of(d.shape), C.byref(p), C.byref(h),
                               C.byref(nbytes), C.byref(st)))
    # 256-byte aligned host buffer
    raw = np.empty(nbytes.value + 256, dtype=np.uint8)
    off = (-raw.ctypes.data) % 256
    buf = raw[off:off + nbytes.value]
    _check(L.vdbc_encode_finish(h, buf.ctypes.data, nbytes.value))
    stats = {name: getattr(st, name) for name, _ in EncodeStats._fields_}
    return buf, stats


def validate(buf: np.ndarray) -> dict:
    L = load()
    b = np.ascontiguousarray(buf, dtype=np.uint8)
    st = EncodeStats()
    _check(L.vdbc_validate(b.ctypes.data, b.size, C.byref(st)))
    return {name: getattr(st, name) for name, _ in EncodeStats._fields_}


# ------------------------------------------------------------------ device

def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t) -> int:
    return t.data_ptr()


class Grid:
    """A canonical buffer resident in device memory (torch uint8 tensor)."""

    def __init__(self, buf: np.ndarray, device="cuda"):
        torch = _torch()
        host = np.ascontiguousarray(buf, dtype=np.uint8)
        self.tensor = torch.from_numpy(host).to(device)
        if self.tensor.data_ptr() % 256:
            raise RuntimeError("device buffer is not 256-byte aligned")
        self.nbytes = host.size
        self.header = host[:256].copy()
        self.c = GridC()
        _check(load().vdbc_grid_init(C.byref(self.c), _dptr(self.tensor), self.nbytes,
                                     self.header.ctypes.data))
        self.dims = tuple(int(x) for x in np.frombuffer(self.header[8:20].tobytes(), "<u4"))
        self.background = float(np.frombuffer(self.header[20:24].tobytes(), "<f4")[0])


def sample(grid: Grid, pos, filter: int = 1, out=None):
    torch = _torch()
    p = pos.contiguous()
    n = p.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=p.device)
    _check(load().vdbc_sample(C.byref(grid.c), _dptr(p), n, filter, _dptr(out), _stream()))
    return out


def sample_dense(dense_t, background: float, pos, filter: int = 1, out=None):
    torch = _torch()
    p = pos.contiguous()
    n = p.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=p.device)
    _check(load().vdbc_sample_dense(_dptr(dense_t), _dims_of(dense_t.shape), background,
                                    _dptr(p), n, filter, _dptr(out), _stream()))
    return out


def lookup(grid: Grid, ijk, out=None):
    torch = _torch()
    q = ijk.to(torch.int32).contiguous()
    n = q.numel() // 3
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=q.device)
    _check(load().vdbc_lookup(C.byref(grid.c), _dptr(q), n, _dptr(out), _stream()))
    return out


def camera_c(cam: dict) -> CameraC:
    c = CameraC()
    c.kind = cam["kind"]
    c.width, c.height = cam["width"], cam["height"]
    for name in ("origin", "lower_left", "du", "dv", "dir"):
        getattr(c, name)[:] = [float(x) for x in cam.get(name, (0.0, 0.0, 0.0))]
    return c


def medium_c(med: dict) -> MediumC:
    m = MediumC()
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
    return m


def params_c(p: dict, mode: int) -> RenderParamsC:
    r = RenderParamsC()
    r.mode = mode
    r.spp = p.get("spp", 1)
    r.max_bounces = p.get("max_bounces", 8)
    r.macrocell = p.get("macrocell", 8)
    r.flags = p.get("flags", 0)
    r.step = p.get("step", 0.5)
    r.t_terminate = p.get("t_terminate", 0.0)
    r.seed = p.get("seed", 0)
    r.frame = p.get("frame", 0)
    return r


class Renderer:
    """Holds the marshalled scene and workspace for repeated launches."""

    def __init__(self, field, camera: dict, medium: dict, params: dict, mode: int,
                 background: float | None = None, aov: bool = False, device="cuda"):
        torch = _torch()
        self.field = field
        self.dense = not isinstance(field, Grid)
        if self.dense:
            self.dims = _dims_of(field.shape)
            self.background = float(background if background is not None else 0.0)
        else:
            nx, ny, nz = field.dims
            self.dims = Dims(nx, ny, nz)
        self.cam, self.med = camera_c(camera), medium_c(medium)
        self.prm = params_c(params, mode)
        ws = C.c_uint64(0)
        _check(load().vdbc_render_workspace(C.byref(self.prm), self.dims, C.byref(ws)))
        self.ws = torch.zeros(max(int(ws.value), 256) + 256, dtype=torch.uint8, device=device)
        self.ws_off = (-self.ws.data_ptr()) % 256
        self.ws_bytes = int(ws.value)
        h, w = camera["height"], camera["width"]
        self.image = torch.empty((h, w, 4), dtype=torch.float32, device=device)
        self.aov = torch.empty((h, w, 2), dtype=torch.float32, device=device) if aov else None

    @property
    def ws_ptr(self) -> int:
        return self.ws.data_ptr() + self.ws_off

    def launch(self, stream=None):
        s = stream if stream is not None else _stream()
        L = load()
        aov = _dptr(self.aov) if self.aov is not None else None
        if self.dense:
            st = L.vdbc_render_dense(_dptr(self.field), self.dims, self.background,
                                     C.byref(self.cam), C.byref(self.med), C.byref(self.prm),
                                     _dptr(self.image), aov, self.ws_ptr, self.ws_bytes, s)
        else:
            st = L.vdbc_render(C.byref(self.field.c), C.byref(self.cam), C.byref(self.med),
                               C.byref(self.prm), _dptr(self.image), aov, self.ws_ptr,
                               self.ws_bytes, s)
        _check(st)
        return self.image

    def build_majorant(self, stream=None):
        """Majorant grid of this scene into the workspace (vdbc_majorant),
        for a following launch with RENDER_KEEP_MAJORANT."""
        s = stream if stream is not None else _stream()
        L = load()
        out = self.ws_ptr + 256
        if self.dense:
            st = L.vdbc_majorant_dense(_dptr(self.field), self.dims, self.background,
                                       C.byref(self.med), self.prm.macrocell, out, s)
        else:
            st = L.vdbc_majorant(C.byref(self.field.c), C.byref(self.med), self.prm.macrocell,
                                 out, s)
        _check(st)

    def sample_count(self) -> int:
        torch = _torch()
        return int(self.ws[self.ws_off:self.ws_off + 8].view(torch.int64).item())

    def cell_count(self) -> int:
        torch = _torch()
        return int(self.ws[self.ws_off + 8:self.ws_off + 16].view(torch.int64).item())

    def majorant(self):
        torch = _torch()
        C_ = self.prm.macrocell
        g = [(-(-n // C_)) for n in (self.dims.nz, self.dims.ny, self.dims.nx)]
        cnt = g[0] * g[1] * g[2]
        return self.ws[self.ws_off + 256:self.ws_off + 256 + 4 * cnt].view(torch.float32).reshape(g)


def render(field, camera: dict, medium: dict, params: dict, mode: int,
           background: float | None = None, aov: bool = False):
    r = Renderer(field, camera, medium, params, mode, background, aov)
    img = r.launch()
    return (img, r.aov) if aov else img


def majorant(field, medium: dict, macrocell: int = 8, background: float | None = None):
    torch = _torch()
    if isinstance(field, Grid):
        nx, ny, nz = field.dims
    else:
        nz, ny, nx = field.shape
    g = [(-(-n // macrocell)) for n in (nz, ny, nx)]
    out = torch.empty(g, dtype=torch.float32, device="cuda")
    m = medium_c(medium)
    L = load()
    if isinstance(field, Grid):
        _check(L.vdbc_majorant(C.byref(field.c), C.byref(m), macrocell, _dptr(out), _stream()))
    else:
        _check(L.vdbc_majorant_dense(_dptr(field), _dims_of(field.shape),
                                     float(background or 0.0), C.byref(m), macrocell,
                                     _dptr(out), _stream()))
    return out


def philox(ctr, key):
    torch = _torch()
    c = ctr.to(torch.int32).contiguous()
    k = key.to(torch.int32).contiguous()
    n = c.numel() // 4
    out = torch.empty_like(c)
    _check(load().vdbc_philox(_dptr(c), _dptr(k), n, _dptr(out), _stream()))
    return out
