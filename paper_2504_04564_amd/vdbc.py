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
ABI_VERSION = 2        # VDBC_ABI_VERSION of include/vdbc.h

OK, E_INVALID, E_NOMEM, E_BUFFER_TOO_SMALL, E_FORMAT, E_DEVICE, E_UNSUPPORTED = range(7)
BG_EXPLICIT, NO_CORNERS, NO_PRUNE, PARTIAL = 1, 2, 4, 8
MODE_EA, MODE_PT, MODE_ISO = 0, 1, 2
RENDER_HDDA, RENDER_COUNT, RENDER_KEEP_MAJORANT, RENDER_RR = 1, 2, 4, 8
RENDER_CACHE_NONE, RENDER_CACHE_LEAF, RENDER_COST_ORDER = 16, 32, 64
# accessor cache policy -> render flag (2 = last leaf and last lower node, the default)
CACHE_FLAGS = {0: RENDER_CACHE_NONE, 1: RENDER_CACHE_LEAF, 2: 0}
# node layouts (bits): Morton child-slot order, SoA node words
LAYOUT_V1, LAYOUT_MORTON, LAYOUT_SOA = 0, 1, 2
LAYOUTS = (0, 1, 2, 3)


class VdbcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vdbc status {status}: {msg}")
        self.status = status


class Dims(C.Structure):
    _fields_ = [("nx", C.c_uint32), ("ny", C.c_uint32), ("nz", C.c_uint32)]


class EncodeParams(C.Structure):
    _fields_ = [("rate", C.c_float), ("metric", C.c_uint32), ("flags", C.c_uint32),
                ("background", C.c_float), ("threads", C.c_uint32),
                ("partial_fraction", C.c_float), ("partial_threshold", C.c_float)]


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
                ("ambient", C.c_float * 3), ("env", C.c_void_p), ("env_w", C.c_uint32),
                ("env_h", C.c_uint32)]


class RenderParamsC(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("spp", C.c_uint32), ("max_bounces", C.c_uint32),
                ("macrocell", C.c_uint32), ("flags", C.c_uint32), ("step", C.c_float),
                ("t_terminate", C.c_float), ("seed", C.c_uint64), ("frame", C.c_uint32),
                ("tile_w", C.c_uint32), ("iso", C.c_float), ("refine", C.c_uint32),
                ("chunk_spp", C.c_uint32)]


SYMBOLS = [
    "vdbc_status_string", "vdbc_last_error", "vdbc_abi_version", "vdbc_encode_begin",
    "vdbc_encode_finish", "vdbc_encode_abort", "vdbc_encode", "vdbc_validate",
    "vdbc_grid_init", "vdbc_sample", "vdbc_sample_dense", "vdbc_lookup",
    "vdbc_render_workspace", "vdbc_render", "vdbc_render_dense", "vdbc_majorant",
    "vdbc_majorant_dense", "vdbc_philox",
]

_lib = None


def _torch_hip_first():
    """Imports torch before libvdbc.so is loaded.  The torch wheel carries its
    own HIP runtime under the same soname (libamdhip64.so.7) as the ROCm one
    the library is linked against: loaded after torch, the library binds to
    torch's runtime; loaded first, the process ends up with two HIP runtimes,
    and torch's memory and streams are unknown to the library's kernels (the
    first launch fails with "no ROCm-capable device")."""
    import torch  # noqa: F401


def load():
    """Loads libvdbc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2504_04564_amd._build`")
    _torch_hip_first()
    L = C.CDLL(LIB_PATH)
    P, u32, u64, f32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_float
    st = C.c_int
    L.vdbc_status_string.argtypes = [st]
    L.vdbc_status_string.restype = C.c_char_p
    L.vdbc_last_error.argtypes = []
    L.vdbc_last_error.restype = C.c_char_p
    L.vdbc_abi_version.restype = u32
    if L.vdbc_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {L.vdbc_abi_version()}, the binding "
                          f"expects {ABI_VERSION}: rebuild it")
    L.vdbc_encode_begin.argtypes = [P, Dims, C.POINTER(EncodeParams), C.POINTER(P),
                                    C.POINTER(u64), C.POINTER(EncodeStats)]
    L.vdbc_encode_finish.argtypes = [P, P, u64]
    L.vdbc_encode_abort.argtypes = [P]
    L.vdbc_encode_abort.restype = None
    L.vdbc_encode.argtypes = [P, Dims, C.POINTER(EncodeParams), P, u64, C.POINTER(u64),
                              C.POINTER(EncodeStats)]
    L.vdbc_validate.argtypes = [P, u64, C.POINTER(EncodeStats)]
    L.vdbc_relayout.argtypes = [P, u64, u32, P, u64, C.POINTER(u64)]
    L.vdbc_grid_init.argtypes = [C.POINTER(GridC), P, u64, P]
    L.vdbc_sample.argtypes = [C.POINTER(GridC), P, u64, u32, P, P]
    L.vdbc_sample_dense.argtypes = [P, Dims, f32, P, u64, u32, P, P]
    L.vdbc_lookup.argtypes = [C.POINTER(GridC), P, u64, P, P]
    L.vdbc_compare_workspace.argtypes = [Dims, C.POINTER(u64)]
    L.vdbc_compare_dense.argtypes = [C.POINTER(GridC), P, P, P, u64, P]
    L.vdbc_render_workspace.argtypes = [C.POINTER(RenderParamsC), Dims, C.POINTER(CameraC), C.POINTER(u64)]
    L.vdbc_render.argtypes = [C.POINTER(GridC), C.POINTER(CameraC), C.POINTER(MediumC),
                              C.POINTER(RenderParamsC), P, P, P, u64, P]
    L.vdbc_render_dense.argtypes = [P, Dims, f32, C.POINTER(CameraC), C.POINTER(MediumC),
                                    C.POINTER(RenderParamsC), P, P, P, u64, P]
    L.vdbc_render_noalloc.argtypes = [C.POINTER(GridC), C.POINTER(CameraC), C.POINTER(MediumC),
                                      C.POINTER(RenderParamsC), P, P, P]
    L.vdbc_majorant.argtypes = [C.POINTER(GridC), C.POINTER(MediumC), u32, P, P]
    L.vdbc_majorant_dense.argtypes = [P, Dims, f32, C.POINTER(MediumC), u32, P, P]
    L.vdbc_philox.argtypes = [P, P, u64, P, P]
    for name in ["vdbc_encode_begin", "vdbc_encode_finish", "vdbc_encode", "vdbc_validate", "vdbc_relayout",
                 "vdbc_grid_init", "vdbc_sample", "vdbc_sample_dense", "vdbc_lookup",
                 "vdbc_render_workspace", "vdbc_render", "vdbc_render_dense", "vdbc_render_noalloc",
                 "vdbc_majorant", "vdbc_majorant_dense", "vdbc_philox"]:
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

def _aligned(nbytes: int) -> np.ndarray:
    """Host uint8 array of nbytes starting on a 256-byte boundary."""
    raw = np.empty(nbytes + 256, dtype=np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw[off:off + nbytes]


def encode(dense: np.ndarray, rate: float, metric: int = 2, flags: int = 0,
           background: float = 0.0, threads: int = 0, layout: int = LAYOUT_V1,
           partial=None):
    """Encode a host float32 volume (nz, ny, nx) -> (uint8 buffer, stats);
    a non-zero node layout is produced from the layout-0 buffer by relayout().
    `partial` = (fraction, threshold) selects partial-brick activation
    (sets PARTIAL)."""
    L = load()
    d = np.ascontiguousarray(dense, dtype=np.float32)
    if d.ndim != 3:
        raise ValueError("dense must be 3-D (nz, ny, nx)")
    pf, pt = (0.0, 0.0) if partial is None else partial
    if partial is not None:
        flags |= PARTIAL
    p = EncodeParams(rate, metric, flags, background, threads, pf, pt)
    h = C.c_void_p()
    nbytes = C.c_uint64(0)
    st = EncodeStats()
    _check(L.vdbc_encode_begin(d.ctypes.data, _dims_of(d.shape), C.byref(p), C.byref(h),
                               C.byref(nbytes), C.byref(st)))
    buf = _aligned(nbytes.value)
    _check(L.vdbc_encode_finish(h, buf.ctypes.data, nbytes.value))
    stats = {name: getattr(st, name) for name, _ in EncodeStats._fields_}
    if layout != LAYOUT_V1:
        buf = relayout(buf, layout)
        stats["bytes"] = buf.size
    return buf, stats


def relayout(buf: np.ndarray, layout: int) -> np.ndarray:
    """The same tree in node layout `layout` (0..3) as a new host buffer."""
    L = load()
    b = np.ascontiguousarray(buf, dtype=np.uint8)
    need = C.c_uint64(0)
    st = L.vdbc_relayout(b.ctypes.data, b.size, layout, None, 0, C.byref(need))
    if st != E_BUFFER_TOO_SMALL:
        _check(st)
    out = _aligned(need.value)
    _check(L.vdbc_relayout(b.ctypes.data, b.size, layout, out.ctypes.data, out.size, C.byref(need)))
    return out


def layout_of(buf: np.ndarray) -> int:
    return int(np.frombuffer(np.ascontiguousarray(buf[36:40]).tobytes(), "<u4")[0])


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
        self.layout = layout_of(self.header)


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


def compare_dense(grid: Grid, dense) -> dict:
    """vdbc_compare_dense: error statistics of `grid` against the dense
    float32 device volume [nz][ny][nx] (MSE, max error, differing voxels,
    value range and PSNR over that range)."""
    torch = _torch()
    d = dense.contiguous()
    dims = _dims_of(tuple(d.shape))
    need = C.c_uint64(0)
    _check(load().vdbc_compare_workspace(dims, C.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=d.device)
    out = torch.empty(5, dtype=torch.float64, device=d.device)
    _check(load().vdbc_compare_dense(C.byref(grid.c), _dptr(d), _dptr(out), _dptr(ws), need.value,
                                     _stream()))
    sse, mx, nd, lo, hi = out.cpu().tolist()
    n = d.numel()
    mse = sse / n
    rng = hi - lo
    psnr = float("inf") if mse == 0 else (10.0 * np.log10(rng * rng / mse) if rng > 0 else float("-inf"))
    return dict(sse=sse, mse=mse, max_abs=mx, differing=int(nd), min=lo, max=hi, psnr=psnr)


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
    env = med.get("env")
    if env is not None:
        # device float32 tensor [h][w][3]; kept alive on the struct
        if env.dim() != 3 or env.shape[2] != 3 or not env.is_cuda:
            raise ValueError("env must be a device tensor [h][w][3]")
        e = env.to(_torch().float32).contiguous()
        m._env = e
        m.env = e.data_ptr()
        m.env_h, m.env_w = e.shape[0], e.shape[1]
    return m


def params_c(p: dict, mode: int) -> RenderParamsC:
    """vdbc_render_params from a dict: spp (1), max_bounces (8), macrocell
    (8), flags (0; RENDER_*), step (0.5), t_terminate (0), seed (0), frame
    (0), tile_w (8: pixels per wave row), iso (0.5), refine (12), chunk_spp
    (0: one work item per tile; else samples per work item)."""
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
    r.tile_w = p.get("tile_w", 8)
    r.iso = p.get("iso", 0.5)
    r.refine = p.get("refine", 12)
    r.chunk_spp = p.get("chunk_spp", 0)
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
        # the iso-surface mode reads no medium
        self.cam, self.med = camera_c(camera), (medium_c(medium) if medium else MediumC())
        self.prm = params_c(params, mode)
        ws = C.c_uint64(0)
        _check(load().vdbc_render_workspace(C.byref(self.prm), self.dims, C.byref(self.cam), C.byref(ws)))
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

    def segment_count(self) -> int:
        """Path segments (camera, shadow and scattered rays) of the last
        path-traced launch with RENDER_COUNT."""
        torch = _torch()
        return int(self.ws[self.ws_off + 24:self.ws_off + 32].view(torch.int64).item())

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


NOALLOC_SCRATCH_BYTES = 16 << 20


def render_noalloc(grid: Grid, camera: dict, medium: dict, params: dict, mode: int,
                   image=None, aov=None, stream=None):
    """vdbc_render_noalloc: the render of a VDB into caller-owned outputs
    (allocated here only when not given) with the library's fixed scratch
    instead of a workspace."""
    torch = _torch()
    h, w = camera["height"], camera["width"]
    if image is None:
        image = torch.empty((h, w, 4), dtype=torch.float32, device="cuda")
    cam, med, prm = camera_c(camera), (medium_c(medium) if medium else MediumC()), params_c(params, mode)
    s = stream if stream is not None else _stream()
    _check(load().vdbc_render_noalloc(C.byref(grid.c), C.byref(cam), C.byref(med), C.byref(prm),
                                      _dptr(image), _dptr(aov) if aov is not None else None, s))
    return image


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


# ------------------------------------------------------------------ denoiser

def _nn_signatures(L):
    P, u32, u64, f32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_float
    L.vdbc_nn_param_count.argtypes = [C.POINTER(u64)]
    L.vdbc_nn_to_bf16.argtypes = [P, P, P]
    L.vdbc_denoise_workspace.argtypes = [u32, u32, u32, u32, C.POINTER(u64)]
    L.vdbc_denoise_pack.argtypes = [P, P, u64, P, P]
    L.vdbc_denoise.argtypes = [P, P, P, u32, u32, u32, P, P, u64, P]
    L.vdbc_denoise_train_step.argtypes = [P, P, P, P, u32, f32, P, P, u32, u32, u32, P, P, P,
                                          u64, P]
    L.vdbc_conv3x3.argtypes = [P, u32, P, u32, u32, u32, u32, u32, u32, P, P, u32, u32, P, P, P]
    L.vdbc_conv3x3_grad_workspace.argtypes = [u32, u32, u32, u32, u32, C.POINTER(u64)]
    L.vdbc_conv3x3_dgrad.argtypes = [P, u32, u32, u32, u32, u32, P, u32, u32, u32, u32, P, P,
                                     u64, P]
    L.vdbc_conv3x3_wgrad.argtypes = [P, u32, P, u32, u32, u32, u32, u32, u32, P, u32, u32, P, P,
                                     P, u64, P]
    for name in ["vdbc_nn_param_count", "vdbc_nn_to_bf16", "vdbc_denoise_workspace",
                 "vdbc_denoise_pack", "vdbc_denoise", "vdbc_denoise_train_step", "vdbc_conv3x3",
                 "vdbc_conv3x3_grad_workspace", "vdbc_conv3x3_dgrad", "vdbc_conv3x3_wgrad"]:
        getattr(L, name).restype = C.c_int


def _nn():
    L = load()
    if not getattr(L, "_nn_ready", False):
        _nn_signatures(L)
        L._nn_ready = True
    return L


def nn_param_count() -> int:
    n = C.c_uint64(0)
    _check(_nn().vdbc_nn_param_count(C.byref(n)))
    return int(n.value)


def _aligned_empty(nbytes: int, device="cuda"):
    torch = _torch()
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


def conv3x3(a, b, upsample, stride, w_bf16, bias, cout, relu, out_f32=False):
    """One 3x3 conv layer on NHWC BF16 tensors (a: (n, hs, ws, ca), b: None or
    (n, hs, ws, cb)); returns NHWC BF16 (or FP32) output."""
    torch = _torch()
    n, hs, ws_, ca = a.shape
    cb = 0 if b is None else b.shape[-1]
    hv, wv = (2 * hs, 2 * ws_) if upsample else (hs, ws_)
    ho, wo = (hv - 1) // stride + 1, (wv - 1) // stride + 1
    out = torch.empty((n, ho, wo, cout), dtype=torch.float32 if out_f32 else torch.bfloat16,
                      device=a.device)
    _check(_nn().vdbc_conv3x3(_dptr(a), ca, _dptr(b) if b is not None else None, cb,
                              int(bool(upsample)), n, hs, ws_, stride, _dptr(w_bf16), _dptr(bias),
                              cout, int(bool(relu)), None if out_f32 else _dptr(out),
                              _dptr(out) if out_f32 else None, _stream()))
    return out


def conv3x3_dgrad(dz, cout, w_bf16, cin, stride, hv, wv):
    torch = _torch()
    n, ho, wo, coutp = dz.shape
    ws = C.c_uint64(0)
    _check(_nn().vdbc_conv3x3_grad_workspace(cin, cout, n, ho, wo, C.byref(ws)))
    buf, ptr = _aligned_empty(int(ws.value), dz.device)
    dx = torch.empty((n, hv, wv, cin), dtype=torch.float32, device=dz.device)
    _check(_nn().vdbc_conv3x3_dgrad(_dptr(dz), coutp, cout, n, ho, wo, _dptr(w_bf16), cin, stride,
                                    hv, wv, _dptr(dx), ptr, int(ws.value), _stream()))
    torch.cuda.synchronize()
    del buf
    return dx


def conv3x3_wgrad(a, b, upsample, stride, dz, cout):
    torch = _torch()
    n, hs, ws_, ca = a.shape
    cb = 0 if b is None else b.shape[-1]
    _, ho, wo, coutp = dz.shape
    ws = C.c_uint64(0)
    _check(_nn().vdbc_conv3x3_grad_workspace(ca + cb, cout, n, ho, wo, C.byref(ws)))
    buf, ptr = _aligned_empty(int(ws.value), a.device)
    dw = torch.empty((cout, 3, 3, ca + cb), dtype=torch.float32, device=a.device)
    db = torch.empty(cout, dtype=torch.float32, device=a.device)
    _check(_nn().vdbc_conv3x3_wgrad(_dptr(a), ca, _dptr(b) if b is not None else None, cb,
                                    int(bool(upsample)), n, hs, ws_, stride, _dptr(dz), coutp,
                                    cout, _dptr(dw), _dptr(db), ptr, int(ws.value), _stream()))
    torch.cuda.synchronize()
    del buf
    return dw, db


def init_denoiser_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the three zero
    input channels of the first layer get zero weights; last layer x0.1."""
    layers = [(8, 32), (32, 64), (64, 64), (64, 32), (64, 32), (32, 3)]
    rng = np.random.default_rng(seed)
    out = []
    for i, (cin, cout) in enumerate(layers):
        fan = 9 * (5 if i == 0 else cin)
        w = rng.normal(0.0, np.sqrt(2.0 / fan), size=(cout, 3, 3, cin)).astype(np.float32)
        if i == 0:
            w[..., 5:] = 0.0
        if i == len(layers) - 1:
            w *= 0.1
        out += [w.ravel(), np.zeros(cout, np.float32)]
    return np.concatenate(out)


class Denoiser:
    """Device state of the denoiser: FP32 master parameters, BF16 copy, Adam
    moments and a step counter."""

    def __init__(self, params: np.ndarray | None = None, seed: int = 0, device="cuda"):
        torch = _torch()
        n = nn_param_count()
        p = init_denoiser_params(seed) if params is None else np.asarray(params, np.float32)
        if p.size != n:
            raise ValueError(f"expected {n} parameters, got {p.size}")
        self.params = torch.from_numpy(p.copy()).to(device)
        self.wbf16 = torch.empty(n, dtype=torch.bfloat16, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self._ws = {}
        _check(_nn().vdbc_nn_to_bf16(_dptr(self.params), _dptr(self.wbf16), _stream()))

    def _workspace(self, n, h, w, training):
        key = (n, h, w, training)
        if key not in self._ws:
            b = C.c_uint64(0)
            _check(_nn().vdbc_denoise_workspace(n, h, w, int(training), C.byref(b)))
            self._ws[key] = (_aligned_empty(int(b.value)), int(b.value))
        (buf, ptr), nb = self._ws[key]
        return ptr, nb

    def train_step(self, x, target, lr: float, grad_out=None):
        n, h, w, _ = x.shape
        ptr, nb = self._workspace(n, h, w, True)
        self.step += 1
        _check(_nn().vdbc_denoise_train_step(
            _dptr(self.params), _dptr(self.wbf16), _dptr(self.m), _dptr(self.v), self.step,
            float(lr), _dptr(x), _dptr(target), n, h, w, _dptr(self.loss),
            _dptr(grad_out) if grad_out is not None else None, ptr, nb, _stream()))
        return self.loss

    def __call__(self, x, out=None):
        torch = _torch()
        n, h, w, _ = x.shape
        ptr, nb = self._workspace(n, h, w, False)
        if out is None:
            out = torch.empty((n, h, w, 3), dtype=torch.float32, device=x.device)
        _check(_nn().vdbc_denoise(_dptr(self.params), _dptr(self.wbf16), _dptr(x), n, h, w,
                                  _dptr(out), ptr, nb, _stream()))
        return out


def denoise_pack(rgba, aov, out=None):
    """Network input (BF16 [..., 8]) from render image and AOV tensors."""
    torch = _torch()
    shape = rgba.shape[:-1]
    if out is None:
        out = torch.empty(tuple(shape) + (8,), dtype=torch.bfloat16, device=rgba.device)
    pixels = rgba.numel() // 4
    _check(_nn().vdbc_denoise_pack(_dptr(rgba), _dptr(aov), pixels, _dptr(out), _stream()))
    return out


# ------------------------------------------------------------------ batches

class BatchItemC(C.Structure):
    _fields_ = [("grid", GridC), ("camera", CameraC), ("medium", MediumC),
                ("spp", C.c_uint32), ("max_bounces", C.c_uint32), ("seed", C.c_uint64),
                ("frame", C.c_uint32), ("image", C.c_void_p)]


class TuningC(C.Structure):
    _fields_ = [("macrocell", C.c_uint32), ("tile_w", C.c_uint32),
                ("blocks_per_cu", C.c_uint32), ("persistent", C.c_uint32), ("chunk_spp", C.c_uint32)]


def _batch_signatures(L):
    P, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
    L.vdbc_batch_workspace.argtypes = [P, u32, P, C.POINTER(u64)]
    L.vdbc_batch_create.argtypes = [P, u32, P, P, u64, P, C.POINTER(P)]
    L.vdbc_batch_launch.argtypes = [P, P]
    L.vdbc_batch_capture.argtypes = [P, P]
    L.vdbc_batch_graph_launch.argtypes = [P, P]
    L.vdbc_batch_destroy.argtypes = [P]
    L.vdbc_batch_destroy.restype = None
    for name in ["vdbc_batch_workspace", "vdbc_batch_create", "vdbc_batch_launch",
                 "vdbc_batch_capture", "vdbc_batch_graph_launch"]:
        getattr(L, name).restype = C.c_int


def _bt():
    L = load()
    if not getattr(L, "_batch_ready", False):
        _batch_signatures(L)
        L._batch_ready = True
    return L


def tuning_c(t: dict | None) -> TuningC:
    t = t or {}
    return TuningC(t.get("macrocell", 16), t.get("tile_w", 8), t.get("blocks_per_cu", 4),
                   int(t.get("persistent", 1)), int(t.get("chunk_spp", 0)))


class Batch:
    """Many volumes rendered by one persistent launch (or one launch per
    volume with persistent=0), optionally replayed from a captured graph.

    items: list of dicts with grid (Grid), camera, medium, spp, max_bounces,
    seed, frame; every item gets its own image tensor (h, w, 4)."""

    def __init__(self, items: list, tuning: dict | None = None, device="cuda"):
        torch = _torch()
        L = _bt()
        self.items = items
        self.images = []
        arr = (BatchItemC * len(items))()
        for i, it in enumerate(items):
            cam = it["camera"]
            img = torch.empty((cam["height"], cam["width"], 4), dtype=torch.float32, device=device)
            self.images.append(img)
            a = arr[i]
            a.grid = it["grid"].c
            a.camera = camera_c(cam)
            a.medium = medium_c(it["medium"])
            a.spp = it.get("spp", 1)
            a.max_bounces = it.get("max_bounces", 8)
            a.seed = it.get("seed", 0)
            a.frame = it.get("frame", 0)
            a.image = _dptr(img)
        self._arr = arr
        self.tuning = tuning_c(tuning)
        nb = C.c_uint64(0)
        _check(L.vdbc_batch_workspace(C.cast(arr, C.c_void_p), len(items), C.byref(self.tuning),
                                      C.byref(nb)))
        self.ws, self.ws_ptr = _aligned_empty(int(nb.value), device)
        self.ws_bytes = int(nb.value)
        self.plan = C.c_void_p()
        _check(L.vdbc_batch_create(C.cast(arr, C.c_void_p), len(items), C.byref(self.tuning),
                                   self.ws_ptr, self.ws_bytes, _stream(), C.byref(self.plan)))
        self.captured = False

    def launch(self, stream=None):
        _check(_bt().vdbc_batch_launch(self.plan, stream if stream is not None else _stream()))

    def capture(self, stream):
        """Capture the launch sequence on a non-default torch stream."""
        _check(_bt().vdbc_batch_capture(self.plan, C.c_void_p(stream.cuda_stream)))
        self.captured = True

    def replay(self, stream=None):
        _check(_bt().vdbc_batch_graph_launch(self.plan,
                                             stream if stream is not None else _stream()))

    def close(self):
        if self.plan:
            _bt().vdbc_batch_destroy(self.plan)
            self.plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
