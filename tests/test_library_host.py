"""Host-side checks of libvdbc.so that need no GPU: the C ABI exports every
declared symbol, the host encoder writes the oracle's canonical bytes, the
validator, and argument errors reported before any device work."""
import ctypes as C
import os
from collections import Counter
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2504_04564_amd import _build, vdbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def lib():
    _build.ensure_built()
    return vdbc.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "vdbc.h")).read()
    names = set(re.findall(r"\b(vdbc_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 18
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert lib.vdbc_abi_version() == vdbc.ABI_VERSION == 2


def test_library_records_its_sources_and_stale_builds_are_refused(lib, monkeypatch):
    # the loaded library was built from the sources in the tree ...
    assert _build.built_hash() == _build.source_hash()
    assert len(_build.source_hash()) == 16
    # ... and a library built from other sources is refused, not loaded
    monkeypatch.setattr(_build, "source_hash", lambda: "0" * 16)
    with pytest.raises(_build.StaleLibrary):
        _build.ensure_built()


def test_one_hip_runtime_whatever_the_import_order():
    # torch's wheel carries its own libamdhip64.so.7; loading the library
    # before torch must not leave a second HIP runtime in the process
    import subprocess
    import sys
    code = ("from paper_2504_04564_amd import _build, vdbc\n"
            "_build.ensure_built(); vdbc.load()\n"
            "m = open('/proc/self/maps').read()\n"
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"


def _rand(shape, seed, zero=0.6):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < zero] = 0.0
    return v


ENC_CASES = [
    ((64, 64, 64), 0.25, 2, 0), ((37, 50, 70), 0.3, 1, 0), ((37, 50, 70), 0.3, 3, 4),
    ((130, 20, 140), 0.5, 2, 2), ((8, 8, 8), 1.0, 2, 0), ((200, 9, 3), 0.6, 2, 0),
    ((1, 1, 1), 1.0, 2, 0), ((1, 1, 1), 0.1, 2, 0), ((40, 40, 40), 0.01, 2, 1),
    ((129, 257, 33), 0.07, 2, 0), ((16, 300, 16), 1.0, 3, 0),
]


@pytest.mark.parametrize("shape,q,metric,flags", ENC_CASES)
def test_encoder_bytes_equal_oracle(shape, q, metric, flags):
    v = _rand(shape, 31)
    v[: shape[0] // 2, : shape[1] // 2, : shape[2] // 2] = np.float32(0.75)
    bg = 0.5 if flags & 1 else 0.0
    b1, s1 = vdbc.encode(v, q, metric, flags, bg)
    b2, s2 = oracle.encode(v, q, metric, flags, bg)
    assert b1.size == b2.size
    assert np.array_equal(b1, b2)
    assert s1 == s2
    assert vdbc.validate(b1)["n_leaf"] == s2["n_leaf"]


PARTIAL_CASES = [
    ((64, 96, 128), 0.25, 2, 0, (0.5, 1e30)), ((37, 50, 70), 0.3, 1, 0, (0.3, 0.6)),
    ((37, 50, 70), 0.3, 3, 4, (0.7, 0.4)), ((130, 20, 140), 0.5, 2, 2, (0.25, 1e30)),
    ((45, 70, 90), 1.0, 2, 0, (0.1, 1e30)), ((8, 200, 9), 0.6, 2, 0, (0.01, 1e30)),
    ((1, 1, 1), 1.0, 2, 0, (0.5, 1e30)), ((40, 40, 40), 0.2, 2, 1, (0.5, 1e30)),
    ((129, 257, 33), 0.07, 2, 0, (0.5, 0.99)), ((64, 64, 64), 0.3, 2, 0, (1.0, 1e30)),
]


@pytest.mark.parametrize("shape,q,metric,flags,part", PARTIAL_CASES)
def test_partial_encoder_bytes_equal_oracle(shape, q, metric, flags, part):
    # partial-brick activation: the host encoder writes the oracle's bytes
    v = _rand(shape, 33)
    v[: shape[0] // 2, : shape[1] // 2, : shape[2] // 2] = np.float32(0.75)
    v[v > 0.9] = np.float32(0.95)   # ties in |v - B| inside bricks
    bg = 0.5 if flags & 1 else 0.0
    b1, s1 = vdbc.encode(v, q, metric, flags, bg, partial=part)
    b2, s2 = oracle.encode(v, q, metric, flags, bg, partial=part)
    assert b1.size == b2.size
    assert np.array_equal(b1, b2)
    assert s1 == s2
    assert vdbc.validate(b1)["active_voxels"] == s2["active_voxels"]


def test_partial_encoder_clouds_and_threads():
    v = synth.mid_volume(n=160)
    order, K = oracle.brick_order(v, 0.1)
    for part in ((0.5, 1e30), (0.25, 0.5)):
        b2, _ = oracle.encode(v, 0.1, partial=part)
        for threads in (1, 3, 0):
            b1, _ = vdbc.encode(v, 0.1, threads=threads, partial=part)
            assert np.array_equal(b1, b2), (part, threads)


def test_partial_encoder_rejects_bad_parameters():
    v = _rand((32, 32, 32), 1)
    for part in ((0.0, 1.0), (1.5, 1.0), (float("nan"), 1.0), (0.5, float("nan"))):
        with pytest.raises(vdbc.VdbcError):
            vdbc.encode(v, 0.5, partial=part)
    with pytest.raises(vdbc.VdbcError):
        vdbc.encode(v, 0.5, flags=64)


def test_encoder_bytes_equal_oracle_clouds():
    for v, q in ((synth.tiny_volume(), 0.25), (synth.mid_volume(n=160), 0.1),
                 (synth.mid_volume(n=128), 0.05)):
        for threads in (1, 3, 0):
            b1, _ = vdbc.encode(v, q, threads=threads)
            b2, _ = oracle.encode(v, q)
            assert np.array_equal(b1, b2)


def test_encoder_background_without_dominant_value():
    # dense noise: no bucket dominates, the exact mode falls back to sorting
    v = synth.dense_noise(40, seed=5)
    v.ravel()[::97] = np.float32(0.3125)     # a clear mode
    b1, s1 = vdbc.encode(v, 1.0)
    assert s1["background"] == np.float32(0.3125)
    assert s1["background"] == oracle.background(v)
    w = synth.dense_noise(24, seed=6)         # a few duplicates: smallest of them wins
    _, s2 = vdbc.encode(w, 0.5)
    c = Counter(float(x) for x in w.ravel())
    top = max(c.values())
    assert s2["background"] == oracle.background(w) == min(x for x, k in c.items() if k == top)


def test_encoder_negative_zero_background():
    v = np.zeros((16, 16, 16), np.float32)
    v[::2] = -0.0
    v[0, 0, :3] = 1.0
    _, s = vdbc.encode(v, 0.5)
    assert s["background"] == 0.0 and not np.signbit(s["background"])


def test_encoder_rejects_bad_input():
    v = np.zeros((4, 4, 4), np.float32)
    for q in (0.0, -0.5, 1.01, float("nan")):
        with pytest.raises(vdbc.VdbcError) as e:
            vdbc.encode(v, q)
        assert e.value.status == vdbc.E_INVALID
    w = v.copy()
    w[3, 2, 1] = np.inf
    with pytest.raises(vdbc.VdbcError):
        vdbc.encode(w, 0.5)
    with pytest.raises(vdbc.VdbcError):
        vdbc.encode(v, 0.5, metric=0)
    with pytest.raises(vdbc.VdbcError):
        vdbc.encode(v, 0.5, flags=vdbc.BG_EXPLICIT, background=float("nan"))


def test_one_shot_encode_size_query(lib):
    v = _rand((20, 20, 20), 3)
    d = vdbc.Dims(20, 20, 20)
    p = vdbc.EncodeParams(0.5, 2, 0, 0.0, 0)
    need = C.c_uint64(0)
    st = lib.vdbc_encode(v.ctypes.data, d, C.byref(p), None, 0, C.byref(need), None)
    assert st == vdbc.E_BUFFER_TOO_SMALL and need.value > 0
    raw = np.zeros(need.value + 256, np.uint8)
    off = (-raw.ctypes.data) % 256
    out = raw[off:off + need.value]
    st = lib.vdbc_encode(v.ctypes.data, d, C.byref(p), out.ctypes.data, need.value - 1,
                         C.byref(need), None)
    assert st == vdbc.E_BUFFER_TOO_SMALL
    st = lib.vdbc_encode(v.ctypes.data, d, C.byref(p), out.ctypes.data, need.value,
                         C.byref(need), None)
    assert st == vdbc.OK
    assert np.array_equal(out, oracle.encode(v, 0.5)[0])


def test_validator_rejects_corruption():
    v = _rand((40, 40, 40), 9)
    buf, _ = vdbc.encode(v, 0.5)
    vdbc.validate(buf)
    # magic, version, an unknown node layout, the SoA layout (its node
    # sections are smaller, so the offsets no longer match), sizes, offsets
    for off, val in ((0, 0x58), (4, 2), (36, 4), (36, 2), (152, 1), (104, 1)):
        bad = buf.copy()
        bad[off] = val
        with pytest.raises(vdbc.VdbcError) as e:
            vdbc.validate(bad)
        assert e.value.status == vdbc.E_FORMAT
    # a prefix word in the upper node
    bad = buf.copy()
    h = np.frombuffer(buf[:256].tobytes(), np.uint8)
    off_upper = int(np.frombuffer(h[104:112].tobytes(), "<u8")[0])
    bad[off_upper + 32 + 8] ^= 1
    with pytest.raises(vdbc.VdbcError):
        vdbc.validate(bad)
    with pytest.raises(vdbc.VdbcError):
        vdbc.validate(buf[:-256])


def test_device_calls_reject_bad_arguments_before_launch(lib):
    # every check below fails before any HIP call, so it runs without a GPU
    g = vdbc.GridC()
    assert lib.vdbc_grid_init(C.byref(g), None, 0, None) == vdbc.E_INVALID
    buf, _ = vdbc.encode(_rand((16, 16, 16), 1), 0.5)
    assert lib.vdbc_grid_init(C.byref(g), 256, 16, buf.ctypes.data) == vdbc.E_FORMAT
    assert lib.vdbc_grid_init(C.byref(g), 257, buf.size, buf.ctypes.data) == vdbc.E_INVALID
    assert lib.vdbc_grid_init(C.byref(g), 512, buf.size, buf.ctypes.data) == vdbc.OK
    assert lib.vdbc_sample(C.byref(g), 1024, 10, 2, 2048, None) == vdbc.E_INVALID
    assert lib.vdbc_sample(C.byref(g), None, 10, 1, 2048, None) == vdbc.E_INVALID
    assert lib.vdbc_sample(C.byref(g), None, 0, 1, None, None) == vdbc.OK   # empty
    d = vdbc.Dims(0, 4, 4)
    assert lib.vdbc_sample_dense(1024, d, 0.0, 2048, 4, 1, 4096, None) == vdbc.E_INVALID
    cam = vdbc.camera_c(dict(kind=0, width=0, height=4))
    med = vdbc.medium_c(dict(sigma_scale=1.0, tf=[(0, 0, 0, 0), (1, 1, 1, 1)]))
    prm = vdbc.params_c(dict(), vdbc.MODE_EA)
    assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(med), C.byref(prm), 4096, None,
                           None, 0, None) == vdbc.E_INVALID
    cam = vdbc.camera_c(dict(kind=0, width=4, height=4, dir=(0, 0, 1)))
    bad = vdbc.medium_c(dict(sigma_scale=1.0, tf=[(0, 0, 0, 0)]))
    assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(bad), C.byref(prm), 4096, None,
                           None, 0, None) == vdbc.E_INVALID
    pt = vdbc.params_c(dict(spp=1), vdbc.MODE_PT)
    ws = C.c_uint64(0)
    assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), None, C.byref(ws)) == 0
    assert ws.value == 256 + 256 + 256   # counters | 2^3 majorants | coarse bits
    assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(med), C.byref(pt), 4096, None,
                           8192, ws.value - 1, None) == vdbc.E_BUFFER_TOO_SMALL
    pt.macrocell = 3
    assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), None, C.byref(ws)) == \
        vdbc.E_INVALID
    # split tiles (0 < chunk_spp < spp): 40 bytes of pixel sums per pixel after
    # the occupancy bits, which needs the camera; unsplit launches need neither
    pt.macrocell = 8
    big = vdbc.camera_c(dict(kind=0, width=100, height=30, dir=(0, 0, 1)))
    for spp, chunk, extra in ((8, 2, 120064), (8, 7, 120064), (8, 8, 0), (8, 9, 0), (8, 0, 0), (1, 1, 0)):
        pt.spp, pt.chunk_spp = spp, chunk
        assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), C.byref(big), C.byref(ws)) == 0
        assert ws.value == 768 + extra, (spp, chunk)          # align256(40 * 3000) = 120064
        want = vdbc.OK if extra == 0 else vdbc.E_INVALID
        assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), None, C.byref(ws)) == want
    pt.spp, pt.chunk_spp = 1, 0
    # the cost order: 8 bytes per 256-pixel tile + 512, after the pixel sums;
    # 100 x 30 pixels are 4 x 4 tiles of 32 x 8 (8-wide wave tiles) or 1 x 30
    # tiles of 256 x 1 (64-wide rows)
    pt.flags = vdbc.RENDER_COST_ORDER
    for spp, chunk, tw, extra in ((1, 0, 8, 768), (1, 0, 64, 768), (8, 2, 8, 120064 + 768)):
        pt.spp, pt.chunk_spp, pt.tile_w = spp, chunk, tw
        assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), C.byref(big), C.byref(ws)) == 0
        assert ws.value == 768 + extra, (spp, chunk, tw)
        assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), None, C.byref(ws)) == vdbc.E_INVALID
    pt.tile_w = 128
    assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), C.byref(big), C.byref(ws)) == vdbc.E_INVALID
    pt.spp, pt.chunk_spp, pt.tile_w, pt.flags = 1, 0, 8, 0
    assert lib.vdbc_status_string(3) == b"buffer too small"
    # degenerate scenes are refused before launch
    zero_dir = vdbc.camera_c(dict(kind=0, width=4, height=4))
    assert lib.vdbc_render(C.byref(g), C.byref(zero_dir), C.byref(med), C.byref(prm), 4096,
                           None, None, 0, None) == vdbc.E_INVALID
    pt.macrocell = 8
    assert lib.vdbc_render_workspace(C.byref(pt), vdbc.Dims(16, 16, 16), None, C.byref(ws)) == 0
    no_light = vdbc.medium_c(dict(sigma_scale=1.0, tf=[(0, 0, 0, 0), (1, 1, 1, 1)],
                                  light_dir=(0, 0, 0)))
    assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(no_light), C.byref(pt), 4096,
                           None, 8192, ws.value, None) == vdbc.E_INVALID
    tiny_step = vdbc.params_c(dict(step=1e-6), vdbc.MODE_EA)
    assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(med), C.byref(tiny_step), 4096,
                           None, None, 0, None) == vdbc.E_INVALID


def test_binding_structs_match_c_header(tmp_path):
    # the ctypes mirrors of the ABI structs have the C header's size and offsets
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "vdbc.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(vdbc_batch_item), sizeof(vdbc_tuning), sizeof(vdbc_render_params),'
                   'sizeof(vdbc_medium), sizeof(vdbc_camera), sizeof(vdbc_grid),'
                   'sizeof(vdbc_encode_params), sizeof(vdbc_encode_stats),'
                   'offsetof(vdbc_batch_item, image));return 0;}\n')
    exe = tmp_path / "sz"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(vdbc.BatchItemC), C.sizeof(vdbc.TuningC), C.sizeof(vdbc.RenderParamsC),
            C.sizeof(vdbc.MediumC), C.sizeof(vdbc.CameraC), C.sizeof(vdbc.GridC),
            C.sizeof(vdbc.EncodeParams), C.sizeof(vdbc.EncodeStats), vdbc.BatchItemC.image.offset]
    assert got == want


def test_batch_workspace_holds_the_pixel_sums_of_split_volumes(lib):
    # vdbc_batch_workspace plans on the host only (the grid's device pointer
    # and the images are never touched); a volume whose spp exceeds chunk_spp
    # gets 32 bytes of pixel sums per pixel, the others none
    vdbc._batch_signatures(lib)
    g = vdbc.GridC()
    buf, _ = vdbc.encode(_rand((16, 16, 16), 1), 0.5)
    assert lib.vdbc_grid_init(C.byref(g), 512, buf.size, buf.ctypes.data) == vdbc.OK
    items = (vdbc.BatchItemC * 2)()
    for it, spp in zip(items, (8, 2)):
        it.grid = g
        it.camera = vdbc.camera_c(dict(kind=0, width=100, height=30, dir=(0, 0, 1)))
        it.medium = vdbc.medium_c(dict(sigma_scale=1.0, tf=[(0, 0, 0, 0), (1, 1, 1, 1)]))
        it.spp, it.max_bounces, it.image = spp, 4, 4096

    def ws(**t):
        n = C.c_uint64(0)
        st = lib.vdbc_batch_workspace(C.cast(items, C.c_void_p), 2, C.byref(vdbc.tuning_c(t)), C.byref(n))
        return st, n.value

    st, whole = ws(macrocell=8)
    assert st == vdbc.OK
    for chunk, extra in ((0, 0), (8, 0), (9, 0), (4, 96000), (3, 96000), (1, 2 * 96000)):
        st, n = ws(macrocell=8, chunk_spp=chunk)
        assert st == vdbc.OK
        # align256(32 * 3000) = 96000 per split volume; the item list holds 4
        # bytes per work item (16 tiles of 32 x 8 pixels each) in 256-byte steps
        chunks = [(spp + chunk - 1) // chunk if 0 < chunk < spp else 1 for spp in (8, 2)]
        list_extra = -(-sum(16 * c for c in chunks) * 4 // 256) * 256 - 256
        assert n == whole + extra + list_extra, (chunk, n, whole)
    # more than 2^20 - 1 work items for one volume is refused before any launch
    items[0].camera = vdbc.camera_c(dict(kind=0, width=2048, height=2048, dir=(0, 0, 1)))
    items[0].spp = 65536
    assert ws(macrocell=8, chunk_spp=1)[0] == vdbc.E_INVALID
    assert ws(macrocell=8)[0] == vdbc.OK


def test_iso_and_compare_reject_bad_arguments_before_launch(lib):
    # iso-surface mode and the compression-error call validate everything on
    # the host, so these run without a GPU
    g = vdbc.GridC()
    buf, _ = vdbc.encode(_rand((16, 16, 16), 2), 0.5)
    assert lib.vdbc_grid_init(C.byref(g), 512, buf.size, buf.ctypes.data) == vdbc.OK
    cam = vdbc.camera_c(dict(kind=0, width=4, height=4, dir=(0, 0, 1)))
    for bad in (dict(step=0.0), dict(step=float("nan")), dict(step=1e-6), dict(refine=65),
                dict(iso=float("inf"))):
        prm = vdbc.params_c(bad, vdbc.MODE_ISO)
        assert lib.vdbc_render(C.byref(g), C.byref(cam), None, C.byref(prm), 4096, None, None, 0,
                               None) == vdbc.E_INVALID, bad
    prm = vdbc.params_c(dict(), 3)
    assert lib.vdbc_render(C.byref(g), C.byref(cam), None, C.byref(prm), 4096, None, None, 0,
                           None) == vdbc.E_INVALID
    # the iso mode needs no workspace unless counting
    ws = C.c_uint64(1)
    assert lib.vdbc_render_workspace(C.byref(vdbc.params_c(dict(), vdbc.MODE_ISO)),
                                     vdbc.Dims(16, 16, 16), None, C.byref(ws)) == 0 and ws.value == 0
    # compare: workspace = 5 doubles per workgroup, 64x8x8 voxels per workgroup
    for dims, blocks in (((16, 16, 16), 4), ((64, 8, 8), 1), ((65, 9, 9), 8),
                         ((2048, 2048, 2048), 4096)):
        assert lib.vdbc_compare_workspace(vdbc.Dims(*dims), C.byref(ws)) == 0
        assert ws.value == 40 * blocks, dims
    assert lib.vdbc_compare_workspace(vdbc.Dims(0, 4, 4), C.byref(ws)) == vdbc.E_INVALID
    assert lib.vdbc_compare_dense(C.byref(g), None, 4096, 8192, 160, None) == vdbc.E_INVALID
    assert lib.vdbc_compare_dense(C.byref(g), 4096, 8192, 8192, 8, None) == vdbc.E_BUFFER_TOO_SMALL
    assert lib.vdbc_compare_dense(C.byref(g), 4096, 8192, 8193, 160, None) == vdbc.E_INVALID


def test_path_tracer_limits_rejected_before_launch(lib):
    g = vdbc.GridC()
    buf, _ = vdbc.encode(_rand((16, 16, 16), 3), 0.5)
    assert lib.vdbc_grid_init(C.byref(g), 512, buf.size, buf.ctypes.data) == vdbc.OK
    cam = vdbc.camera_c(dict(kind=0, width=4, height=4, dir=(0, 0, 1)))
    med = vdbc.medium_c(dict(sigma_scale=1.0, tf=[(0, 0, 0, 0), (1, 1, 1, 1)], light_dir=(0, 0, 1)))
    ws = C.c_uint64(0)
    for bad in (dict(spp=0), dict(spp=65537), dict(max_bounces=0), dict(max_bounces=65536),
                dict(tile_w=4), dict(tile_w=12), dict(tile_w=128)):
        prm = vdbc.params_c(dict(dict(spp=1), **bad), vdbc.MODE_PT)
        assert lib.vdbc_render_workspace(C.byref(prm), vdbc.Dims(16, 16, 16), None, C.byref(ws)) == 0
        assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(med), C.byref(prm), 4096, None,
                               8192, ws.value, None) == vdbc.E_INVALID, bad
    # a split launch whose work items overflow the 32-bit queue: 2^23 tiles x
    # 2^16 items of one sample each (the workspace pointer is never touched)
    huge = vdbc.camera_c(dict(kind=0, width=65536, height=32768, dir=(0, 0, 1)))
    prm = vdbc.params_c(dict(spp=65536, chunk_spp=1), vdbc.MODE_PT)
    assert lib.vdbc_render(C.byref(g), C.byref(huge), C.byref(med), C.byref(prm), 4096, None,
                           8192, 1 << 50, None) == vdbc.E_INVALID
    assert b"work items" in lib.vdbc_last_error()
    env_bad = vdbc.medium_c(dict(sigma_scale=1.0, tf=[(0, 0, 0, 0), (1, 1, 1, 1)],
                                 light_dir=(0, 0, 1)))
    env_bad.env, env_bad.env_w, env_bad.env_h = 4096, 0, 4
    prm = vdbc.params_c(dict(spp=1), vdbc.MODE_PT)
    assert lib.vdbc_render(C.byref(g), C.byref(cam), C.byref(env_bad), C.byref(prm), 4096, None,
                           8192, ws.value, None) == vdbc.E_INVALID
