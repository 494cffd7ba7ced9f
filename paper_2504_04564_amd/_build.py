"""Builds libvdbc.so in-tree: host C++ with g++, HIP kernels with hipcc for
gfx950, linked by hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libvdbc.so")
OBJ = os.path.join(HERE, "_obj")

HOST_SOURCES = ["api.cpp", "encode.cpp", "layout.cpp"]
HIP_SOURCES = ["sample.hip", "render.hip", "denoise.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # no packed-FP32 instructions anywhere in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra",
              "-Wno-unused-parameter", "-I", os.path.join(ROOT, "include")]


def source_hash() -> str:
    """Hash of everything the library is built from: the sources under
    csrc/, the public header and the compiler flags (16 hex digits)."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".h", ".hip")))
    for f in files:
        h.update(f.encode() + b"\0")
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "vdbc.h"), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join(HIP_FLAGS[:1] + HOST_FLAGS[:1] + [ARCH]).encode())
    return h.hexdigest()[:16]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libvdbc.so (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    stamp = [f'-DVDBC_SOURCE_HASH="{source_hash()}"']
    for s in HOST_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        jobs.append(["g++"] + HOST_FLAGS + (stamp if s == "api.cpp" else []) +
                    ["-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        jobs.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-pthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def built_hash(path: str = LIB) -> str:
    """Source hash recorded in a built library (vdbc_source_hash)."""
    import ctypes
    import torch  # noqa: F401  (torch's HIP runtime first: see vdbc._torch_hip_first)
    L = ctypes.CDLL(path)
    L.vdbc_source_hash.restype = ctypes.c_char_p
    return L.vdbc_source_hash().decode()


class StaleLibrary(RuntimeError):
    pass


def ensure_built() -> str:
    """Builds when no library exists yet; refuses (StaleLibrary) a library
    built from sources other than the ones in the tree, so a stale binary is
    never tested or measured."""
    if not os.path.exists(LIB):
        build()
        return LIB
    have, want = built_hash(), source_hash()
    if have != want:
        raise StaleLibrary(f"{LIB} was built from sources {have}, the tree holds {want}: "
                           "rebuild with `python -m paper_2504_04564_amd._build`")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
