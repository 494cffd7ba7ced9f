"""Seeded synthetic inputs shaped like the paper's evaluation volumes.

The paper evaluates on structured-regular float32 volumes (Section 5, table
``tab:datasets``): sparse clouds whose most common value is an empty-space
background.  None of those data sets is available here, so every workload is a
seeded fractal (fBm) value-noise cloud with the same shape, size and sparsity
structure.  This module only *makes inputs*: it holds none of the compression,
sampling or rendering arithmetic, and both the CPU oracle and the GPU path
consume what it returns.

Layout: every volume is a C-contiguous ``float32`` array of shape
``(nz, ny, nx)``, i.e. x is the fastest axis (``idx = x + nx*(y + ny*z)``).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "fbm",
    "tiny_volume",
    "mid_volume",
    "cloud_volume",
    "paper_volume",
    "dense_noise",
    "batch_sizes",
]


def _fade_weights(n: int, spacing: float):
    """Per-axis lattice index and quintic-fade weight for n samples."""
    u = np.arange(n, dtype=np.float64) / spacing
    i = np.floor(u).astype(np.int64)
    t = u - i
    w1 = t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
    return i, w1.astype(np.float32), (1.0 - w1).astype(np.float32)


def _interp(arr: np.ndarray, axis: int, n: int, spacing: float) -> np.ndarray:
    """Separable lattice -> grid interpolation along one axis (elementwise ops
    only, so the result does not depend on a BLAS kernel)."""
    i, w1, w0 = _fade_weights(n, spacing)
    shape = [1, 1, 1]
    shape[axis] = n
    a0 = np.take(arr, i, axis=axis)
    a1 = np.take(arr, i + 1, axis=axis)
    a0 *= w0.reshape(shape)
    a1 *= w1.reshape(shape)
    a0 += a1
    return a0


def _octave(shape, seed: int, octave: int, spacing: float, z0: int = 0,
            nz_total: int | None = None) -> np.ndarray:
    nz, ny, nx = shape
    nzt = nz_total if nz_total is not None else nz
    lx = int((nx - 1) // spacing) + 2
    ly = int((ny - 1) // spacing) + 2
    lz = int((nzt - 1) // spacing) + 2
    rng = np.random.default_rng([int(seed), int(octave)])
    lat = rng.random((lz, ly, lx), dtype=np.float32)
    a = _interp(lat, 2, nx, spacing)            # (lz, ly, nx)
    a = _interp(a, 1, ny, spacing)              # (lz, ny, nx)
    # z pass for the slab [z0, z0+nz) only
    iz, w1, w0 = _fade_weights(nzt, spacing)
    iz, w1, w0 = iz[z0:z0 + nz], w1[z0:z0 + nz], w0[z0:z0 + nz]
    out = a[iz] * w0[:, None, None]
    out += a[iz + 1] * w1[:, None, None]
    return out


def fbm(shape, seed: int, period: float, octaves: int = 4, lacunarity: float = 2.0,
        gain: float = 0.5, billow: bool = False, z0: int = 0,
        nz_total: int | None = None) -> np.ndarray:
    """Fractal sum of value noise in [0, 1], shape (nz, ny, nx).

    Octave o has lattice spacing ``period / lacunarity**o`` voxels; lattice
    values are uniform in [0, 1) from numpy's PCG64 seeded by (seed, o); the
    interpolant uses the quintic fade 6t^5 - 15t^4 + 10t^3 per axis.  With
    ``billow`` each octave contributes |2n - 1| instead of n.  ``z0`` and
    ``nz_total`` select a z-slab of a taller volume (for chunked generation).
    """
    acc = None
    norm = 0.0
    amp = 1.0
    for o in range(octaves):
        n = _octave(shape, seed, o, period / (lacunarity ** o), z0, nz_total)
        if billow:
            n = np.abs(n * np.float32(2.0) - np.float32(1.0))
        n *= np.float32(amp)
        acc = n if acc is None else acc + n
        norm += amp
        amp *= gain
    acc *= np.float32(1.0 / norm)
    return acc


def tiny_volume(seed: int = 1, n: int = 64) -> np.ndarray:
    """64^3 fBm value noise in [0, 1] inside a sphere of radius 28 voxels
    centred at (31.5, 31.5, 31.5), zero outside (background 0)."""
    f = fbm((n, n, n), seed, period=16.0)
    c = (n - 1) / 2.0
    r = 28.0 * n / 64.0
    z, y, x = np.ogrid[0:n, 0:n, 0:n]
    inside = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= r * r
    f[~inside] = 0.0
    return np.ascontiguousarray(np.clip(f, 0.0, 1.0), dtype=np.float32)


def _ellipsoid_mask(shape, semi, z0=0, nz_total=None):
    nz, ny, nx = shape
    nzt = nz_total if nz_total is not None else nz
    cz, cy, cx = (nzt - 1) / 2.0, (ny - 1) / 2.0, (nx - 1) / 2.0
    ax, ay, az = semi[0] * nx, semi[1] * ny, semi[2] * nzt
    z = (np.arange(z0, z0 + nz, dtype=np.float32)[:, None, None] - cz) / az
    y = (np.arange(ny, dtype=np.float32)[None, :, None] - cy) / ay
    x = (np.arange(nx, dtype=np.float32)[None, None, :] - cx) / ax
    return (x * x + y * y + z * z) <= 1.0


def _cloud_from(f, mask, tau, gain):
    d = (f - np.float32(tau)) * np.float32(gain)
    np.clip(d, 0.0, 1.0, out=d)
    d[~mask] = 0.0
    return d


def mid_volume(seed: int = 2, n: int = 512, active: float = 0.30) -> np.ndarray:
    """Sparse cloud: fBm density times an ellipsoid mask, about ``active`` of
    all voxels non-zero, values in [0, 1], background 0."""
    return cloud_volume((n, n, n), seed, active=active)


def cloud_volume(shape, seed: int, active: float = 0.30, billow: bool = False,
                 semi=(0.48, 0.42, 0.46), gain: float = 2.5) -> np.ndarray:
    """fBm cloud of arbitrary shape (nz, ny, nx).  The clip threshold is the
    fBm quantile that leaves ``active`` of all voxels non-zero inside the
    ellipsoid mask (estimated on a fixed strided subsample)."""
    nz, ny, nx = shape
    period = max(nx, ny, nz) / 8.0
    f = fbm(shape, seed, period=period, billow=billow)
    mask = _ellipsoid_mask(shape, semi)
    frac_mask = float(mask.mean())
    keep = min(1.0, active / max(frac_mask, 1e-9))
    sub = f[mask][::7]
    tau = float(np.quantile(sub, 1.0 - keep)) if sub.size else 0.0
    return np.ascontiguousarray(_cloud_from(f, mask, tau, gain))


def paper_volume(seed: int = 3, dims=(1987, 1351, 2449), active: float = 0.25,
                 threads: int = 16, out: np.ndarray | None = None) -> np.ndarray:
    """Paper-scale billowed cloud, dims (nx, ny, nz) = 1987 x 1351 x 2449
    (the WDAS cloud's resolution), generated in z-slabs on several threads.
    About 26.3 GB of float32."""
    nx, ny, nz = dims
    period = max(dims) / 8.0
    semi = (0.48, 0.42, 0.46)
    # threshold from a low-resolution proxy of the same field (every 8th slab)
    probe_z = list(range(0, nz, max(1, nz // 24)))
    vals = []
    for z in probe_z:
        f = fbm((1, ny, nx), seed, period, billow=True, z0=z, nz_total=nz)
        m = _ellipsoid_mask((1, ny, nx), semi, z0=z, nz_total=nz)
        vals.append(f[m][::5])
    sub = np.concatenate(vals)
    frac_mask = 4.0 / 3.0 * math.pi * semi[0] * semi[1] * semi[2]
    keep = min(1.0, active / frac_mask)
    tau = float(np.quantile(sub, 1.0 - keep)) if sub.size else 0.0
    if out is None:
        out = np.empty((nz, ny, nx), dtype=np.float32)
    slab = 32

    def work(z0):
        h = min(slab, nz - z0)
        f = fbm((h, ny, nx), seed, period, billow=True, z0=z0, nz_total=nz)
        m = _ellipsoid_mask((h, ny, nx), semi, z0=z0, nz_total=nz)
        out[z0:z0 + h] = _cloud_from(f, m, tau, 2.5)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, range(0, nz, slab)))
    return out


def dense_noise(n, seed: int = 11) -> np.ndarray:
    """Truly dense white noise in [0, 1): no brick is background-like (the
    adversarial case of the paper's worst-case table).  ``n`` is the cube
    edge or a shape (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if isinstance(n, (int, np.integer)) else tuple(int(x) for x in n)
    return rng.random(shape, dtype=np.float32)


def batch_sizes(count: int = 64, seed: int = 7, lo: int = 32, hi: int = 768):
    """Side lengths log-uniform in [lo, hi] and rates drawn from
    {1:4, 1:6, 1:10, 1:20} for a multi-volume batch."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(int)
    rates = rng.choice(np.array([0.25, 0.15, 0.10, 0.05]), size=count)
    spp = rng.integers(1, 9, size=count)
    return [(int(s), float(q), int(p)) for s, q, p in zip(sides, rates, spp)]
