"""Training data, training loop and evaluation of the learned denoiser.

Everything numeric runs in libvdbc.so: the renders (vdbc_render with AOVs),
the input packing, the training step (forward, loss, backward, Adam) and the
inference.  This module only sequences the calls.  Volumes and cameras are
passed in by the caller.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from . import vdbc


def render_pair(grid, camera: dict, medium: dict, spp_in: int, spp_ref: int, seed: int,
                max_bounces: int = 8, macrocell: int = 16):
    """One training example: network input (BF16 [h][w][8]) from a spp_in
    render with AOVs, and the RGB of an independent spp_ref render (FP32)."""
    torch = vdbc._torch()
    lo = vdbc.Renderer(grid, camera, medium,
                       dict(spp=spp_in, max_bounces=max_bounces, seed=seed, macrocell=macrocell),
                       vdbc.MODE_PT, aov=True)
    img = lo.launch()
    x = vdbc.denoise_pack(img, lo.aov)
    hi = vdbc.Renderer(grid, camera, medium,
                       dict(spp=spp_ref, max_bounces=max_bounces, seed=seed ^ 0x9E3779B97F4A7C15,
                            macrocell=macrocell), vdbc.MODE_PT)
    ref = hi.launch()[..., :3].contiguous()
    return x.clone(), ref.clone()


def relmse(x, y):
    """Mean over pixels and channels of (x - y)^2 / (y^2 + 0.01)."""
    torch = vdbc._torch()
    x = x.to(torch.float64)
    y = y.to(torch.float64)
    return float(((x - y) ** 2 / (y * y + 0.01)).mean().item())


def train(dn: "vdbc.Denoiser", xs, ts, steps: int, batch: int, lr: float, seed: int = 0,
          log_every: int = 0):
    """Adam on random batches of the (x, target) crops; returns the loss
    history (one value per step, read back at the end)."""
    torch = vdbc._torch()
    rng = np.random.default_rng(seed)
    n = xs.shape[0]
    losses = torch.empty(steps, dtype=torch.float32, device=xs.device)
    # every step's batch drawn up front and uploaded once: a per-step upload
    # from pageable host memory would wait for the previous step's kernels
    picks = np.stack([rng.choice(n, size=min(batch, n), replace=False) for _ in range(steps)]) \
        if steps else np.zeros((0, min(batch, n)), np.int64)
    all_idx = torch.from_numpy(picks).to(xs.device)
    for s in range(steps):
        idx = all_idx[s]
        loss = dn.train_step(xs.index_select(0, idx).contiguous(),
                             ts.index_select(0, idx).contiguous(), lr)
        losses[s] = loss[0]
        if log_every and (s + 1) % log_every == 0:
            print(f"[denoiser] step {s + 1}/{steps} loss {loss.item():.5f}", file=sys.stderr, flush=True)
    return losses.cpu().numpy()


def evaluate(dn: "vdbc.Denoiser", grid, camera: dict, medium: dict, seed: int,
             spp_in: int = 4, spp_plain: int = 64, spp_ref: int = 1024, max_bounces: int = 8,
             macrocell: int = 16, reps: int = 3):
    """relMSE against a spp_ref reference of: the plain spp_in render, the
    plain spp_plain render and the denoised spp_in render; and the wall time
    (HIP events, median of `reps`) of the plain spp_plain render and of the
    denoised pipeline (spp_in render + pack + network)."""
    torch = vdbc._torch()
    prm = lambda spp, sd: dict(spp=spp, max_bounces=max_bounces, seed=sd, macrocell=macrocell)
    ref = vdbc.Renderer(grid, camera, medium, prm(spp_ref, seed ^ 0xABCDEF), vdbc.MODE_PT)
    ref_img = ref.launch()[..., :3].clone()
    lo = vdbc.Renderer(grid, camera, medium, prm(spp_in, seed), vdbc.MODE_PT, aov=True)
    plain = vdbc.Renderer(grid, camera, medium, prm(spp_plain, seed + 1), vdbc.MODE_PT)
    h, w = camera["height"], camera["width"]
    out = torch.empty((1, h, w, 3), dtype=torch.float32, device="cuda")

    def pipeline():
        img = lo.launch()
        x = vdbc.denoise_pack(img, lo.aov).view(1, h, w, 8)
        dn(x, out)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    t_den = timed(pipeline)
    den = out[0].clone()
    t_plain = timed(lambda: plain.launch())
    plain_img = plain.image[..., :3].clone()
    lo_img = lo.image[..., :3].clone()
    return {
        "relmse_plain_lo": relmse(lo_img, ref_img),
        "relmse_plain_hi": relmse(plain_img, ref_img),
        "relmse_denoised": relmse(den, ref_img),
        "ms_plain_hi": t_plain,
        "ms_denoised_pipeline": t_den,
        "spp_in": spp_in, "spp_plain": spp_plain, "spp_ref": spp_ref,
    }


def timed_section(label: str):
    """Small wall-clock helper for drivers."""
    class _T:
        def __enter__(self):
            self.t = time.time()
            return self

        def __exit__(self, *a):
            print(f"[denoiser] {label}: {time.time() - self.t:.1f}s", file=sys.stderr, flush=True)
    return _T()
