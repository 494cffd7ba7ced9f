"""Autotuner for the path tracer and the batched launch.

Times every candidate of a small search space on the device (one warm-up,
median of `reps` HIP-event timings) and keeps the fastest; choices are
persisted to a JSON file keyed by workload class so later runs reuse them.
Candidates only change launch geometry (wave tile shape, samples per work
item, order of the tiles in the work queue, persistent grid size), the VDB
accessor's per-thread cache policy
(none, last leaf, last leaf and last lower node) or the majorant cell size;
all but the cell size leave
every image bit-identical, the cell size changes the estimator's random
stream but not its expectation.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import vdbc

RENDER_SPACE = {"macrocell": (8, 16, 32, 64), "tile_w": (8, 16, 32, 64), "cache": (0, 1, 2),
                "chunk_spp": (0, 4, 8, 16)}
# the cost order of the work queue is tried on this many of the fastest
# raster-order candidates (a second stage instead of doubling the grid)
ORDER_STAGE = 8
BATCH_SPACE = {"macrocell": (8, 16, 32, 64), "tile_w": (8, 16, 32), "blocks_per_cu": (2, 4, 8),
               "persistent": (1,), "chunk_spp": (0, 1, 2, 4)}


def _median_ms(fn, reps: int) -> float:
    torch = vdbc._torch()
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


def workload_key(kind: str, dims, rate: float, spp: int) -> str:
    """Class of a workload: field kind, log2 bucket of the largest side,
    rate rounded to 1/100, samples per pixel."""
    return f"{kind}/n{int(round(math.log2(max(dims))))}/q{rate:.2f}/spp{spp}"


def load(path: str) -> dict:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(path: str, table: dict):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_render(field, camera: dict, medium: dict, params: dict, background=None,
                space: dict | None = None, reps: int = 5):
    """Best (macrocell, tile_w, cache, chunk_spp, order) for a path-traced
    frame; returns (best, all).  The cache policy is searched for VDB grids
    only; work-item sizes of spp samples or more are the same launch as 0 and
    are skipped; the cost order (order 1) is timed on the ORDER_STAGE fastest
    raster-order (order 0) candidates."""
    space = dict(RENDER_SPACE, **(space or {}))
    caches = space["cache"] if isinstance(field, vdbc.Grid) else (2,)
    spp = params.get("spp", 1)
    chunks = [c for c in space["chunk_spp"] if c == 0 or c < spp]
    results = []
    for C_ in space["macrocell"]:
        for tw in space["tile_w"]:
            for cp in caches:
                for ch in chunks:
                    p = dict(params, macrocell=C_, tile_w=tw, chunk_spp=ch,
                             flags=params.get("flags", 0) | vdbc.CACHE_FLAGS[cp])
                    r = vdbc.Renderer(field, camera, medium, p, vdbc.MODE_PT, background=background)
                    ms = _median_ms(r.launch, reps)
                    del r
                    results.append({"macrocell": C_, "tile_w": tw, "cache": cp, "chunk_spp": ch, "order": 0,
                                    "ms": ms})
    for c in sorted(results, key=lambda x: x["ms"])[:ORDER_STAGE]:
        p = dict(params, macrocell=c["macrocell"], tile_w=c["tile_w"], chunk_spp=c["chunk_spp"],
                 flags=params.get("flags", 0) | vdbc.CACHE_FLAGS[c["cache"]] | vdbc.RENDER_COST_ORDER)
        r = vdbc.Renderer(field, camera, medium, p, vdbc.MODE_PT, background=background)
        ms = _median_ms(r.launch, reps)
        del r
        results.append(dict(c, order=1, ms=ms))
    best = min(results, key=lambda x: x["ms"])
    return best, results


def tune_batch(items: list, space: dict | None = None, reps: int = 5):
    """Best batched-launch tuning for a list of batch items: the grid over
    macrocell, wave tile width, workgroups per CU and launch kind with whole
    tiles as work items, then the item sizes of `chunk_spp` (if the space
    has them) at the fastest candidate of the grid."""
    space = space or BATCH_SPACE

    def timed(t):
        b = vdbc.Batch(items, t)
        ms = _median_ms(b.launch, reps)
        b.close()
        return dict(t, ms=ms)

    results = []
    for C_ in space["macrocell"]:
        for tw in space["tile_w"]:
            for bpc in space["blocks_per_cu"]:
                for pers in space["persistent"]:
                    results.append(timed(dict(macrocell=C_, tile_w=tw, blocks_per_cu=bpc, persistent=pers,
                                              chunk_spp=0)))
    best = min(results, key=lambda x: x["ms"])
    for ch in space.get("chunk_spp", ()):
        if ch:
            t = {k: v for k, v in best.items() if k != "ms"}
            results.append(timed(dict(t, chunk_spp=ch)))
    best = min(results, key=lambda x: x["ms"])
    return best, results


def cached_render_tuning(path: str, key: str, tune_fn):
    """Tuned choice for `key` from the JSON table at `path`, tuning (and
    persisting) it on first use."""
    table = load(path)
    if key not in table:
        best, _ = tune_fn()
        table[key] = best
        save(path, table)
    return table[key]
