#!/usr/bin/env python3
"""Benchmark: path-traced Mrays/s of the compressed VDB at 1:10 against the
dense float32 baseline on one MI355X, plus trilinear samples/s, the roofline
of the dominant kernel and the CPU oracle timed on a sample of the same work.

Headline (default, ``--workload paper``): the paper-scale frame.  A
1987x1351x2449 billowed fBm cloud (26.3 GB of float32, the WDAS cloud's
resolution), encoded at 1:10 and resident in HBM; one step = majorant grid
rebuild (the transfer function may change per frame) + delta-tracking path
tracer, 1920x1080 pixels x 64 samples, <= 16 bounces.  The dense array is
rendered on the same GPU with the same kernels as the baseline.
``--workload mid`` runs the same step on the 512^3 cloud (1024x1024 x 16 spp,
<= 8 bounces).  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VDB vs dense samples/s & path-traced Mrays/s at 1:10; relMSE vs oracle"
HBM_PEAK_GBS = 8000.0
BYTES_PER_RENDER_SAMPLE = 32      # 8 float32 corners of one trilinear sample
BYTES_PER_RANDOM_SAMPLE = 48      # + 12 B position + 4 B result (vdbc_sample)
BRICK = 32                        # brick edge of the encoder (Alg. 1)

# majorant cell edge of each frame: the fastest candidate of the render
# autotuner (--workload tune --tune-frame paper / mid) for both the VDB and
# the dense array
DEFAULT_MACROCELL = {"paper": 64, "sweep": 64, "mid": 16,
                     # lossless noise: every block is a stored leaf, and at 16 the
                     # majorant rebuild dominates both frames; 64 gives the fastest
                     # frame for both arrays at 1024^3 and 2048^3
                     "worstcase": 64}
# wave tile width (pixels per wave row) of each frame, the same autotuner's
# choice; the image does not depend on it
DEFAULT_TILE_W = {"paper": 16, "sweep": 16, "mid": 16}
# samples per work item (each 256-pixel tile split into spp / chunk items that
# different workgroups run; 0 = one item per tile), the same autotuner's
# choice; the image does not depend on it
DEFAULT_CHUNK_SPP = {"paper": 8, "sweep": 8, "mid": 4}
# work queue in decreasing estimated tile cost (1) or in raster order (0), the
# same autotuner's choice; the image does not depend on it
DEFAULT_COST_ORDER = {"paper": 1, "sweep": 1, "mid": 1}
# committed rocprofv3 counter summaries of pt_kernel<VdbAcc>, one per frame
PROFILES = {"paper": os.path.join(ROOT, "profiles", "pt_kernel_vdb_paper_1to10.md"),
            "mid": os.path.join(ROOT, "profiles", "pt_kernel_vdb_mid512_1to10.md")}
PROFILE = PROFILES["paper"]
# sources of the PT kernel and its launch: the committed counters are valid
# while these files are unchanged
KERNEL_SOURCES = ["paper_2504_04564_amd/csrc/pt.h", "paper_2504_04564_amd/csrc/render.hip",
                  "paper_2504_04564_amd/csrc/kcommon.h", "paper_2504_04564_amd/csrc/device.h",
                  "paper_2504_04564_amd/csrc/format.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def relmse(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean((x - y) ** 2 / (y * y + 0.01)))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_values(path: str | None = None, launch: str | None = None):
    """Figures of a committed rocprofv3 counter summary of the PT kernel (HBM
    bytes per launch, VALU lane utilisation, L2 hit rate), or {} if the kernel
    sources changed since the counters were taken or (with `launch`, e.g.
    "macrocell=64 tile_w=16 chunk_spp=8 cost_order") the summary describes another launch."""
    path = path or PROFILE
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return {}
    if launch is not None and vals.get("launch") != launch:
        return {}
    try:
        return {"traffic": int(float(vals["traffic_bytes_per_launch"])),
                "valu_lane_utilisation": float(vals["valu_lane_utilisation"]),
                "l2_hit_rate": float(vals["l2_hit_rate"])}
    except (KeyError, ValueError):
        return {}


def host_cpu():
    """CPU model, `nproc` and the cores this process may run on (affinity
    and cgroup quota)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    try:
        q, p = open("/sys/fs/cgroup/cpu.max").read().split()
        if q != "max":
            usable = min(usable, max(1, math.ceil(int(q) / int(p))))
    except (OSError, ValueError):
        pass
    return {"cpu_model": model, "nproc": nproc, "usable_cores": usable}


def time_frames(torch, r, steps, warmup):
    """Times `steps` frames (majorant + path tracer) with HIP events on the
    stream the kernels are launched on (torch's current stream)."""
    for _ in range(warmup):
        r.build_majorant()
        r.launch()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for e in ev:
        e[0].record()
        r.build_majorant()
        e[1].record()
        r.launch()
        e[2].record()
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    maj_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    pt_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    return total_ms / steps, maj_ms, pt_ms


def time_sampler(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def occupied_bricks(vol: np.ndarray, background: float, threads: int) -> np.ndarray:
    """(bx, by, bz) of every 32^3 brick holding a voxel other than the
    background (input preparation for the random-position microbenchmark)."""
    from concurrent.futures import ThreadPoolExecutor
    nz, ny, nx = vol.shape
    nbx, nby, nbz = -(-nx // BRICK), -(-ny // BRICK), -(-nz // BRICK)

    def slab(bz):
        s = vol[bz * BRICK:(bz + 1) * BRICK]
        nzs = s.shape[0]
        occ = np.zeros((nby, nbx), bool)
        for by in range(nby):
            row = s[:, by * BRICK:(by + 1) * BRICK, :] != background
            cols = row.reshape(nzs * row.shape[1], nx).any(axis=0)
            pad = np.zeros(nbx * BRICK, bool)
            pad[:nx] = cols
            occ[by] = pad.reshape(nbx, BRICK).any(axis=1)
        return occ

    with ThreadPoolExecutor(max_workers=threads) as ex:
        occ = np.stack(list(ex.map(slab, range(nbz))))       # (nbz, nby, nbx)
    bz, by, bx = np.nonzero(occ)
    return np.stack([bx, by, bz], axis=1).astype(np.int64)


def oracle_baseline(fld, cam, med, prm, img, W, H, spp, pixels, threads, cpu):
    """The CPU oracle timed on the GPU host: majorant grid over the whole
    volume (disjoint cell ranges on `threads` concurrent calls; its
    single-core time is the sum of the calls' thread CPU times), then the
    path tracer on `pixels` random pixels on one core and on `threads` x
    `pixels` more pixels in concurrent calls.  Returns (cpu_baseline, relMSE
    of the GPU image against the oracle on every oracle pixel)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    C = prm["macrocell"]
    f = fld.f
    g = [(-(-n // C)) for n in (f.nz, f.ny, f.nx)]
    mj = np.zeros(g, np.float64)
    cuts = np.linspace(0, mj.size, 8 * threads + 1).astype(np.int64)

    def chunk(i):
        t0 = time.thread_time()
        oracle.majorant(fld, med, C, (cuts[i], cuts[i + 1]), mj)
        return time.thread_time() - t0

    t = time.time()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        maj_cpu = float(sum(ex.map(chunk, range(len(cuts) - 1))))
    maj_wall = time.time() - t
    log(f"[bench] oracle majorant: {maj_wall:.1f}s on {threads} threads ({maj_cpu:.1f} core-s)")
    rng = np.random.default_rng(52)
    n_all = min(pixels * (threads + 1), W * H)   # at most every pixel once
    pix_all = np.sort(rng.choice(W * H, n_all, replace=False)).astype(np.uint32)
    pix1 = pix_all[::threads + 1]
    rest = np.setdiff1d(pix_all, pix1)
    t = time.time()
    ref1 = oracle.render_pt(fld, cam, med, prm, pixels=pix1, majorant=mj)
    t1 = time.time() - t
    rays = W * H * spp
    frame1 = maj_cpu + t1 * (W * H / len(pix1))
    out = {"value": round(rays / frame1 / 1e6, 6), "unit": "Mrays/s", "cores": 1,
           "kind": "oracle",
           "sample": f"{len(pix1)} random pixels x {spp} spp of the same frame on one core "
                     f"({t1:.1f}s) plus the majorant grid of the whole volume ({maj_cpu:.1f} "
                     f"core-s); frame time extrapolated as majorant + paths x {W * H}/{len(pix1)}",
           **cpu}
    errs = [relmse(img[pix1], ref1) * len(pix1)]
    log(f"[bench] oracle 1 core: {out['value']:.4f} Mrays/s ({len(pix1)} pixels in {t1:.1f}s)")
    if threads > 1 and len(rest):
        parts = np.array_split(rest, threads)
        t = time.time()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            refs = list(ex.map(lambda pp: oracle.render_pt(fld, cam, med, prm, pixels=pp,
                                                           majorant=mj), parts))
        tp = time.time() - t
        frame_p = maj_wall + tp * (W * H / len(rest))
        out["all_cores"] = {
            "value": round(rays / frame_p / 1e6, 6), "unit": "Mrays/s", "cores": threads,
            "sample": f"{len(rest)} random pixels x {spp} spp in {threads} concurrent oracle "
                      f"calls ({tp:.1f}s) after the threaded majorant ({maj_wall:.1f}s); frame "
                      f"time extrapolated as majorant + paths x {W * H}/{len(rest)}"}
        errs += [relmse(img[pp], rr) * len(pp) for pp, rr in zip(parts, refs)]
        log(f"[bench] oracle {threads} threads: {out['all_cores']['value']:.3f} Mrays/s")
    rel = float(sum(errs) / len(pix_all if threads > 1 else pix1))
    out["relmse_pixels"] = int(len(pix_all) if threads > 1 else len(pix1))
    return out, rel


def main():
    cpu = host_cpu()
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rate", type=float, default=0.10)
    ap.add_argument("--size", type=int, default=512, help="mid workload: cloud edge")
    ap.add_argument("--cpu-pixels", type=int, default=None,
                    help="pixels the single-core CPU oracle renders (default 32768 on the "
                         "paper frame, 65536 on the mid frame)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=cpu["usable_cores"],
                    help="host threads for the majorant and the all-core oracle figure "
                         "(default: the cores this process may use)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the dense renderer and the random-sample microbenchmark")
    ap.add_argument("--macrocell", type=int, default=None,
                    help="majorant cell edge in voxels (default: the render autotuner's choice for the "
                         "workload's frame, 64 for the paper-scale frame, 16 for the 512^3 one)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales the HBM byte counters)")
    ap.add_argument("--train-steps", type=int, default=1500, help="denoiser workload: Adam steps")
    ap.add_argument("--denoiser-full", action="store_true",
                    help="denoiser workload: 1,000 crops of 512^2 with 1024-spp targets from 256^3..512^3 "
                         "clouds (about 14 minutes) instead of 96 crops of 256^2 with 512-spp targets")
    ap.add_argument("--denoiser-part", type=int, default=0, choices=(0, 1, 2),
                    help="with --denoiser-full: 1 = crops of volumes 0..49, train, write the "
                         "checkpoint; 2 = resume from it with the crops of volumes 50..99")
    ap.add_argument("--denoiser-ckpt", default="denoiser_ckpt.npz",
                    help="checkpoint file of --denoiser-part")
    ap.add_argument("--workload", default="paper",
                    choices=("paper", "mid", "sweep", "denoiser", "batch", "quality", "worstcase",
                             "iso", "ea", "tune"),
                    help="paper: the headline 1987x1351x2449 frame at --rate; mid: the same step "
                         "on the 512^3 cloud; sweep: paper-scale rates 1:20..1:4 and dense; "
                         "denoiser: train and evaluate the learned denoiser; batch: 64 volumes; "
                         "quality: MSE/PSNR vs rate and metric; worstcase: lossless dense noise; "
                         "iso: iso-surface marcher; ea: emission-absorption marcher; "
                         "tune: the render autotuner on the mid frame")
    ap.add_argument("--vdb-cache", default=None,
                    help="paper/mid frame: file holding the encoded buffer.  Written after "
                         "encoding; with --no-extras an existing file is read instead of "
                         "generating and encoding the volume (profiling passes)")
    ap.add_argument("--tune-frame", default="mid", choices=("mid", "paper"),
                    help="tune workload: the frame whose launch configuration is searched")
    ap.add_argument("--worst-max", type=int, default=1024,
                    help="worstcase workload: largest noise cube edge (2048 = the paper's 34 GB)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the compressed volume and the dense baseline both "
              "fit in one MI355X's 288 GB, so no multi-GPU run exists (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_04564_amd import _build, vdbc
    import synth
    from synth import scenes

    _build.ensure_built()
    vdbc.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        # a plain copy kernel of known size: 1 GiB read + 1 GiB written per launch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "launches": 3}))
        return
    if args.macrocell is None:
        args.macrocell = DEFAULT_MACROCELL.get(args.workload, 16)
    args.chunk_spp = DEFAULT_CHUNK_SPP.get(args.workload, 0)
    args.tile_w = DEFAULT_TILE_W.get(args.workload, 8)
    args.order_flag = vdbc.RENDER_COST_ORDER if DEFAULT_COST_ORDER.get(args.workload, 0) else 0
    if args.workload not in ("paper", "mid"):
        import bench_workloads
        line = getattr(bench_workloads, args.workload)(args, torch, vdbc, synth, scenes, log)
        print(json.dumps(line), flush=True)
        return

    threads = max(1, args.cpu_threads)
    if args.workload == "paper":
        S = scenes.PAPER
        nx, ny, nz = S["dims"]
        name = f"fbm-cloud-{nx}x{ny}x{nz}-billowed"
        cpu_pixels = args.cpu_pixels or 32768
    else:
        S = scenes.MID
        nx = ny = nz = args.size
        name = f"fbm-cloud-{nx}^3"
        cpu_pixels = args.cpu_pixels or 65536
    dims = (nx, ny, nz)
    W, H, spp, bounces = S["width"], S["height"], S["spp"], S["max_bounces"]
    vol_bytes = 4 * nx * ny * nz
    cached = bool(args.vdb_cache and args.no_extras and os.path.exists(args.vdb_cache))
    if cached:
        # a profiling pass: the buffer an earlier run of this workload encoded
        raw = np.fromfile(args.vdb_cache, dtype=np.uint8)
        buf = vdbc._aligned(raw.size)
        buf[:] = raw
        del raw
        st = vdbc.validate(buf)
        st["achieved_rate"] = st["active_voxels"] / (nx * ny * nz)
        h = tuple(int(x) for x in np.frombuffer(buf[8:20].tobytes(), "<u4"))
        if h != dims:
            raise SystemExit(f"{args.vdb_cache} holds a {h} volume, not {dims}")
        vol = None
        encode_s = 0.0
        log(f"[bench] read the encoded buffer from {args.vdb_cache} ({buf.size / 1e6:.1f} MB)")
    else:
        log(f"[bench] generating the {name} cloud on {threads} threads")
        t = time.time()
        vol = (synth.paper_volume(dims=S["dims"], threads=threads) if args.workload == "paper"
               else synth.mid_volume(n=nx))
        log(f"[bench] volume ready in {time.time() - t:.1f}s ({vol.nbytes / 1e9:.2f} GB); "
            f"encoding at rate {args.rate}")
        t = time.time()
        buf, st = vdbc.encode(vol, args.rate)
        encode_s = time.time() - t
        log(f"[bench] encoded {buf.size / 1e6:.1f} MB in {encode_s:.2f}s "
            f"(achieved rate {st['achieved_rate']:.4f})")
        if args.vdb_cache:
            buf.tofile(args.vdb_cache)
            if args.no_extras:
                del vol
                vol = None
    torch.cuda.synchronize()
    t = time.time()
    grid = vdbc.Grid(buf)
    torch.cuda.synchronize()
    upload_s = time.time() - t
    cam = scenes.orbit_camera(dims, W, H)
    med = scenes.pt_medium(64.0)
    C = args.macrocell
    # the timed frames run the kernels without counters; one more frame with
    # them (the same paths: the image must be bit-identical) gives the
    # trilinear samples and path segments per frame
    prm = dict(spp=spp, max_bounces=bounces, seed=S["seed"], macrocell=C,
               tile_w=args.tile_w, chunk_spp=args.chunk_spp,
               flags=vdbc.RENDER_KEEP_MAJORANT | args.order_flag)
    prm_count = dict(prm, flags=vdbc.RENDER_COUNT | vdbc.RENDER_KEEP_MAJORANT | args.order_flag)
    rays = W * H * spp

    def counted(field, timed_image, **kw):
        r = vdbc.Renderer(field, cam, med, prm_count, vdbc.MODE_PT, **kw)
        r.build_majorant()
        r.launch()
        torch.cuda.synchronize()
        if not torch.equal(r.image.view(torch.int32), timed_image.view(torch.int32)):
            raise RuntimeError("the counting launch rendered another image")
        return r.sample_count(), r.segment_count()

    r_vdb = vdbc.Renderer(grid, cam, med, prm, vdbc.MODE_PT)
    ms_step, maj_ms, pt_ms = time_frames(torch, r_vdb, args.steps, args.warmup)
    samples, segments = counted(grid, r_vdb.image)
    img = r_vdb.image.cpu().numpy().reshape(-1, 4)
    del r_vdb
    vdb_mrays = rays / (ms_step * 1e-3) / 1e6
    log(f"[bench] VDB PT: {ms_step:.2f} ms/frame (majorant {maj_ms:.2f} ms, PT {pt_ms:.2f} ms), "
        f"{vdb_mrays:.1f} Mrays/s, {samples / 1e6:.1f} M samples and {segments / 1e6:.1f} M segments/frame")

    extras = {}
    if not args.no_extras and vol is not None:
        t = time.time()
        dense = torch.from_numpy(vol).cuda()
        torch.cuda.synchronize()
        log(f"[bench] dense array uploaded in {time.time() - t:.1f}s")
        r_d = vdbc.Renderer(dense, cam, med, prm, vdbc.MODE_PT, background=0.0)
        d_step, d_maj, d_pt = time_frames(torch, r_d, args.steps, args.warmup)
        d_samples, d_segments = counted(dense, r_d.image, background=0.0)
        del r_d
        dense_mrays = rays / (d_step * 1e-3) / 1e6
        log(f"[bench] dense PT: {d_step:.2f} ms/frame (majorant {d_maj:.2f} ms, PT {d_pt:.2f} ms), "
            f"{dense_mrays:.1f} Mrays/s")
        # random-position trilinear microbenchmark: positions uniform inside
        # bricks that hold a non-background voxel
        occ = occupied_bricks(vol, 0.0, threads)
        ns = 1 << 26
        g = torch.Generator(device="cuda").manual_seed(7)
        ob = torch.from_numpy(occ).cuda()
        pick = torch.randint(0, ob.shape[0], (ns,), device="cuda", generator=g)
        off = torch.rand((ns, 3), device="cuda", generator=g) * BRICK - 0.5
        hi = torch.tensor([nx - 0.5, ny - 0.5, nz - 0.5], device="cuda")
        pos = torch.minimum(ob[pick].to(torch.float32) * BRICK + off, hi).contiguous()
        del pick, off, ob
        out = torch.empty(ns, dtype=torch.float32, device="cuda")
        sv_ms = time_sampler(torch, lambda: vdbc.sample(grid, pos, 1, out), args.steps, 2)
        sd_ms = time_sampler(torch, lambda: vdbc.sample_dense(dense, 0.0, pos, 1, out),
                             args.steps, 2)
        extras = {
            "dense_mrays_per_s": round(dense_mrays, 3),
            "vdb_over_dense_mrays": round(vdb_mrays / dense_mrays, 4),
            "dense_ms_per_step": round(d_step, 4),
            "dense_majorant_ms": round(d_maj, 4),
            "segments_per_s": {   # camera + shadow + scattered rays per second of frame
                "vdb_render": round(segments / (ms_step * 1e-3), 1),
                "dense_render": round(d_segments / (d_step * 1e-3), 1),
            },
            "samples_per_s": {
                "vdb_render": round(samples / (pt_ms * 1e-3), 1),
                "dense_render": round(d_samples / (d_pt * 1e-3), 1),
                "vdb_sample_random_2^26": round(ns / (sv_ms * 1e-3), 1),
                "dense_sample_random_2^26": round(ns / (sd_ms * 1e-3), 1),
            },
            "random_sample_positions": f"2^26 uniform inside the {len(occ)} of "
                                       f"{math.prod(-(-d // BRICK) for d in dims)} bricks that hold "
                                       "a non-background voxel",
            "random_sample_gbs": {
                "vdb": round(ns * BYTES_PER_RANDOM_SAMPLE / (sv_ms * 1e-3) / 1e9, 2),
                "dense": round(ns * BYTES_PER_RANDOM_SAMPLE / (sd_ms * 1e-3) / 1e9, 2),
            },
        }
        log(f"[bench] random samples/s: VDB {ns / (sv_ms * 1e-3) / 1e9:.2f} G, "
            f"dense {ns / (sd_ms * 1e-3) / 1e9:.2f} G")
        del pos, out, dense
        torch.cuda.empty_cache()
        # the HBM bandwidth a plain streaming copy reaches on this GPU (1 GiB
        # read + 1 GiB written per launch), next to the 8 TB/s datasheet figure
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        copy_ms = time_sampler(torch, lambda: y.copy_(x), 5, 2)
        extras["hbm_copy_gbs"] = round(2 * x.numel() * 4 / (copy_ms * 1e-3) / 1e9, 1)
        log(f"[bench] streaming copy: {extras['hbm_copy_gbs']:.0f} GB/s")
        del x, y
    del vol

    cpu_line = None
    rel = None
    if not args.no_cpu_baseline:
        import oracle
        log(f"[bench] CPU oracle on {cpu_pixels} (+{cpu_pixels * threads} on {threads} threads) "
            f"of {W * H} pixels")
        oprm = dict(spp=spp, max_bounces=bounces, seed=S["seed"], macrocell=C)
        cpu_line, rel = oracle_baseline(oracle.VdbField(buf), cam, med, oprm, img, W, H, spp,
                                        cpu_pixels, threads, cpu)
        log(f"[bench] relMSE GPU vs oracle {rel:.3e} on {cpu_line['relmse_pixels']} pixels")

    pt_s = pt_ms * 1e-3
    prof_path = PROFILES[args.workload]
    standard = (args.rate == 0.10 and C == DEFAULT_MACROCELL[args.workload] and
                (args.workload == "paper" or nx == 512))
    launch = f"macrocell={C} tile_w={prm['tile_w']} chunk_spp={prm['chunk_spp']}" + \
        (" cost_order" if args.order_flag else "")
    prof = profile_values(prof_path, launch) if standard else {}
    achieved = samples * BYTES_PER_RENDER_SAMPLE / pt_s / 1e9
    line = {
        "metric": METRIC,
        "value": round(vdb_mrays, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{name}-vdb-1:{round(1 / args.rate)}-pt-{W}x{H}x{spp}spp-"
                        f"{bounces}bounces",
            "dims": list(dims), "rate": args.rate, "width": W, "height": H, "spp": spp,
            "max_bounces": bounces, "macrocell": C, "tile_w": prm["tile_w"], "chunk_spp": prm["chunk_spp"],
            "cost_order": bool(args.order_flag),
            "vdb_bytes": int(buf.size), "dense_bytes": vol_bytes,
            "achieved_rate": round(st["achieved_rate"], 5),
        },
        "roofline": {
            # the committed counters describe this exact workload only
            "kernel": "pt_kernel<VdbAcc>",
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "frac_of_measured_copy": (round(achieved / extras["hbm_copy_gbs"], 5)
                                      if "hbm_copy_gbs" in extras else None),
            "traffic": prof.get("traffic"),
            "limiter": ({"kind": "VALU issue of divergent lanes (counters of the same kernel build)",
                         "valu_lane_utilisation": prof["valu_lane_utilisation"],
                         "l2_hit_rate": prof["l2_hit_rate"],
                         "source": os.path.relpath(prof_path, ROOT)} if prof else None),
            "per_launch": {"samples": int(samples), "segments": int(segments),
                           "bytes_per_sample": BYTES_PER_RENDER_SAMPLE,
                           "algorithmic_bytes": int(samples * BYTES_PER_RENDER_SAMPLE),
                           "avg_ms": round(pt_ms, 4)},
        },
        "cpu_baseline": cpu_line,
        "relmse_vs_oracle": rel,
        "encode_s": round(encode_s, 3),
        "upload_s": round(upload_s, 4),
        "majorant_ms": round(maj_ms, 4),
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
