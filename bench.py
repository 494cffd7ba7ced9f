#!/usr/bin/env python3
"""Benchmark: path-traced Mrays/s of the compressed VDB at 1:10 against the
dense float32 baseline on one MI355X, plus trilinear samples/s, the roofline
of the dominant kernel and the CPU oracle timed on a sample of the same work.

One step = one frame of the hot path on the resident 512^3 cloud: majorant
grid rebuild (the transfer function may change per frame) + delta-tracking
path tracer, 1024x1024 pixels x 16 samples, <= 8 bounces.  Prints one JSON
line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def relmse(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean((x - y) ** 2 / (y * y + 0.01)))


PROFILE = os.path.join(ROOT, "profiles", "pt_kernel_vdb_mid512_1to10.md")
# sources of the PT kernel and its launch: the committed counters are valid
# while these files are unchanged
KERNEL_SOURCES = ["paper_2504_04564_amd/csrc/pt.h", "paper_2504_04564_amd/csrc/render.hip",
                  "paper_2504_04564_amd/csrc/kcommon.h", "paper_2504_04564_amd/csrc/device.h",
                  "paper_2504_04564_amd/csrc/format.h"]


def profile_values():
    """Figures of the committed rocprofv3 counter summary of the PT kernel
    (HBM bytes per launch, VALU lane utilisation, L2 hit rate), or {} if the
    kernel sources changed since the counters were taken."""
    import hashlib
    if not os.path.exists(PROFILE):
        return {}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    for line in open(PROFILE):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != h.hexdigest()[:16]:
        return {}
    try:
        return {"traffic": int(float(vals["traffic_bytes_per_launch"])),
                "valu_lane_utilisation": float(vals["valu_lane_utilisation"]),
                "l2_hit_rate": float(vals["l2_hit_rate"])}
    except (KeyError, ValueError):
        return {}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rate", type=float, default=0.10)
    ap.add_argument("--size", type=int, default=512, help="cloud edge (512 = the workload)")
    ap.add_argument("--cpu-pixels", type=int, default=65536,
                    help="pixels of the frame the CPU oracle renders for its baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads for the all-core oracle figure (1 = single-core only)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the dense renderer and the random-sample microbenchmark")
    ap.add_argument("--macrocell", type=int, default=16, help="majorant cell edge in voxels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales the HBM byte counters)")
    ap.add_argument("--train-steps", type=int, default=1500, help="denoiser workload: Adam steps")
    ap.add_argument("--denoiser-full", action="store_true",
                    help="denoiser workload: 1,000 crops of 512^2 with 1024-spp targets from 256^3..512^3 "
                         "clouds (about 14 minutes) instead of 96 crops of 256^2 with 512-spp targets")
    ap.add_argument("--workload", default="mid",
                    choices=("mid", "paper", "denoiser", "batch", "quality", "worstcase", "iso", "ea", "tune"),
                    help="mid: the headline 512^3 frame; paper: 1987x1351x2449 rate sweep; "
                         "denoiser: train and evaluate the learned denoiser; batch: 64 volumes; "
                         "quality: MSE/PSNR vs rate and metric; worstcase: lossless dense noise; "
                         "iso: iso-surface marcher; ea: emission-absorption marcher; "
                         "tune: the render autotuner on the headline frame")
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
    if args.workload != "mid":
        import bench_workloads
        line = getattr(bench_workloads, args.workload)(args, torch, vdbc, synth, scenes, log)
        print(json.dumps(line), flush=True)
        return
    M = scenes.MID
    n = args.size
    W, H, spp, bounces = M["width"], M["height"], M["spp"], M["max_bounces"]

    log(f"[bench] generating {n}^3 cloud")
    t = time.time()
    vol = synth.mid_volume(n=n)
    log(f"[bench] volume ready in {time.time() - t:.1f}s; encoding at rate {args.rate}")
    t = time.time()
    buf, st = vdbc.encode(vol, args.rate)
    encode_s = time.time() - t
    log(f"[bench] encoded {buf.size / 1e6:.1f} MB in {encode_s:.2f}s "
        f"(achieved rate {st['achieved_rate']:.4f})")
    torch.cuda.synchronize()
    t = time.time()
    grid = vdbc.Grid(buf)
    torch.cuda.synchronize()
    upload_s = time.time() - t
    dense = torch.from_numpy(vol).cuda()
    cam = scenes.orbit_camera((n, n, n), W, H)
    med = scenes.pt_medium(64.0)
    C = args.macrocell
    prm = dict(spp=spp, max_bounces=bounces, seed=M["seed"], macrocell=C,
               flags=vdbc.RENDER_COUNT | vdbc.RENDER_KEEP_MAJORANT)
    rays = W * H * spp

    r_vdb = vdbc.Renderer(grid, cam, med, prm, vdbc.MODE_PT)
    ms_step, maj_ms, pt_ms = time_frames(torch, r_vdb, args.steps, args.warmup)
    samples = r_vdb.sample_count()
    img = r_vdb.image.cpu().numpy().reshape(-1, 4)
    vdb_mrays = rays / (ms_step * 1e-3) / 1e6
    log(f"[bench] VDB PT: {ms_step:.2f} ms/frame (majorant {maj_ms:.2f} ms, PT {pt_ms:.2f} ms), "
        f"{vdb_mrays:.1f} Mrays/s, {samples / 1e6:.1f} M samples/frame")

    extras = {}
    if not args.no_extras:
        r_d = vdbc.Renderer(dense, cam, med, prm, vdbc.MODE_PT, background=0.0)
        d_step, d_maj, d_pt = time_frames(torch, r_d, args.steps, args.warmup)
        d_samples = r_d.sample_count()
        dense_mrays = rays / (d_step * 1e-3) / 1e6
        log(f"[bench] dense PT: {d_step:.2f} ms/frame, {dense_mrays:.1f} Mrays/s")
        # random-position trilinear microbenchmark
        ns = 1 << 26
        g = torch.Generator(device="cuda").manual_seed(7)
        pos = (torch.rand((ns, 3), device="cuda", generator=g) * (n + 1.0) - 1.0).contiguous()
        out = torch.empty(ns, dtype=torch.float32, device="cuda")
        sv_ms = time_sampler(torch, lambda: vdbc.sample(grid, pos, 1, out), args.steps, 2)
        sd_ms = time_sampler(torch, lambda: vdbc.sample_dense(dense, 0.0, pos, 1, out),
                             args.steps, 2)
        extras = {
            "dense_mrays_per_s": round(dense_mrays, 3),
            "vdb_over_dense_mrays": round(vdb_mrays / dense_mrays, 4),
            "dense_ms_per_step": round(d_step, 4),
            "samples_per_s": {
                "vdb_render": round(samples / (pt_ms * 1e-3), 1),
                "dense_render": round(d_samples / (d_pt * 1e-3), 1),
                "vdb_sample_random_2^26": round(ns / (sv_ms * 1e-3), 1),
                "dense_sample_random_2^26": round(ns / (sd_ms * 1e-3), 1),
            },
            "random_sample_gbs": {
                "vdb": round(ns * BYTES_PER_RANDOM_SAMPLE / (sv_ms * 1e-3) / 1e9, 2),
                "dense": round(ns * BYTES_PER_RANDOM_SAMPLE / (sd_ms * 1e-3) / 1e9, 2),
            },
        }
        log(f"[bench] random samples/s: VDB {ns / (sv_ms * 1e-3) / 1e9:.2f} G, "
            f"dense {ns / (sd_ms * 1e-3) / 1e9:.2f} G")
        del pos, out
        # the HBM bandwidth a plain streaming copy reaches on this GPU (1 GiB
        # read + 1 GiB written per launch), next to the 8 TB/s datasheet figure
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        copy_ms = time_sampler(torch, lambda: y.copy_(x), 5, 2)
        extras["hbm_copy_gbs"] = round(2 * x.numel() * 4 / (copy_ms * 1e-3) / 1e9, 1)
        log(f"[bench] streaming copy: {extras['hbm_copy_gbs']:.0f} GB/s")
        del x, y

    cpu = None
    rel = None
    if not args.no_cpu_baseline:
        import oracle
        log(f"[bench] CPU oracle on {args.cpu_pixels} of {W * H} pixels")
        rng = np.random.default_rng(52)
        pix = np.sort(rng.choice(W * H, args.cpu_pixels, replace=False)).astype(np.uint32)
        fld = oracle.VdbField(buf)
        t = time.time()
        oracle.majorant(fld, med, C)
        t_maj = time.time() - t
        t = time.time()
        ref = oracle.render_pt(fld, cam, med, dict(spp=spp, max_bounces=bounces,
                                                   seed=M["seed"], macrocell=C), pixels=pix)
        t_all = time.time() - t
        t_paths = max(t_all - t_maj, 1e-9)
        frame_s = t_maj + t_paths * (W * H / len(pix))
        rel = relmse(img[pix], ref)
        cpu = {"value": round(rays / frame_s / 1e6, 6), "unit": "Mrays/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(pix)} random pixels x {spp} spp of the same frame "
                         f"({t_all:.1f}s incl. a {t_maj:.1f}s majorant build); frame time "
                         f"extrapolated as majorant + paths x {W * H}/{len(pix)}"}
        log(f"[bench] oracle {cpu['value']:.4f} Mrays/s; relMSE GPU vs oracle {rel:.3e}")
        if args.cpu_threads > 1:
            # the same oracle on every host core: disjoint pixel sets rendered
            # by concurrent calls (ctypes releases the GIL during each call)
            from concurrent.futures import ThreadPoolExecutor
            nt = args.cpu_threads
            pix_all = np.sort(rng.choice(W * H, args.cpu_pixels * nt, replace=False)).astype(np.uint32)
            parts = np.array_split(pix_all, nt)
            prm_o = dict(spp=spp, max_bounces=bounces, seed=M["seed"], macrocell=C)
            t = time.time()
            with ThreadPoolExecutor(max_workers=nt) as ex:
                list(ex.map(lambda pp: oracle.render_pt(fld, cam, med, prm_o, pixels=pp), parts))
            t_par = time.time() - t
            # each call also builds its own majorant (t_maj of work per thread)
            paths_s = max(t_par - t_maj, 1e-9)
            frame_par = t_maj + paths_s * (W * H / len(pix_all))
            cpu["all_cores"] = {
                "value": round(rays / frame_par / 1e6, 6), "unit": "Mrays/s", "cores": nt,
                "sample": f"{len(pix_all)} random pixels x {spp} spp in {nt} concurrent oracle calls "
                          f"({t_par:.1f}s); frame time extrapolated as majorant + paths x "
                          f"{W * H}/{len(pix_all)}"}
            log(f"[bench] oracle on {nt} threads: {cpu['all_cores']['value']:.3f} Mrays/s")

    pt_s = pt_ms * 1e-3
    prof = profile_values() if (args.rate == 0.10 and n == 512 and C == 16) else {}
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
            "workload": f"fbm-cloud-{n}^3-vdb-1:{round(1 / args.rate)}-pt-{W}x{H}x{spp}spp-"
                        f"{bounces}bounces",
            "dims": [n, n, n], "rate": args.rate, "width": W, "height": H, "spp": spp,
            "max_bounces": bounces, "macrocell": C,
            "vdb_bytes": int(buf.size), "dense_bytes": int(vol.nbytes),
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
                         "source": os.path.relpath(PROFILE, ROOT)} if prof else None),
            "per_launch": {"samples": int(samples), "bytes_per_sample": BYTES_PER_RENDER_SAMPLE,
                           "algorithmic_bytes": int(samples * BYTES_PER_RENDER_SAMPLE),
                           "avg_ms": round(pt_ms, 4)},
        },
        "cpu_baseline": cpu,
        "relmse_vs_oracle": rel,
        "encode_s": round(encode_s, 3),
        "upload_s": round(upload_s, 4),
        "majorant_ms": round(maj_ms, 4),
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
