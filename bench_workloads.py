"""Secondary measurements of bench.py: the paper-scale rate sweep, the
learned denoiser and the batched multi-volume launch.  Each returns one JSON
object (printed by bench.py)."""
from __future__ import annotations

import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def _median_ms(torch, fn, reps, warmup=1):
    for _ in range(warmup):
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


def sweep(args, torch, vdbc, synth, scenes, log):
    """1987x1351x2449 billowed cloud (26.3 GB): encode at 1:20..1:4, path
    trace 1920x1080 at 64 spp with <= 16 bounces from every VDB and from the
    dense array on the same GPU."""
    P = scenes.PAPER
    nx, ny, nz = P["dims"]
    t = time.time()
    vol = synth.paper_volume(dims=P["dims"])
    log(f"[paper] volume {vol.nbytes / 1e9:.1f} GB in {time.time() - t:.0f}s")
    W, H, spp, bounces = P["width"], P["height"], P["spp"], P["max_bounces"]
    C = args.macrocell
    cam = scenes.orbit_camera((nx, ny, nz), W, H)
    med = scenes.pt_medium(64.0)
    # timed without the counters; samples from one more counting launch
    prm = dict(spp=spp, max_bounces=bounces, seed=P["seed"], macrocell=C, tile_w=args.tile_w,
               chunk_spp=args.chunk_spp, flags=args.order_flag)
    rays = W * H * spp

    def samples_of(field, **kw):
        rc = vdbc.Renderer(field, cam, med, dict(prm, flags=vdbc.RENDER_COUNT), vdbc.MODE_PT, **kw)
        rc.launch()
        torch.cuda.synchronize()
        return rc.sample_count()

    out = {"metric": "paper-scale VDB vs dense path-traced Mrays/s", "unit": "Mrays/s",
           "config": {"workload": "fbm-cloud-1987x1351x2449-pt-1920x1080x64spp-16bounces",
                      "dims": list(P["dims"]), "macrocell": C, "tile_w": args.tile_w,
                      "chunk_spp": args.chunk_spp}, "rates": []}
    for q in P["rates"]:
        t = time.time()
        buf, st = vdbc.encode(vol, q)
        enc = time.time() - t
        g = vdbc.Grid(buf)
        r = vdbc.Renderer(g, cam, med, prm, vdbc.MODE_PT)
        ms = _median_ms(torch, r.launch, 3)
        rec = {"rate": q, "encode_s": round(enc, 2), "vdb_bytes": int(buf.size),
               "achieved_rate": round(st["achieved_rate"], 5), "ms": round(ms, 2),
               "mrays_per_s": round(rays / ms / 1e3, 2),
               "samples_per_s": round(samples_of(g) / ms * 1e3, 1)}
        log(f"[paper] q={q}: {rec}")
        out["rates"].append(rec)
        del r, g, buf
        torch.cuda.empty_cache()
    t = time.time()
    dense = torch.from_numpy(vol).cuda()
    log(f"[paper] dense upload {time.time() - t:.1f}s")
    r = vdbc.Renderer(dense, cam, med, prm, vdbc.MODE_PT, background=0.0)
    ms = _median_ms(torch, r.launch, 3)
    out["dense"] = {"ms": round(ms, 2), "mrays_per_s": round(rays / ms / 1e3, 2),
                    "samples_per_s": round(samples_of(dense, background=0.0) / ms * 1e3, 1),
                    "bytes": int(vol.nbytes)}
    ten = [x for x in out["rates"] if abs(x["rate"] - 0.10) < 1e-9][0]
    out["value"] = ten["mrays_per_s"]
    out["vdb_over_dense_at_1:10"] = round(ten["mrays_per_s"] / out["dense"]["mrays_per_s"], 4)
    log(f"[paper] dense {out['dense']}")
    return out


def denoiser(args, torch, vdbc, synth, scenes, log):
    """Learned denoiser: training pairs rendered from seeded clouds at 1:10
    (4-spp input with AOVs, high-spp target), training with the library's
    BF16-MFMA step, evaluation on held-out clouds against a 1024-spp
    reference."""
    from paper_2504_04564_amd import denoiser as dz
    rng = np.random.default_rng(1000)
    part = args.denoiser_part
    vols = None
    if args.denoiser_full:
        # the recipe's crops (512^2 from 256^3..512^3 clouds, 1024-spp targets).
        # Rendering its 2,000 crops takes ~26 min of GPU time at 0.77 s per
        # crop, beyond one 20-minute run: --denoiser-part 1 renders the crops
        # of volumes 0..49, trains and writes a checkpoint (parameters, Adam
        # moments, step); --denoiser-part 2 resumes from it with the crops of
        # volumes 50..99
        n_vol, views, size, spp_tgt, lo, hi = 100 if part else 50, 20, 512, 1024, 256, 512
        if part:
            vols = range(0, 50) if part == 1 else range(50, 100)
    else:
        n_vol, views, size, spp_tgt, lo, hi = 16, 6, 256, 512, 128, 256
    if vols is None:
        vols = range(n_vol)
    spp_in = 4
    med = scenes.pt_medium(64.0)
    xs, ts = [], []
    t = time.time()
    sides = [int(rng.integers(lo, hi + 1)) for _ in range(n_vol)]
    # camera draws per volume, so a part renders the same crops as a full run
    cam_rng = {i: np.random.default_rng([1000, i]) for i in vols} if part else None

    def make(i):
        # host side of one training volume: generate and encode (overlaps the
        # GPU renders of the previous volume)
        v = synth.cloud_volume((sides[i], sides[i], sides[i]), seed=1000 + i)
        return vdbc.encode(v, 0.10)[0]

    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=2)
    order = list(vols)
    pending = [pool.submit(make, i) for i in order[:2]]
    for j, i in enumerate(order):
        if args.denoiser_full and j % 5 == 0:
            log(f"[denoiser] volume {i} ({j}/{len(order)}), {len(xs)} crops, {time.time() - t:.0f}s")
        buf = pending.pop(0).result()
        if j + 2 < len(order):
            pending.append(pool.submit(make, order[j + 2]))
        g = vdbc.Grid(buf)
        r = cam_rng[i] if cam_rng else rng
        for k in range(views):
            cam = scenes.orbit_camera(g.dims, size, size, azimuth_deg=float(r.uniform(0, 360)),
                                      elevation_deg=float(r.uniform(-30, 45)),
                                      distance=float(r.uniform(1.2, 2.0)))
            x, ref = dz.render_pair(g, cam, med, spp_in, spp_tgt, seed=7919 * i + k)
            xs.append(x)
            ts.append(ref)
    pool.shutdown()
    torch.cuda.synchronize()
    gen_s = time.time() - t
    X = torch.stack(xs)
    T = torch.stack(ts)
    log(f"[denoiser] {X.shape[0]} training crops of {size}^2 in {gen_s:.1f}s")
    steps, batch = args.train_steps, 8
    if part == 2:
        ck = np.load(args.denoiser_ckpt)
        dn = vdbc.Denoiser(params=ck["params"])
        dn.m.copy_(torch.from_numpy(ck["m"]))
        dn.v.copy_(torch.from_numpy(ck["v"]))
        dn.step = int(ck["step"])
        log(f"[denoiser] resumed from {args.denoiser_ckpt} at step {dn.step}")
    else:
        dn = vdbc.Denoiser(seed=5)
    t = time.time()
    losses = dz.train(dn, X, T, steps=steps, batch=batch, lr=1e-3, seed=part or 1, log_every=200)
    torch.cuda.synchronize()
    train_s = time.time() - t
    if part == 1:
        np.savez(args.denoiser_ckpt, params=dn.params.cpu().numpy(), m=dn.m.cpu().numpy(),
                 v=dn.v.cpu().numpy(), step=dn.step)
        log(f"[denoiser] checkpoint at step {dn.step} written to {args.denoiser_ckpt}")
    del X, T, xs, ts
    evals = []
    for j in range(3):
        side = 384
        v = synth.cloud_volume((side, side, side), seed=5000 + j)
        buf, _ = vdbc.encode(v, 0.10)
        g = vdbc.Grid(buf)
        cam = scenes.orbit_camera(g.dims, 512, 512, azimuth_deg=40.0 + 90 * j)
        evals.append(dz.evaluate(dn, g, cam, med, seed=31 + j))
        log(f"[denoiser] eval {j}: {evals[-1]}")
    keys = ("relmse_plain_lo", "relmse_plain_hi", "relmse_denoised", "ms_plain_hi",
            "ms_denoised_pipeline")
    mean = {k: float(np.mean([e[k] for e in evals])) for k in keys}
    return {"metric": "denoised 4-spp relMSE vs plain 64-spp relMSE (1024-spp reference)",
            "value": mean["relmse_denoised"], "unit": "relMSE", "higher_is_better": False,
            "config": {"workload": f"{len(order)}x{views} crops {size}^2 of {lo}^3..{hi}^3 clouds at 1:10,"
                                   f" targets {spp_tgt} spp, eval 3 clouds 384^3 at 512^2",
                       "train_steps": steps, "batch": batch, "lr": 1e-3,
                       "part": part, "volumes": [order[0], order[-1]],
                       "total_steps": dn.step},
            "train_s": round(train_s, 2), "gen_s": round(gen_s, 2),
            "ms_per_train_step": round(train_s / steps * 1e3, 3),
            "loss_first": float(losses[0]), "loss_last": float(np.mean(losses[-20:])),
            "mean": mean, "evals": evals}


def batch(args, torch, vdbc, synth, scenes, log):
    """64 volumes, sides log-uniform in [32, 768], rates from {1:4, 1:6,
    1:10, 1:20}, 256x256 images with 1-8 spp: per-volume launches vs one
    persistent launch vs graph replay, with the autotuned tuning."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2504_04564_amd import autotune
    specs = synth.batch_sizes(64, seed=7)
    t = time.time()

    def make(i):
        side, q, spp = specs[i]
        v = synth.cloud_volume((side, side, side), seed=7000 + i)
        buf, _ = vdbc.encode(v, q, threads=1)
        return buf, v.nbytes

    with ThreadPoolExecutor(max_workers=16) as ex:
        made = list(ex.map(make, range(len(specs))))
    log(f"[batch] 64 volumes generated and encoded in {time.time() - t:.0f}s, "
        f"dense total {sum(m[1] for m in made) / 1e9:.1f} GB")
    med = scenes.pt_medium(64.0)
    items = []
    for i, ((buf, _), (side, q, spp)) in enumerate(zip(made, specs)):
        g = vdbc.Grid(buf)
        items.append(dict(grid=g, camera=scenes.orbit_camera(g.dims, 256, 256, azimuth_deg=7.0 * i),
                          medium=med, spp=spp, max_bounces=8, seed=0xB00 + i, frame=0))
    rays = sum(256 * 256 * it["spp"] for it in items)
    best, allr = autotune.tune_batch(items, autotune.BATCH_SPACE, reps=3)
    log(f"[batch] tuned: {best}")
    t_best = dict(best)
    t_best.pop("ms")
    per = vdbc.Batch(items, dict(t_best, persistent=0))
    ms_per = _median_ms(torch, per.launch, 5)
    pers = vdbc.Batch(items, dict(t_best, persistent=1))
    ms_pers = _median_ms(torch, pers.launch, 5)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    pers.capture(s)

    def replay():
        with torch.cuda.stream(s):
            pers.replay()
        s.synchronize()

    ms_graph = _median_ms(torch, replay, 5)
    same = all(torch.equal(a.view(torch.int32), b.view(torch.int32))
               for a, b in zip(per.images, pers.images))
    return {"metric": "batched multi-volume path-traced Mrays/s", "unit": "Mrays/s",
            "value": round(rays / ms_graph / 1e3, 2),
            "config": {"workload": "64 fbm clouds 32^3-768^3, rates 1:4..1:20, 256x256, 1-8 spp",
                       "tuning": t_best},
            "ms_per_volume_launches": round(ms_per, 3), "ms_persistent": round(ms_pers, 3),
            "ms_graph_replay": round(ms_graph, 3),
            "mrays_per_volume_launches": round(rays / ms_per / 1e3, 2),
            "images_bit_identical": bool(same), "tuning_candidates": allr}


def quality(args, torch, vdbc, synth, scenes, log):
    """Compression error against the dense original (Section 5.2): MSE and
    PSNR of the 512^3 cloud at rates 10 %..100 % for the three similarity
    metrics (tab:stats and fig:distance on the synthetic stand-in)."""
    n = args.size
    vol = synth.mid_volume(n=n)
    dense = torch.from_numpy(vol).cuda()
    names = {1: "closest", 2: "farthest", 3: "median"}
    rows = []
    for metric in (1, 2, 3):
        for q in [round(0.1 * k, 1) for k in range(1, 11)]:
            buf, st = vdbc.encode(vol, q, metric=metric)
            g = vdbc.Grid(buf)
            ms = _median_ms(torch, lambda: vdbc.compare_dense(g, dense), 3)
            c = vdbc.compare_dense(g, dense)
            rec = {"metric": names[metric], "rate": q, "mse": c["mse"], "psnr": c["psnr"],
                   "max_abs": c["max_abs"], "differing_voxels": c["differing"],
                   "vdb_bytes": int(buf.size), "achieved_rate": round(st["achieved_rate"], 5),
                   "compare_ms": round(ms, 3)}
            log(f"[quality] {rec}")
            rows.append(rec)
            del g
    lossless = {names[m]: min([r["rate"] for r in rows if r["metric"] == names[m] and r["differing_voxels"] == 0],
                              default=None) for m in (1, 2, 3)}
    # partial-brick activation (Section 3.2.1 future work) at the same voxel
    # budget: bricks below the similarity of the brick ranked K/2 (or every
    # brick) keep a fraction p of their most dissimilar voxels
    partial_rows = []
    lo, hi = [], []
    for q in (0.05, 0.1, 0.2, 0.3):
        buf0, st0 = vdbc.encode(vol, q)
        plain = vdbc.compare_dense(vdbc.Grid(buf0), dense)
        K = int(st0["k_bricks"])
        # similarity (Eq. 2) of the brick ranked K/2, from the brick ranges
        nz_, ny_, nx_ = vol.shape
        if not lo:
            for bz in range(0, nz_, 32):
                for by in range(0, ny_, 32):
                    for bx in range(0, nx_, 32):
                        blk = vol[bz:bz + 32, by:by + 32, bx:bx + 32]
                        lo.append(float(blk.min()))
                        hi.append(float(blk.max()))
        B = float(st0["background"])
        f = np.sort(np.maximum(np.abs(np.array(lo) - B), np.abs(np.array(hi) - B)))[::-1]
        for p, tau_name, tau in ((0.5, "all", 1e30), (0.25, "all", 1e30),
                                 (0.5, "rank K/2", float(f[K // 2]) if K else 1e30)):
            buf, st = vdbc.encode(vol, q, partial=(p, tau))
            c = vdbc.compare_dense(vdbc.Grid(buf), dense)
            rec = {"rate": q, "fraction": p, "partial_from": tau_name, "mse": c["mse"],
                   "psnr": c["psnr"], "plain_psnr": plain["psnr"], "vdb_bytes": int(buf.size),
                   "plain_bytes": int(buf0.size), "achieved_rate": round(st["achieved_rate"], 5)}
            log(f"[quality] partial {rec}")
            partial_rows.append(rec)
    return {"metric": "MSE / PSNR of the compressed cloud vs the dense original", "unit": "dB",
            "value": [r for r in rows if r["metric"] == "farthest" and r["rate"] == 0.1][0]["psnr"],
            "config": {"workload": f"fbm-cloud-{n}^3-rates-0.1..1.0-metrics-f1f2f3",
                       "psnr_peak": "max - min of the dense volume"},
            "lowest_lossless_rate": lossless, "rows": rows, "partial_rows": partial_rows}


def worstcase(args, torch, vdbc, synth, scenes, log):
    """Lossless encoding of truly dense noise, 32^3 up to --worst-max^3
    (tab:worstcase): bytes of the VDB and of the dense array, path-traced
    frame rate of both on the same GPU, and whether the images agree
    bitwise (they must at 1:1)."""
    rows = []
    W = H = 1024
    spp, bounces = 4, 8
    med = scenes.pt_medium(64.0)
    n = 32
    while n <= args.worst_max:
        t = time.time()
        vol = synth.dense_noise(n, seed=n)
        log(f"[worstcase] {n}^3 generated in {time.time() - t:.1f}s, encoding")
        t = time.time()
        if n >= 2048:
            # white noise has no dominant value: the exact mode of 8.6e9
            # values would need a 34 GB sort, and at 1:1 every voxel is kept
            # whatever the background, so it is given (0) instead
            buf, st = vdbc.encode(vol, 1.0, flags=vdbc.BG_EXPLICIT, background=0.0)
        else:
            buf, st = vdbc.encode(vol, 1.0)
        enc = time.time() - t
        g = vdbc.Grid(buf)
        dense = torch.from_numpy(vol).cuda()
        del vol
        cam = scenes.orbit_camera((n, n, n), W, H)
        prm = dict(spp=spp, max_bounces=bounces, seed=0x5EED, macrocell=args.macrocell)
        rv = vdbc.Renderer(g, cam, med, prm, vdbc.MODE_PT)
        rd = vdbc.Renderer(dense, cam, med, prm, vdbc.MODE_PT, background=g.background)
        ms_v = _median_ms(torch, rv.launch, 3)
        ms_d = _median_ms(torch, rd.launch, 3)
        same = bool(torch.equal(rv.image.view(torch.int32), rd.image.view(torch.int32)))
        rec = {"n": n, "dense_bytes": n ** 3 * 4, "vdb_bytes": int(buf.size),
               "background": "explicit 0" if n >= 2048 else "exact mode",
               "overhead": round(buf.size / (n ** 3 * 4) - 1.0, 5), "encode_s": round(enc, 2),
               "vdb_fps": round(1e3 / ms_v, 2), "dense_fps": round(1e3 / ms_d, 2),
               "vdb_over_dense": round(ms_d / ms_v, 4), "images_bitwise_equal": same}
        log(f"[worstcase] {rec}")
        rows.append(rec)
        del rv, rd, g, dense, buf
        torch.cuda.empty_cache()
        n *= 2
    return {"metric": "worst case: lossless dense noise, VDB vs dense bytes and frame rate",
            "unit": "fps", "value": rows[-1]["vdb_fps"],
            "config": {"workload": f"dense-noise-32^3..{args.worst_max}^3-1to1-pt-{W}x{H}x{spp}spp-{bounces}bounces",
                       "macrocell": args.macrocell},
            "rows": rows}


def iso(args, torch, vdbc, synth, scenes, log):
    """Iso-surface marcher at iso 0.5 (Section 5.4) on the 512^3 cloud at
    1:10 and on the dense array: frame time and samples/s, with and without
    empty-node skipping (VDB only), 1024x1024, step 0.5, 12 bisection steps."""
    n = args.size
    vol = synth.mid_volume(n=n)
    buf, st = vdbc.encode(vol, args.rate)
    g = vdbc.Grid(buf)
    dense = torch.from_numpy(vol).cuda()
    W = H = 1024
    cam = scenes.orbit_camera((n, n, n), W, H)
    base = dict(step=0.5, iso=0.5, refine=12)
    rows = {}
    for name, field, flags, bg in (("vdb", g, 0, None), ("vdb_hdda", g, vdbc.RENDER_HDDA, None),
                                   ("dense", dense, 0, 0.0)):
        r = vdbc.Renderer(field, cam, None, dict(base, flags=flags | vdbc.RENDER_COUNT),
                          vdbc.MODE_ISO, background=bg)
        ms = _median_ms(torch, r.launch, 5)
        rows[name] = {"ms": round(ms, 3), "fps": round(1e3 / ms, 2),
                      "samples_per_s": round(r.sample_count() / ms * 1e3, 1),
                      "hits": int((r.image[..., 3] == 1.0).sum().item())}
        log(f"[iso] {name}: {rows[name]}")
    best = min(("vdb", "vdb_hdda"), key=lambda k: rows[k]["ms"])
    return {"metric": "iso-surface frames/s, VDB (1:10) vs dense", "unit": "fps",
            "value": rows[best]["fps"],
            "config": {"workload": f"fbm-cloud-{n}^3-1to10-iso0.5-{W}x{H}-step0.5-refine12",
                       "vdb_variant": best},
            "vdb_over_dense": round(rows["dense"]["ms"] / rows[best]["ms"], 4), "rows": rows}


def ea(args, torch, vdbc, synth, scenes, log):
    """Emission-absorption ray marching (step 0.5 voxel, no early termination)
    of the 512^3 cloud at 1:10 and of the dense array, 1024x1024, with and
    without empty-node skipping (VDB only)."""
    n = args.size
    vol = synth.mid_volume(n=n)
    buf, st = vdbc.encode(vol, args.rate)
    g = vdbc.Grid(buf)
    dense = torch.from_numpy(vol).cuda()
    W = H = 1024
    cam = scenes.orbit_camera((n, n, n), W, H)
    med = scenes.ea_medium(8.0)
    base = dict(step=0.5, t_terminate=0.0)
    rows = {}
    for name, field, flags, bg in (("vdb", g, 0, None), ("vdb_hdda", g, vdbc.RENDER_HDDA, None),
                                   ("dense", dense, 0, 0.0)):
        r = vdbc.Renderer(field, cam, med, dict(base, flags=flags | vdbc.RENDER_COUNT),
                          vdbc.MODE_EA, background=bg)
        ms = _median_ms(torch, r.launch, 5)
        rows[name] = {"ms": round(ms, 3), "fps": round(1e3 / ms, 2),
                      "samples": r.sample_count(),
                      "samples_per_s": round(r.sample_count() / ms * 1e3, 1),
                      "gbs_at_32B_per_sample": round(r.sample_count() * 32 / ms / 1e6, 1)}
        log(f"[ea] {name}: {rows[name]}")
    best = min(("vdb", "vdb_hdda"), key=lambda k: rows[k]["ms"])
    return {"metric": "emission-absorption frames/s, VDB (1:10) vs dense", "unit": "fps",
            "value": rows[best]["fps"],
            "config": {"workload": f"fbm-cloud-{n}^3-1to10-ea-{W}x{H}-step0.5", "vdb_variant": best},
            "vdb_over_dense": round(rows["dense"]["ms"] / rows[best]["ms"], 4), "rows": rows}


def tune(args, torch, vdbc, synth, scenes, log):
    """The render autotuner on a headline frame: every (macrocell, wave tile,
    accessor cache policy, samples per work item) candidate timed, the
    fastest kept.  --tune-frame
    mid: the 512^3 cloud at 1:10, 1024^2 x 16 spp, <= 8 bounces; paper: the
    1987x1351x2449 cloud at 1:10, 1920x1080 x 64 spp, <= 16 bounces."""
    from paper_2504_04564_amd import autotune
    if args.tune_frame == "paper":
        S = scenes.PAPER
        dims = S["dims"]
        vol = synth.paper_volume(dims=dims)
        name = f"fbm-cloud-{dims[0]}x{dims[1]}x{dims[2]}-billowed"
    else:
        S = scenes.MID
        n = args.size
        dims = (n, n, n)
        vol = synth.mid_volume(n=n)
        name = f"fbm-cloud-{n}^3"
    buf, _ = vdbc.encode(vol, args.rate)
    del vol
    g = vdbc.Grid(buf)
    cam = scenes.orbit_camera(dims, S["width"], S["height"])
    med = scenes.pt_medium(64.0)
    prm = dict(spp=S["spp"], max_bounces=S["max_bounces"], seed=S["seed"])
    rows = []
    for C_ in autotune.RENDER_SPACE["macrocell"]:   # one cell size at a time, with progress
        _, part = autotune.tune_render(g, cam, med, prm, space=dict(macrocell=(C_,)), reps=5)
        rows += part
        log(f"[tune] macrocell {C_}: best {min(part, key=lambda x: x['ms'])}")
    best = min(rows, key=lambda x: x["ms"])
    for r in sorted(rows, key=lambda x: x["ms"]):
        log(f"[tune] {r}")
    return {"metric": "render autotuner: fastest PT launch configuration", "unit": "ms",
            "value": round(best["ms"], 3), "higher_is_better": False,
            "config": {"workload": f"{name}-1to{round(1 / args.rate)}-pt-{S['width']}x{S['height']}x"
                                   f"{S['spp']}spp-{S['max_bounces']}bounces",
                       "space": {k: list(v) for k, v in autotune.RENDER_SPACE.items()}},
            "best": best, "candidates": rows}
