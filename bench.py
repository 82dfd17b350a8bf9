"""Benchmark of the auto-labelling hot path on one MI355X.

Workload: one full Sentinel-2 tile, 10980 x 10980 pixels, 3 uint16
reflectance bands (B2, B3, B4) from the seeded generator (10 % haze, 5 %
shadow), cloud/shadow filter on, 256 x 256 chips, per-256 x 256-patch
class counts.  One step = one sil_label call = one kernel launch over the
whole tile, inputs resident in HBM.

Prints one JSON line (see the keys below).  ``roofline.achieved`` is the
algorithmic bytes of one launch (3 x 2 B in + 1 B label out per pixel + the
count array) over the kernel's mean duration, timed with HIP events on the
stream the kernel is launched on.  ``roofline.traffic`` is the HBM bytes per
launch from rocprofv3 FETCH_SIZE + WRITE_SIZE counters, scaled by the same
counters' reading for a plain copy of known size; it is read from
profiles/ and reported only while the kernel source is unchanged since the
counters were taken.  ``cpu_baseline`` is the C oracle, single-threaded, on
the same tile: the median of 3 runs, with the host's CPU model and core count.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H = W = 10980
PITCH = 10980
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_filter_tile10980_traffic.txt")
# the labeller kernel's sources: the kernel file and the headers it includes
KERNEL_SRCS = [os.path.join(ROOT, "paper_2403_13135_amd", "csrc", n)
               for n in ("sil.hip", "chip_walk.h", "rescale.h")]


def say(msg):
    """Progress line on stderr (long sections report as they go)."""
    print(f"# {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(H, W, ny, nx, in_bytes_per_px=6):
    return H * W * in_bytes_per_px + H * W + ny * nx * 3 * 4


def kernel_src_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """(bytes per launch, source hash) recorded from rocprofv3 counters, if current."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_src_sha256_16") != kernel_src_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def calib_copy(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    print(json.dumps({"calib_copy_bytes": nbytes, "read_plus_write_bytes": 2 * nbytes,
                      "ms": ms, "gbs": 2 * nbytes / ms / 1e6}), flush=True)


VARIANT_LIMITS = dict(lo=[[0, 40, 0], [20, 0, 60], [100, 10, 150]],
                      hi=[[90, 255, 120], [179, 200, 220], [170, 255, 255]])


def run_variants(sil, scene, H, W, stream, reps=20):
    """The general labeller (sil_label_ex) on the resident full tile: full-HSV
    limits with 256 x 256 chips, and the whole tile as one filter unit, with
    and without the filtered colour image.  Algorithmic bytes per pixel:
    pass A reads 6 and writes the 1-byte median, pass C reads 6 + 1 and
    writes the 1-byte mask (+ 3 colour bytes)."""
    import torch
    out = {}
    cases = [("full_hsv_chip256_rgb", dict(chip=256, **VARIANT_LIMITS), True),
             ("scene_level_rgb", dict(chip=1 << 20), True),
             ("scene_level_masks", dict(chip=1 << 20), False)]
    for name, kw, rgb in cases:
        p = sil.Params(dtype=sil.U16, **kw)
        ws = torch.empty((sil.workspace_bytes(H, W, p),), dtype=torch.uint8, device=scene.device)
        buf = sil.label_ex(scene, p, W=W, rgb=rgb, workspace=ws, stream=stream)
        for _ in range(3):
            sil.label_ex(scene, p, W=W, rgb=rgb, workspace=ws, out=buf, stream=stream)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            sil.label_ex(scene, p, W=W, rgb=rgb, workspace=ws, out=buf, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        bpp = 15 + (3 if rgb else 0)
        out[name] = {"ms": ms, "gpx_s": H * W / (ms / 1e3) / 1e9,
                     "algorithmic_bytes_per_px": bpp,
                     "achieved_gbs": H * W * bpp / (ms / 1e3) / 1e9}
        del ws, buf
    # the colour rendering of the class ids (1 byte in, 3 out per pixel)
    labels, _ = sil.label(scene, sil.Params(dtype=sil.U16), W=W, stream=stream)
    rgb = sil.render_rgb(labels, W=W, stream=stream)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        sil.render_rgb(labels, W=W, out=rgb, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    out["render_rgb"] = {"ms": ms, "gpx_s": H * W / (ms / 1e3) / 1e9,
                         "algorithmic_bytes_per_px": 4,
                         "achieved_gbs": H * W * 4 / (ms / 1e3) / 1e9}
    del labels, rgb
    return out


def run_serving(n_requests, chips_per_launch, seeds_per_size=4):
    """Continuous-batching server on the mixed-size request trace: capacity
    (all requests arriving at once), p50/p99 latency under Poisson arrivals at
    0.5 and 0.8 of capacity, and a bit-exactness pass in which every result
    is compared with its scene's solo sil_label output; every distinct pool
    scene's solo output is compared with the oracle (host threads).  The same
    trace with the scenes in page-locked host memory, copied into the
    server's arena at admission (PCIe included), is reported separately."""
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from oracle import sil_ref as R
    from paper_2403_13135_amd import serve, sil

    p = sil.Params(dtype=sil.U16)
    pool = serve.make_pool(seeds_per_size=seeds_per_size)
    refs = {}
    for size, items in pool.items():
        for i, (_, t) in enumerate(items):
            lab, hist = sil.label(t, p)
            refs[(size, i)] = (lab, hist)
    torch.cuda.synchronize()

    def oracle_check(key):
        size, i = key
        s_np = pool[size][i][1].cpu().numpy().view(np.uint16)
        ol, oh = R.label(s_np, R.make_params(dtype=R.U16))
        lab, hist = refs[key]
        return bool((lab.cpu().numpy() == ol).all()
                    and (hist.cpu().numpy().astype(np.uint32) == oh).all())

    keys = sorted(refs)
    say(f"serving: {len(keys)} pool scenes against the oracle")
    with ThreadPoolExecutor(max_workers=min(16, len(os.sched_getaffinity(0)))) as ex:
        oks = list(ex.map(oracle_check, keys))
    out = {"requests": n_requests, "sizes": list(serve.SIZES), "dtype": "u16",
           "scenes_per_size": seeds_per_size, "chips_per_launch": chips_per_launch,
           "pool_vs_oracle": f"{sum(oks)}/{len(oks)} pool scenes' solo results equal the oracle"}

    def play(rate, release, arena, src, n=n_requests):
        arr, picks = serve.make_trace(n, rate, pool, seed=11)
        scenes = [src[sz][k][1] for sz, k in picks]
        srv = serve.Server(p, arena_bytes=arena, max_chips_per_launch=chips_per_launch,
                           max_inflight=4, nstreams=2)
        comps, start = srv.run(scenes, arr, release=release)
        st = srv.stats()
        return srv, comps, start, arr, picks, st

    px = lambda picks: sum(sz * sz for sz, _ in picks)

    def trace(src, out, n_exact):
        say(f"serving trace of {n_requests} requests ({'host' if src is not pool else 'device'} scenes)")
        # capacity: every request present at t = 0
        srv, comps, start, arr, picks, st = play(0.0, True, 8 << 30, src)
        span = max(c.t_done_ms for c in comps) - start
        cap_req_per_ms = n_requests / span
        out["capacity"] = {"gpx_s": px(picks) / (span * 1e-3) / 1e9,
                           "requests_per_s": cap_req_per_ms * 1e3, "span_ms": span,
                           "launches": st["launches"], "arena_peak_bytes": st["arena_peak"]}
        srv.close()
        for rho in (0.5, 0.8):
            srv, comps, start, arr, picks, st = play(rho * cap_req_per_ms, True, 8 << 30, src)
            lat = np.array([c.t_done_ms - (start + a) for c, a in zip(comps, arr)])
            span = max(c.t_done_ms for c in comps) - start
            by_size = {}
            for (sz, _), l in zip(picks, lat):
                by_size.setdefault(sz, []).append(l)
            out[f"rho_{rho}"] = {
                "arrival_rate_per_s": rho * cap_req_per_ms * 1e3,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "throughput_gpx_s": px(picks) / (span * 1e-3) / 1e9, "launches": st["launches"],
                "arena_peak_bytes": st["arena_peak"],
                "p99_ms_by_size": {str(k): float(np.percentile(v, 99)) for k, v in by_size.items()}}
            srv.close()
        # bit-exactness: a burst with every output kept, each compared
        srv, comps, start, arr, picks, st = play(0.0, False, 80 << 30, src, n_exact)
        torch.cuda.synchronize()
        exact = 0
        for c, (sz, k) in zip(comps, picks):
            lab, hist = refs[(sz, k)]
            exact += int(torch.equal(c.labels(), lab) and torch.equal(c.hist(), hist))
            srv.release(c.tag)
        out["bit_exact"] = f"{exact}/{n_exact} results equal their scene's solo run"
        srv.close()

    trace(pool, out, n_requests)
    # the scenes in page-locked host memory: copied into the arena at admission
    host = {sz: [(seed, t.cpu().pin_memory()) for seed, t in items] for sz, items in pool.items()}
    out["host_scenes"] = {"note": "scenes in page-locked host memory, copied into the server's "
                                  "arena at admission (input bytes counted there)"}
    # (kept outputs and copied bands of 200 requests fit the exactness pass's arena)
    trace(host, out["host_scenes"], min(n_requests, 200))
    del host
    return out


def run_learned(steps, n_fallback, n_capacity, fb_batch, seeds_per_size):
    """U-Net (32-64-128-256) trained on GPU auto-labels at batch 32 of 256^2
    chips: step time and MFMA throughput, held-out accuracy against the
    synthetic truth beside the labeller.  Then serving with the labeller as
    fallback on the serving trace's mixed sizes: continuous batching of
    chips across requests (learn.serve_mix), capacity from a burst of
    `n_capacity` requests, Poisson arrivals at 0.5 and 0.8 of it."""
    import numpy as np
    import torch
    from paper_2403_13135_amd import learn, serve, unet

    widths = (32, 64, 128, 256)
    train_sc = learn.make_scenes(12, 2048, seed0=3000)
    test_sc = learn.make_scenes(3, 2048, seed0=4000)
    X, Y = learn.build_training_set(train_sc)
    model = unet.UNet(widths, seed=0)
    say(f"U-Net training, {steps} steps, each replaying one recorded HIP graph")
    losses, sec = learn.train(model, X, Y, steps=steps, batch=32, lr=1e-3, graph=True)
    flops_step = 3 * learn.unet_flops_per_image(widths) * 32
    ev = learn.evaluate(model, test_sc)
    # the same step launched eagerly, on a second model, for comparison
    say("U-Net training, 12 eager steps")
    _, sec_eager = learn.train(unet.UNet(widths, seed=0), X, Y, steps=12, batch=32, lr=1e-3)
    out = {"widths": list(widths), "batch": 32, "train_chips": int(X.shape[0]), "steps": steps,
           "step_ms": sec * 1e3, "images_per_s": 32 / sec,
           "tflops": flops_step / sec / 1e12,
           "mfma_frac_of_bf16_dense_peak": flops_step / sec / 2.5e15,
           "step_ms_eager_launches": sec_eager * 1e3,
           "loss_first_last": [losses[0], float(np.mean(losses[-10:]))], "held_out": ev}
    del X, Y, train_sc
    torch.cuda.empty_cache()
    if n_fallback <= 0:
        return out
    pool = serve.make_pool(seeds_per_size=seeds_per_size)
    infer_flops_px = learn.unet_flops_per_image(widths) / (learn.CHIP * learn.CHIP)

    def play(n, rate, seed):
        arr, picks = serve.make_trace(n, rate, pool, seed=seed)
        scenes = [pool[sz][k][1] for sz, k in picks]
        recs = learn.serve_mix(model, scenes, arr, threshold=0.02, batch=fb_batch,
                               progress=lambda d, m: say(f"serving with fallback: {d}/{m} served"))
        return recs, picks

    say("serving with fallback: capacity burst")
    res = {"requests": n_fallback, "sizes": list(serve.SIZES), "scenes_per_size": seeds_per_size,
           "threshold": 0.02, "chips_per_launch": fb_batch, "sequential": False}
    recs, picks = play(n_capacity, 0.0, 31)
    span = max(r.done_ms for r in recs)
    px = sum(r.H * r.W for r in recs)
    cap = n_capacity / span  # requests per ms
    res["capacity"] = {"requests": n_capacity, "span_ms": span, "gpx_s": px / (span * 1e-3) / 1e9,
                       "requests_per_s": cap * 1e3,
                       "unet_tflops": px * infer_flops_px / (span * 1e-3) / 1e12}
    for rho in (0.5, 0.8):
        say(f"serving with fallback: {n_fallback} requests at {rho} of capacity")
        recs, picks = play(n_fallback, rho * cap, 33)
        lat = np.array([r.done_ms - r.arrival_ms for r in recs])
        span = max(r.done_ms for r in recs)
        px = sum(r.H * r.W for r in recs)
        by_size = {}
        for (sz, _), l in zip(picks, lat):
            by_size.setdefault(sz, []).append(l)
        res[f"rho_{rho}"] = {
            "arrival_rate_per_s": rho * cap * 1e3, "span_ms": span,
            "throughput_gpx_s": px / (span * 1e-3) / 1e9,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "p99_ms_by_size": {str(k): float(np.percentile(v, 99)) for k, v in by_size.items()},
            "mean_mismatch_vs_labeller": float(np.mean([r.disagreement for r in recs])),
            "fallback_rate": float(np.mean([r.fallback for r in recs])),
            "fallback_rate_at_5pct": float(np.mean([r.disagreement > 0.05 for r in recs])),
            "fallback_rate_at_10pct": float(np.mean([r.disagreement > 0.10 for r in recs]))}
    out["serving_with_fallback"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the oracle CPU baseline")
    ap.add_argument("--pitch", type=int, default=PITCH)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a 1 GiB device copy (for counter scaling)")
    ap.add_argument("--skip-variants", action="store_true",
                    help="omit the general-labeller section")
    ap.add_argument("--skip-serving", action="store_true", help="omit the serving section")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--chips-per-launch", type=int, default=1024)
    ap.add_argument("--skip-learned", action="store_true", help="omit the U-Net section")
    ap.add_argument("--unet-steps", type=int, default=120)
    ap.add_argument("--fallback-requests", type=int, default=2000,
                    help="requests of the serving-with-fallback trace (0: skip)")
    ap.add_argument("--fallback-capacity-requests", type=int, default=200)
    ap.add_argument("--fallback-batch", type=int, default=128, help="chips per inference launch")
    ap.add_argument("--pool-seeds", type=int, default=4, help="scenes per size in the serving pools")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: labelling needs no cross-GPU step (a scene shards "
              "by chip rows with a one-row halo, and requests shard with no communication), "
              "and no multi-GPU path is built; use --gpus 1.",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calib_copy:
        calib_copy()
        return

    import synth
    from paper_2403_13135_amd import sil

    t_gen = time.time()
    spec = synth.config_tile(pitch=args.pitch)
    scene_np = synth.generate(spec)
    t_gen = time.time() - t_gen
    print(f"# generated {H}x{W} uint16 tile in {t_gen:.1f} s", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    scene = torch.from_numpy(scene_np.view(np.int16)).to(dev)
    params = sil.Params(dtype=sil.U16)
    ny, nx = sil.hist_dims(H, W, params)
    # label rows on 128-byte boundaries (pitch 11008 for the 10980-wide tile)
    labels = sil.alloc_labels(H, W, dev)
    hist = torch.empty((ny, nx, 3), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()

    def step():
        sil.label(scene, params, W=W, labels=labels, hist=hist, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K launches bracketed by events on the launch stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps

    # per-launch distribution (separate pass)
    per = []
    for _ in range(min(args.steps, 50)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step()
        b.record(stream)
        b.synchronize()
        per.append(a.elapsed_time(b))
    per.sort()

    npx = H * W
    gpx_s = npx * args.steps / (ms_total / 1e3) / 1e9
    alg = algorithmic_bytes(H, W, ny, nx)
    achieved = alg / (ms_per_step / 1e3) / 1e9
    traffic = read_traffic()

    # measured device-to-device copy bandwidth: practical ceiling on this machine
    nb = 1 << 30
    ca = torch.empty(nb, dtype=torch.uint8, device=dev)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        cb.copy_(ca)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nb * 5 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del ca, cb

    # thresholds-only mode (the paper's unfiltered segmentation) on the same tile
    p0 = sil.Params(dtype=sil.U16, filter=0)
    labels0 = sil.alloc_labels(H, W, dev)
    hist0 = torch.empty_like(hist)
    for _ in range(3):
        sil.label(scene, p0, W=W, labels=labels0, hist=hist0, stream=stream)
    f0a = torch.cuda.Event(enable_timing=True)
    f0b = torch.cuda.Event(enable_timing=True)
    f0a.record(stream)
    for _ in range(20):
        sil.label(scene, p0, W=W, labels=labels0, hist=hist0, stream=stream)
    f0b.record(stream)
    torch.cuda.synchronize()
    f0_ms = f0a.elapsed_time(f0b) / 20

    cpu = None
    if not args.skip_cpu:
        say("CPU baseline: the oracle on the tile, 3 runs")
        from oracle import sil_ref as R
        times, ok = [], True
        for _ in range(3):
            t = time.perf_counter()
            ol, oh = R.label(scene_np, R.make_params(dtype=R.U16), W=W)
            times.append(time.perf_counter() - t)
            ok = ok and bool((labels.cpu().numpy() == ol).all()
                             and (hist.cpu().numpy().astype(np.uint32) == oh).all())
        dt = statistics.median(times)
        cpu = {"value": npx / dt / 1e9, "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
               "sample": f"the full {H}x{W} uint16 tile, single-threaded C oracle, median of "
                         f"3 runs ({', '.join(f'{t:.2f}' for t in times)} s); GPU output "
                         f"bit-identical: {ok}",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "cores_available": len(os.sched_getaffinity(0))}

    variants = None
    if not args.skip_variants:
        variants = run_variants(sil, scene, H, W, stream)

    serving = None
    if not args.skip_serving:
        del scene, labels, hist, labels0, hist0
        torch.cuda.empty_cache()
        serving = run_serving(args.serving_requests, args.chips_per_launch, args.pool_seeds)
    learned = None
    if not args.skip_learned:
        torch.cuda.empty_cache()
        learned = run_learned(args.unet_steps, args.fallback_requests,
                              args.fallback_capacity_requests, args.fallback_batch, args.pool_seeds)

    out = {
        "metric": "auto-labelled Gpixel/s",
        "value": gpx_s,
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": f"full-tile labelling, {H}x{W} uint16 x 3 bands "
                               f"(pitch {args.pitch}), cloud/shadow filter on, chip 256, "
                               f"per-256x256-patch counts, label rows "
                               f"{sil.label_pitch_for(W)} bytes apart",
                   "global_batch": 1, "pixels_per_step": npx, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "extra": {
            "kernel": "k_filter<uint16_t, vec, fast24>",
            "algorithmic_bytes_per_launch": alg,
            "launch_ms_p10_p50_p90": [per[len(per) // 10], statistics.median(per),
                                      per[(9 * len(per)) // 10]],
            "device_copy_gbs": copy_gbs,
            "frac_of_device_copy": achieved / copy_gbs,
            "thresholds_only_ms": f0_ms,
            "thresholds_only_gpx_s": npx / (f0_ms / 1e3) / 1e9,
            "wall_s_timed_region": wall,
        },
        "variants": variants,
        "serving": serving,
        "learned": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
