"""Benchmark: lost processing blocks per second of Frequency Selective
Extrapolation on one MI355X.

Workload: 1920x1080 synthetic luma requests, 25 % of the 4x4 blocks lost
plus 1 % isolated defect pixels, 32x32 support and DFT, K = 100, rho = 0.8,
gamma = 0.5, recon weight 0.5, FP64 arithmetic, exact raster semantics per
request.

A step is one batched extrapolation of ``--batch`` requests on inputs already
resident in HBM: host planning of every request's blocks and dependency
order, upload of the plan, and one persistent dependency-driven kernel that
runs the blocks of all requests.  ``value`` = processing blocks per second
over the timed steps (default twelve), which rotate over ``--streams``
streams (default four) so that the host planning of one batch and the
launches of the batches before it overlap; the timed region starts and ends
with an idle device, so it includes the filling and draining of that
pipeline.  The outputs are checked bitwise against steps run one at a time.  The roofline, the kernel time and the step latencies come from
those one-at-a-time steps (a launch alone on the device).  Also reported:
one request alone, the paper's tile framework on one request, the tile-border
and tiling comparisons, the 3840x2160 tiled batch, FP32 and BF16x3 against
FP64, served Poisson streams (continuous batching, p50/p99 latency), the
plain GPU path (one kernel launch per block, raster order; bitwise-identical
output), and the FP64 CPU oracle on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import itertools
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_FP64_VECTOR_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def progress(msg: str) -> None:
    """One line per finished part of the run, on stderr (the JSON result is the
    only line on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def block_flops(M: int, K: int, B: int) -> float:
    """Algorithmic FP64 flops of one processing block.

    DFT of the two real inputs (w*s and w) as F X F with real GEMMs:
    stage 1 two real M^3 products per input, stage 2 four: 12 M^3 MACs =
    24 M^3 flops.  Each of the K steps updates M^2 complex residuals
    (4 FMA = 8 flops) and forms their energy (mul + fma = 3 flops).
    Synthesis: B^2 pixels x K terms x 2 FMA.
    """
    return 24.0 * M ** 3 + K * M * M * 11.0 + B * B * K * 4.0


def ssim(x, ref) -> float:
    """Mean structural similarity of image x (clipped to [0, 255]) against ref
    (Wang et al. 2004: Gaussian window of sigma 1.5 over 11 x 11 pixels,
    K1 = 0.01, K2 = 0.03, L = 255), the paper's second quality measure."""
    import numpy as np
    from scipy.ndimage import gaussian_filter

    a = np.clip(np.asarray(x, np.float64), 0, 255)
    b = np.asarray(ref, np.float64)

    def f(v):
        return gaussian_filter(v, 1.5, truncate=3.5)

    mu_a, mu_b = f(a), f(b)
    s_aa = f(a * a) - mu_a * mu_a
    s_bb = f(b * b) - mu_b * mu_b
    s_ab = f(a * b) - mu_a * mu_b
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    m = ((2 * mu_a * mu_b + c1) * (2 * s_ab + c2)) / ((mu_a * mu_a + mu_b * mu_b + c1) * (s_aa + s_bb + c2))
    return float(m.mean())


def kernel_source_hash() -> str:
    src = os.path.join(ROOT, "paper_2207_00238_amd", "csrc", "fse_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_from_profiles(workload: str, n_launch_units: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_fse_blocks_{workload}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def phases_from_profiles(workload: str):
    """Per-phase roofline figures of the block kernel from the committed
    rocprofv3 summaries (the DFT phase from a K = 0 launch with MFMA
    counters, the selection loop's LDS and VALU figures from the counters of
    the K = 100 launch), when they were taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"phases_fse_blocks_{workload}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return {k: rec[k] for k in ("dft_phase", "loop", "optimized_order_batch", "profiles") if k in rec}


def end_to_end_with_copies(fse, torch, imgs, msks, outs, params, stream, n_blocks, steps):
    """The batched step with its inputs coming from pinned host memory and its
    outputs going back to it: per step, the images and masks are copied to the
    device, the batch runs, and the outputs are copied back, all on one stream,
    one step at a time.  The headline value keeps its inputs resident in HBM;
    this is the rate over PCIe."""
    h_img = [torch.empty(t.shape, dtype=t.dtype, pin_memory=True) for t in imgs]
    h_msk = [torch.empty(t.shape, dtype=t.dtype, pin_memory=True) for t in msks]
    h_out = [torch.empty(t.shape, dtype=t.dtype, pin_memory=True) for t in outs]
    for h, d in zip(h_img + h_msk, imgs + msks):
        h.copy_(d)
    nbytes_in = sum(t.numel() * t.element_size() for t in imgs + msks)
    nbytes_out = sum(t.numel() * t.element_size() for t in outs)

    def copy_in():
        for h, d in zip(h_img + h_msk, imgs + msks):
            d.copy_(h, non_blocking=True)

    def copy_out():
        for h, d in zip(h_out, outs):
            h.copy_(d, non_blocking=True)

    with torch.cuda.stream(stream):
        # copies alone, timed with events on the step's stream
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        copy_in()
        torch.cuda.synchronize()
        ev[0].record(stream)
        copy_in()
        ev[1].record(stream)
        copy_out()
        ev[2].record(stream)
        torch.cuda.synchronize()
        h2d_ms, d2h_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        t0 = time.perf_counter()
        for _ in range(steps):
            copy_in()
            fse.fse_extrapolate_batch(imgs, msks, params, outs, stream)
            copy_out()
            stream.synchronize()
        dt = (time.perf_counter() - t0) / steps
    return {"value": n_blocks / dt, "unit": "blocks/s", "ms_per_step": dt * 1e3, "h2d_ms": h2d_ms,
            "d2h_ms": d2h_ms, "h2d_gb_per_s": nbytes_in / h2d_ms / 1e6, "d2h_gb_per_s": nbytes_out / d2h_ms / 1e6,
            "note": "one step at a time; images and masks from pinned host memory, outputs back to it"}


def cpu_baseline():
    """The FP64 oracle, single thread, on the top-left 1280x720 crop of the
    workload's first image and mask (the crop is processed as an image of its
    own)."""
    import numpy as np

    from oracle import oracle
    from paper_2207_00238_amd import synth

    wl = synth.workload("hd")
    crop = (720, 1280)
    img = wl.image[:crop[0], :crop[1]]
    msk = wl.mask[:crop[0], :crop[1]]
    nb = len(oracle.plan(msk, wl.classes)[0])
    t0 = time.perf_counter()
    ref = oracle.image(img, msk, wl.classes, rho=wl.rho, gamma=wl.gamma, delta=wl.recon_weight)
    dt = time.perf_counter() - t0
    # the same crop with the blocks of each dependency level on all host cores
    t0 = time.perf_counter()
    par, n_levels, threads = oracle.image_levels(img, msk, wl.classes, rho=wl.rho, gamma=wl.gamma,
                                                 delta=wl.recon_weight)
    dtp = time.perf_counter() - t0
    return {"value": nb / dt, "unit": "blocks/s", "cores": 1, "kind": "oracle",
            "sample": f"top-left {crop[1]}x{crop[0]} crop of the first 1920x1080 request ({nb} blocks, {dt:.1f} s, "
                      f"single-threaded FP64 C oracle)",
            "level_parallel": {"value": nb / dtp, "unit": "blocks/s", "cores": threads, "kind": "oracle",
                               "sample": f"same crop, the blocks of each of its {n_levels} dependency levels run "
                                         f"in parallel (OpenMP), {dtp:.1f} s",
                               "speedup_vs_one_core": dt / dtp,
                               "bitwise_equal_to_one_core": bool(np.array_equal(ref, par))}}


def cpu_tile_framework(one_core_rate: float):
    """The paper's framework on the host (Sec. III): the first 1080p request cut
    into N = (host threads, at most 16) tiles with stripe d = 32 -- the compact
    tiling of Algorithm 1 and, for comparison, N full-height stripes -- each
    extended tile extrapolated by the FP64 C oracle as an image of its own on
    a thread of its own, cores cropped and merged.  Rate in the request's lost
    blocks per wall second, as for the GPU tile rows; speed-up against the
    one-core oracle rate (the shape of the paper's speed-up per node count)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle
    from paper_2207_00238_amd import synth

    wl = synth.workload("hd")
    H, W = wl.mask.shape
    n = max(1, min(16, len(os.sched_getaffinity(0))))
    nb = len(oracle.plan(wl.mask, wl.classes)[0])

    def run(vertical):
        tiles = [t for t in oracle.tiles_with_stripe(W, H, n, 32, 4, vertical=vertical) if t[1][2] > 0 and t[1][3] > 0]
        out = np.zeros((H, W))

        def one(t):
            (cx, cy, cw, ch), (ex, ey, ew, eh) = t
            sub = oracle.image(wl.image[ey:ey + eh, ex:ex + ew], wl.mask[ey:ey + eh, ex:ex + ew], wl.classes,
                               rho=wl.rho, gamma=wl.gamma, delta=wl.recon_weight)
            out[cy:cy + ch, cx:cx + cw] = sub[cy - ey:cy - ey + ch, cx - ex:cx - ex + cw]

        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=n) as ex:
            list(ex.map(one, tiles))
        return len(tiles), time.perf_counter() - t0

    nt, dt = run(False)
    ntv, dtv = run(True)
    t1 = nb / one_core_rate  # the whole request on one core, from the one-core oracle rate
    return {"value": nb / dt, "unit": "blocks/s", "cores": n, "kind": "oracle",
            "sample": f"first 1920x1080 request ({nb} lost blocks), {nt} compact tiles with d = 32, one "
                      f"FP64 C oracle thread per tile, {dt:.1f} s wall",
            "speedup_vs_one_core": t1 / dt,
            "vertical_stripes": {"value": nb / dtv, "unit": "blocks/s", "tiles": ntv, "wall_s": dtv,
                                 "speedup_vs_one_core": t1 / dtv}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16, help="1920x1080 requests per batched step")
    ap.add_argument("--no-autotune", action="store_true", help="use the automatic schedule instead of the autotuner")
    ap.add_argument("--uhd-images", type=int, default=16,
                    help="3840x2160 mixed-loss images for the tiled batch measurement (0 = skip)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-block comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-order", action="store_true", help="skip the optimised-processing-order request")
    ap.add_argument("--streams", type=int, default=4,
                    help="streams the timed batched steps rotate over (1 = one step at a time; with the "
                         "default four, plain streams still get hardware queues of their own)")
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--block-waves", type=int, default=0, help="wave64s per block (0 = autotuned among 1, 2, 4)")
    ap.add_argument("--tiles", type=str, default="64",
                    help="comma-separated tile counts for the tile-framework comparison ('' = none)")
    ap.add_argument("--serve-seconds", type=float, default=4.0, help="length of the served Poisson stream (0 = skip)")
    ap.add_argument("--no-precision-sweep", action="store_true", help="skip the FP32 / BF16x3 comparison")
    ap.add_argument("--no-border-sweep", action="store_true",
                    help="skip the tile-border sweep (PSNR vs stripe width d at N = 32 tiles)")
    ap.add_argument("--serve-rate", type=float, default=16.0, help="requests per second of the served stream")
    ap.add_argument("--serve-mixed-seconds", type=float, default=60.0,
                    help="arrival window of the mixed-size served stream (0 = skip)")
    ap.add_argument("--serve-mixed-below-seconds", type=float, default=8.0,
                    help="arrival window of the same stream at 40 and 80 requests/s (0 = skip)")
    ap.add_argument("--serve-mixed-rate", type=float, default=200.0,
                    help="requests per second of the mixed-size served stream (sides 512..4096)")
    ap.add_argument("--only-uhd", action="store_true",
                    help="measure only the 3840x2160 tiled batch, automatic grid, no autotuning (for profiler runs)")
    ap.add_argument("--only-batched", action="store_true",
                    help="measure the batched step only (for profiler runs): no secondary measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 256 MiB device-to-device copy (a known-size kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the method's tiles are "
              "independent, so several GPUs would each run their own share", file=sys.stderr)
        sys.exit(2)
    if args.streams < 1:
        ap.error("--streams must be at least 1")

    import numpy as np
    import torch

    from paper_2207_00238_amd import fse, synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.only_uhd:
        print(json.dumps({"uhd_tiled_batch": uhd_plain(fse, torch, np, max(1, args.uhd_images), args.steps,
                                                       args.warmup)}), flush=True)
        return

    n_img = max(1, args.batch)
    wls = [synth.workload("hd", i) for i in range(n_img)]
    wl = wls[0]
    imgs = [torch.from_numpy(w.image).to(dev) for w in wls]
    msks = [torch.from_numpy(w.mask).to(dev) for w in wls]
    outs = [torch.empty_like(t) for t in imgs]
    stream = torch.cuda.current_stream()
    B, b, K = wl.classes[-1]
    M = B + 2 * b
    common = dict(classes=wl.classes, rho=wl.rho, gamma=wl.gamma, recon_weight=wl.recon_weight,
                  workgroups=args.workgroups, block_waves=args.block_waves)
    params = fse.fse_params_default(**common)

    # ---- batched step: n_img requests in one persistent launch -------------
    tuned = None
    if not args.no_autotune and args.workgroups == 0:
        params = fse.fse_autotune(imgs, msks, params, outs, stream)
        tuned = {"block_waves": params.block_waves, "workgroups": params.workgroups}
    for _ in range(max(args.warmup, 1)):
        fse.fse_extrapolate_batch(imgs, msks, params, outs, stream)
    st = fse.fse_last_stats()
    n_blocks = st["n_blocks"]

    progress("warm-up and autotuning done")
    # serialised steps: each launch alone on the device (launch duration,
    # roofline and step latency are taken here)
    step_ms, kern_ms, plan_ms = [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        fse.fse_extrapolate_batch(imgs, msks, params, outs, stream)
        s = fse.fse_last_stats()  # waits for the step's stream
        step_ms.append((time.perf_counter() - t0) * 1e3)
        kern_ms.append(s["kernel_ms"])
        plan_ms.append(s["host_plan_ms"])
        if s["device_error"]:
            raise RuntimeError("device dependency wait timed out")
    torch.cuda.synchronize()
    total_serial = time.perf_counter() - t_all
    serial_outs = [o.clone() for o in outs]
    batched_out0 = serial_outs[0]
    end_to_end = end_to_end_with_copies(fse, torch, imgs, msks, outs, params, stream, n_blocks, args.steps)

    progress("serialised steps done")
    # pipelined steps: consecutive batches on `streams` streams (each with
    # its own workspace and outputs), so the host planning of a batch and the
    # launches of the batches before it run at the same time and the
    # dependency chains of two or three batches share the CUs
    pipe = None
    total = total_serial
    if args.streams > 1:
        strs = [stream] + [torch.cuda.Stream() for _ in range(args.streams - 1)]
        pouts = [outs] + [[torch.empty_like(t) for t in imgs] for _ in range(args.streams - 1)]

        def rotate(p, steps):
            for i in range(steps):
                fse.fse_extrapolate_batch(imgs, msks, p, pouts[i % args.streams], strs[i % args.streams])

        # grid for overlapping steps (untimed): the step-at-a-time choice
        # above need not be the best once several launches share the CUs
        p_pipe = params
        if args.workgroups == 0 and not args.no_autotune:
            # the library's tuner for consecutive calls in flight (the waves per
            # block fixed to the single-call choice)
            p_pipe = fse.fse_autotune_overlapped(imgs, msks, params, outs, args.streams)
        rotate(p_pipe, args.streams)
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        rotate(p_pipe, args.steps)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_all
        if fse.fse_last_stats()["device_error"]:
            raise RuntimeError("device dependency wait timed out")
        same = all(torch.equal(a, b) for o in pouts for a, b in zip(o, serial_outs))
        pipe = {"streams": args.streams, "workgroups": p_pipe.workgroups or "automatic",
                "ms_per_step": total * 1e3 / args.steps, "bitwise_equal_to_serialised": bool(same)}
    value = n_blocks * args.steps / total

    flops = block_flops(M, K, B)
    k_avg = float(np.mean(kern_ms)) / 1e3
    achieved = n_blocks * flops / k_avg / 1e12
    traffic = traffic_from_profiles("hd", n_blocks)

    result = {
        "metric": "lost 4x4 blocks/s at K=100 (batched+served vs plain GPU, same acc.); p50/p99 ms",
        "value": value,
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hd: {n_img} requests of 1920x1080, 25% 4x4 blocks + 1% pixels lost, "
                               f"{n_blocks} processing blocks per step, B={B} b={b} M={M} K={K}, rho={wl.rho}, "
                               f"gamma={wl.gamma}, exact raster semantics per request",
                   "schedule": f"one persistent dependency-driven launch per step, "
                               f"{params.block_waves or 4} waves/block, grid {params.workgroups or 'automatic'}"
                               + (" (autotuned)" if tuned else "")
                               + (f"; consecutive steps on {args.streams} streams, grid "
                                  f"{pipe['workgroups']}" if pipe else "")},
        "serialised": {"value": n_blocks * args.steps / total_serial, "ms_per_step": total_serial * 1e3 / args.steps},
        "end_to_end_with_copies": end_to_end,
        "pipelined": pipe,
        "step_p50_ms": float(np.percentile(step_ms, 50)),
        "step_p99_ms": float(np.percentile(step_ms, 99)),
        "kernel_ms": float(np.mean(kern_ms)),
        "host_plan_ms": float(np.mean(plan_ms)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": MI355X_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MI355X_FP64_VECTOR_TFLOPS, "traffic": traffic,
                     "kernel": f"k_fse_blocks<{params.block_waves or 4}>", "flops_per_block": flops,
                     # the same work over the overlapped timed steps (launches share the device there)
                     "achieved_overlapped": n_blocks * flops * args.steps / total / 1e12,
                     "frac_overlapped": n_blocks * flops * args.steps / total / 1e12 / MI355X_FP64_VECTOR_TFLOPS,
                     "phases": phases_from_profiles("hd")},
    }

    progress("pipelined steps done")
    if args.only_batched:
        print(json.dumps(result), flush=True)
        return

    # ---- same masks, new images: prepared plan replayed as a HIP graph -------
    plan = fse.fse_plan_create(msks, params)
    try:
        fse.fse_plan_execute(plan, imgs, outs, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fse.fse_plan_execute(plan, imgs, outs, stream)
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t0) / args.steps
        result["graph_replay"] = {"value": n_blocks / dtg, "unit": "blocks/s", "ms_per_step": dtg * 1e3,
                                  "bitwise_equal_to_batched": bool(torch.equal(outs[0], batched_out0)),
                                  "note": "masks planned once; each step replays the captured launch"}
    finally:
        fse.fse_plan_destroy(plan)

    progress("graph replay done")
    # ---- one request alone ------------------------------------------------
    img, msk, out = imgs[0], msks[0], outs[0]
    fse.fse_extrapolate(img, msk, params, out, stream)
    s = fse.fse_last_stats()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        fse.fse_extrapolate(img, msk, params, out, stream)
        s1 = fse.fse_last_stats()
        times.append(time.perf_counter() - t0)
    nb1 = s1["n_blocks"]
    res_single = out.clone()
    result["single_request"] = {"value": nb1 / float(np.mean(times)), "unit": "blocks/s",
                                "ms": float(np.mean(times)) * 1e3, "kernel_ms": s1["kernel_ms"],
                                "blocks": nb1, "bitwise_equal_to_batched": bool(torch.equal(res_single, batched_out0))}

    progress("single request done")
    # ---- the optimised processing order (Sec. II) on the same request --------
    if not args.no_order:
        result["optimized_order"] = optimized_order(fse, torch, np, img, msk, common, wl, args.steps, res_single,
                                                    s1, float(np.mean(times)))

    if args.tiles:
        m = torch.from_numpy(wl.mask).bool()
        gt = torch.from_numpy(wl.image).double()

        def psnr(x):
            e = (x.double().clamp(0, 255) - gt)[m]
            return float(10 * torch.log10(255.0 ** 2 / (e * e).mean()))

        p_whole = psnr(res_single.cpu())
        s_whole = ssim(res_single.cpu().numpy(), wl.image)
        result["psnr_whole_db"] = p_whole
        result["ssim_whole"] = s_whole
        result["tiled"] = []
        for N in [int(v) for v in args.tiles.split(",") if v]:
            pt = fse.fse_params_default(tiling=fse.FSE_TILED, n_tiles=N, overlap=32, align=16, **common)
            fse.fse_extrapolate(img, msk, pt, out, stream)
            fse.fse_last_stats()
            times = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                fse.fse_extrapolate(img, msk, pt, out, stream)
                s = fse.fse_last_stats()
                times.append(time.perf_counter() - t0)
            dt = float(np.mean(times))
            result["tiled"].append({"n_tiles": N, "overlap": 32, "value": nb1 / dt, "unit": "blocks/s",
                                    "ms_per_step": dt * 1e3, "kernel_ms": s["kernel_ms"],
                                    "blocks_executed": s["n_blocks"],
                                    "dpsnr_vs_whole_db": psnr(out.cpu()) - p_whole,
                                    "dssim_vs_whole": ssim(out.cpu().numpy(), wl.image) - s_whole})

    progress("optimised order and tile framework done")
    # the time to compute a tiling (the paper times its tilings of 6024x4024
    # images): fse_plan_tiles through a bare ctypes call, mean over repeated
    # calls -- an upper bound, the call overhead included
    lib = fse.lib()
    tiles_buf = (fse.fse_tile_t * 64)()
    result["tiling_time_us"] = {"note": "6024x4024, d = 32; one ctypes call, overhead included"}
    for N in (16, 32, 64):
        reps = 20000
        t0 = time.perf_counter()
        for _ in range(reps):
            lib.fse_plan_tiles(6024, 4024, N, 32, 4, tiles_buf)
        result["tiling_time_us"][str(N)] = (time.perf_counter() - t0) / reps * 1e6

    if args.tiles and not args.no_border_sweep:
        result["tile_border_sweep"] = border_sweep(fse, torch, np, img, msk, common, wl, p_whole, s_whole)

    progress("tiling time and border sweep done")
    if args.uhd_images > 0:
        result["uhd_tiled_batch"] = uhd_batch(fse, torch, np, args.uhd_images, args.steps, args.streams)

    progress("3840x2160 tiled batch done")
    if not args.no_precision_sweep:
        ws = synth.workload("small")
        small = (torch.from_numpy(ws.image).to(dev), torch.from_numpy(ws.mask).to(dev))
        result["precision_sweep"] = precision_sweep(fse, torch, np, common, [
            ("128x128, 20% of 4x4 blocks lost", small[0], small[1], ws.image, ws.classes),
            ("1920x1080, 25% of 4x4 blocks + 1% pixels lost", img, msk, wl.image, wl.classes)])

    progress("precision sweep done")
    if args.serve_seconds > 0:
        # served launches hold one to a few requests: the automatic grid (sized
        # from each launch's own blocks per wavefront key), not the batch's
        p_serve = fse.fse_params_default(**{**common, "workgroups": 0, "block_waves": params.block_waves})
        result["served"] = serve_stream(fse, torch, np, imgs, msks, p_serve, args.serve_rate, args.serve_seconds,
                                        nb1, res_single)

    progress("served 1080p stream done")
    if args.serve_mixed_seconds > 0:
        result["served_mixed"] = serve_mixed(fse, torch, np, common, args.serve_mixed_rate,
                                             args.serve_mixed_seconds, plain_sample=40)
        # below capacity: the same trace recipe at lower rates
        result["served_mixed"]["below_capacity"] = [
            {k: v for k, v in serve_mixed(fse, torch, np, common, r, args.serve_mixed_below_seconds).items()
             if k in ("requests", "rate_hz", "seconds", "offered_blocks_per_s", "value", "p50_ms", "p99_ms",
                      "drain_s")}
            for r in (40.0, 80.0)] if args.serve_mixed_below_seconds > 0 else []

    progress("served mixed-size streams done")
    if not args.no_plain:
        p_plain = fse.fse_params_default(schedule=fse.FSE_SCHED_PER_BLOCK, **common)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fse.fse_extrapolate(img, msk, p_plain, out, stream)
        s = fse.fse_last_stats()
        dt = time.perf_counter() - t0
        same = bool(torch.equal(out, res_single))
        result["plain"] = {"value": nb1 / dt, "unit": "blocks/s", "ms": dt * 1e3,
                           "kernel_ms": s["kernel_ms"], "schedule": "one launch per block, raster order, one request",
                           "bitwise_equal_to_batched": same}
        result["speedup_vs_plain"] = value / (nb1 / dt)

    progress("plain path done")
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline()
        if not args.only_batched:
            result["cpu_baseline"]["tile_framework"] = cpu_tile_framework(result["cpu_baseline"]["value"])
    print(json.dumps(result), flush=True)


def optimized_order(fse, torch, np, img, msk, common, wl, steps, res_raster, st_raster, t_raster):
    """One 1080p request in the optimised processing order (FSE_ORDER_OPTIMIZED)
    beside the same request in raster order: dependency levels of the two
    DAGs, host planning and kernel time, end-to-end time, and the PSNR of
    each against the pre-loss image."""
    p = fse.fse_params_default(**{**common, "workgroups": 0, "order": fse.FSE_ORDER_OPTIMIZED})
    out = torch.empty_like(img)
    fse.fse_extrapolate(img, msk, p, out)
    fse.fse_last_stats()
    times, kern, plan = [], [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        fse.fse_extrapolate(img, msk, p, out)
        s = fse.fse_last_stats()
        times.append(time.perf_counter() - t0)
        kern.append(s["kernel_ms"])
        plan.append(s["host_plan_ms"])
    if s["device_error"]:
        raise RuntimeError("device dependency wait timed out")
    m = torch.from_numpy(wl.mask).bool()
    gt = torch.from_numpy(wl.image).double()

    def psnr(x):
        e = (x.double().clamp(0, 255) - gt)[m]
        return float(10 * torch.log10(255.0 ** 2 / (e * e).mean()))

    return {"value": s["n_blocks"] / float(np.mean(times)), "unit": "blocks/s",
            "ms": float(np.mean(times)) * 1e3, "kernel_ms": float(np.mean(kern)),
            "host_plan_ms": float(np.mean(plan)), "levels": s["wavefront_keys"],
            "psnr_db": psnr(out.cpu()), "raster": {"ms": t_raster * 1e3, "kernel_ms": st_raster["kernel_ms"],
                                                  "host_plan_ms": st_raster["host_plan_ms"],
                                                  "levels": st_raster["wavefront_keys"],
                                                  "psnr_db": psnr(res_raster.cpu())}}


def border_sweep(fse, torch, np, img, msk, common, wl, p_whole, s_whole):
    """The paper's tile-border experiment (Sec. IV, PSNR against the stripe
    width d) on the first 1080p request: N = 32 tiles of the compact tiling,
    stripes d in {0, 1, 2, 4, 8, ..., 96} (tile cores on the 4-pixel block grid), each
    tile extrapolated as an independent image, cropped and merged.  PSNR over
    the lost pixels against the ground truth and SSIM of the whole image, their
    change against the whole-image result, and the executed blocks (stripes
    add work)."""
    m = torch.from_numpy(wl.mask).bool()
    gt = torch.from_numpy(wl.image).double()
    out = torch.empty_like(img)
    def run(tiling, d):
        p = fse.fse_params_default(tiling=tiling, n_tiles=32, overlap=d, align=4, **common)
        fse.fse_extrapolate(img, msk, p, out)
        s = fse.fse_last_stats()
        e = (out.cpu().double().clamp(0, 255) - gt)[m]
        ps = float(10 * torch.log10(255.0 ** 2 / (e * e).mean()))
        return {"d": d, "psnr_db": ps, "dpsnr_vs_whole_db": ps - p_whole,
                "dssim_vs_whole": ssim(out.cpu().numpy(), wl.image) - s_whole, "blocks_executed": s["n_blocks"],
                "kernel_ms": s["kernel_ms"]}

    rows = [run(fse.FSE_TILED, d) for d in (0, 1, 2, 4, 8, 16, 24, 32, 48, 64, 96)]
    # the same N and stripes with N full-height stripes instead of the compact
    # grid of eq. (5): the overlap the compact tiling is there to avoid
    vert = [run(fse.FSE_TILED_VERTICAL, d) for d in (0, 8, 32)]
    return {"n_tiles": 32, "align": 4, "rows": rows, "vertical_stripes": vert}


def uhd_plain(fse, torch, np, n, steps, warmup):
    """The 3840x2160 tiled batch of :func:`uhd_batch` launched eagerly with the
    automatic grid and no autotuning: a fixed launch sequence for profilers."""
    from paper_2207_00238_amd import synth
    dev = torch.device("cuda:0")
    wls = [synth.workload("uhd", i) for i in range(n)]
    imgs = [torch.from_numpy(w.image).to(dev) for w in wls]
    msks = [torch.from_numpy(w.mask).to(dev) for w in wls]
    outs = [torch.empty_like(t) for t in imgs]
    p = fse.fse_params_default(classes=wls[0].classes, tiling=fse.FSE_TILED, n_tiles=64, overlap=32, align=16)
    for _ in range(max(warmup, 1)):
        fse.fse_extrapolate_batch(imgs, msks, p, outs)
        fse.fse_last_stats()
    kms = []
    for _ in range(steps):
        fse.fse_extrapolate_batch(imgs, msks, p, outs)
        s = fse.fse_last_stats()
        kms.append(s["kernel_ms"])
    return {"images": n, "blocks_executed": s["n_blocks"], "kernel_ms": float(np.mean(kms)),
            "value": s["n_blocks"] / (float(np.mean(kms)) / 1e3), "unit": "blocks/s (executed, kernel time)"}


def uhd_batch(fse, torch, np, n, steps, streams=1):
    """3840x2160 frames with mixed 8x8 (10 %), 16x16 (5 %) and row (0.5 %)
    losses (64x64 windows with K = 200 for the 8x8 and 16x16 blocks, 32x32 with
    K = 100 for the rest), each cut into 64 tiles with stripe d = 32 by the
    compact tiling, all tiles of all frames in one persistent launch: the
    schedule (persistent grid) autotuned, then the launch captured once as a
    HIP graph and replayed.  With streams > 1, consecutive steps also rotate
    over that many streams (outputs of their own), so the host planning of
    one step overlaps the launches before it."""
    from paper_2207_00238_amd import synth
    dev = torch.device("cuda:0")
    wls = [synth.workload("uhd", i) for i in range(n)]
    imgs = [torch.from_numpy(w.image).to(dev) for w in wls]
    msks = [torch.from_numpy(w.mask).to(dev) for w in wls]
    outs = [torch.empty_like(t) for t in imgs]
    p = fse.fse_params_default(classes=wls[0].classes, tiling=fse.FSE_TILED, n_tiles=64, overlap=32, align=16)
    p = fse.fse_autotune(imgs, msks, p, outs)
    fse.fse_extrapolate_batch(imgs, msks, p, outs)
    fse.fse_last_stats()
    times = []
    for _ in range(max(1, steps // 2)):
        t0 = time.perf_counter()
        fse.fse_extrapolate_batch(imgs, msks, p, outs)
        s = fse.fse_last_stats()
        times.append(time.perf_counter() - t0)
    dt = float(np.mean(times))
    eager0 = outs[0].clone()
    res = {"images": n, "tiles_per_image": 64, "overlap": 32, "blocks_executed": s["n_blocks"],
           "value": s["n_blocks"] / dt, "unit": "blocks/s (executed, incl. stripe overlap)",
           "ms_per_step": dt * 1e3, "kernel_ms": s["kernel_ms"], "host_plan_ms": s["host_plan_ms"],
           "schedule": f"grid {p.workgroups or 'automatic'} (autotuned), 8 waves per 64x64 block"}
    plan = fse.fse_plan_create(msks, p)
    try:
        fse.fse_plan_execute(plan, imgs, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(1, steps // 2)
        for _ in range(reps):
            fse.fse_plan_execute(plan, imgs, outs)
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t0) / reps
        res["graph_replay"] = {"value": s["n_blocks"] / dtg, "ms_per_step": dtg * 1e3,
                               "bitwise_equal_to_eager": bool(torch.equal(outs[0], eager0))}
    finally:
        fse.fse_plan_destroy(plan)
    if streams > 1:
        strs = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(streams - 1)]
        pouts = [outs] + [[torch.empty_like(t) for t in imgs] for _ in range(streams - 1)]
        for j in range(streams):  # each stream's workspace, untimed
            fse.fse_extrapolate_batch(imgs, msks, p, pouts[j], strs[j])
        torch.cuda.synchronize()
        reps = max(2 * streams, steps)
        t0 = time.perf_counter()
        for i in range(reps):
            fse.fse_extrapolate_batch(imgs, msks, p, pouts[i % streams], strs[i % streams])
        torch.cuda.synchronize()
        dtp = (time.perf_counter() - t0) / reps
        res["pipelined"] = {"streams": streams, "value": s["n_blocks"] / dtp, "ms_per_step": dtp * 1e3,
                            "bitwise_equal_to_eager": all(bool(torch.equal(o[0], eager0)) for o in pouts)}
    return res


def precision_sweep(fse, torch, np, common, cases):
    """FP32 and BF16x3 against the FP64 path (which the tests hold to the FP64
    oracle within 1e-5) on each named workload: speed, pixel error, PSNR
    change, the rate of blocks whose basis selections leave the FP64 sequence
    (mirror choices of exactly tied pairs, which give the same real output,
    are not counted), and whether the pixel part of the stated bar holds
    (>= 99.9 % of lost pixels within 0.5, |dPSNR| <= 0.01 dB).  The tests
    apply the full bar, with the oracle's energy gaps, to the 128 x 128
    workload."""
    rows = []
    for (name, img, msk, gt_np, classes) in cases:
        K = max(c[2] for c in classes)
        M = classes[-1][0] + 2 * classes[-1][1]
        m = torch.from_numpy(msk.cpu().numpy()).bool()
        gt = torch.from_numpy(gt_np).double()

        def psnr(x):
            e = (x.double().clamp(0, 255) - gt)[m]
            return float(10 * torch.log10(255.0 ** 2 / (e * e).mean()))

        def run(prec):
            st0 = fse.fse_params_default(**{**common, "classes": classes, "precision": prec, "workgroups": 0})
            out = torch.empty_like(img)
            fse.fse_extrapolate(img, msk, st0, out)
            nb = fse.fse_last_stats()["n_blocks"]
            sel = torch.full((nb, K), -1, dtype=torch.int32, device=img.device)
            st0.trace_sel = sel.data_ptr()
            st0.trace_stride = K
            st0.trace_capacity = nb
            t0 = time.perf_counter()
            fse.fse_extrapolate(img, msk, st0, out)
            s = fse.fse_last_stats()
            dt = time.perf_counter() - t0
            return out.cpu(), sel.cpu().numpy(), nb / dt, s["kernel_ms"]

        ref, sref, v64, k64 = run(0)
        p64 = psnr(ref)
        u, v = np.divmod(sref, M)
        mirror = ((-u) % M) * M + ((-v) % M)
        rows.append({"workload": name, "mode": "fp64", "value": v64, "kernel_ms": k64})
        for mode, prec in (("fp32", 1), ("bf16x3", 2)):
            out, sel, val, km = run(prec)
            d = (out.double() - ref.double()).abs()[m]
            same = (sel == sref) | (sel == mirror)
            bad = (~same).any(axis=1)
            frac = float((d <= 0.5).double().mean())
            dpsnr = psnr(out) - p64
            rows.append({"workload": name, "mode": mode, "value": val, "kernel_ms": km,
                         "max_abs_dpixel": float(d.max()), "frac_le_half": frac, "dpsnr_db": dpsnr,
                         "selection_divergence_rate": float(bad.mean()),
                         "meets_pixel_bar": bool(frac >= 0.999 and abs(dpsnr) <= 0.01)})
    return rows


def serve_stream(fse, torch, np, imgs, msks, params, rate, seconds, blocks_per_req, ref0):
    """Poisson arrivals of 1920x1080 requests (inputs cycled from a pool of
    distinct images) into the continuous-batching server; latency = submit to
    done on the host clock."""
    rng = np.random.default_rng(31)
    arrivals = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        arrivals.append(t)
    srv = fse.fse_serve_create(hbm_budget_bytes=16 << 30, max_slots=4)
    outs = [torch.empty_like(imgs[0]) for _ in arrivals]
    tickets = []
    try:
        t0 = time.perf_counter()
        for i, ta in enumerate(arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            k = i % len(imgs)
            tickets.append((fse.fse_serve_submit(srv, imgs[k], msks[k], params, outs[i]), k))
        stats = [fse.fse_serve_wait(srv, tk, 120_000_000) for tk, _ in tickets]
        t_end = time.perf_counter()
    finally:
        fse.fse_serve_destroy(srv)
    lat = np.array([s["t_done_ms"] - s["t_submit_ms"] for s in stats])
    first0 = next(i for i, (_, k) in enumerate(tickets) if k == 0)
    blocks = sum(s["n_blocks"] for s in stats)
    return {"requests": len(arrivals), "rate_hz": rate, "seconds": seconds,
            "value": blocks / (t_end - t0), "unit": "blocks/s",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "bitwise_equal_to_alone": bool(torch.equal(outs[first0], ref0))}


def serve_mixed(fse, torch, np, common, rate, seconds, pool_per_side=96, plain_sample=0):
    """The serving workload: Poisson arrivals at ``rate`` over ``seconds`` of
    square requests with sides {512, 1024, 2048, 4096} and two mask kinds
    (the serving trace of the input recipe) into the continuous-batching
    server.  Inputs come from a pool of one image and mask per (side, kind);
    outputs from a pool of ``pool_per_side`` buffers per side, recycled as
    requests finish: a request that arrives while every buffer of its side is
    in use waits in arrival order for the next free one.  Latency runs from
    the request's arrival (not its submission) to its completion on the host
    clock, so waiting for a buffer counts as queueing.  Above capacity the
    achieved rate is the saturation throughput and the latencies grow with
    the backlog, which is reported once per second (requests arrived and not
    finished).  With ``plain_sample`` > 0 the first requests of the trace are
    also run one at a time through fse_extrapolate, the plain per-request
    path."""
    from collections import deque
    from paper_2207_00238_amd import synth
    dev = torch.device("cuda:0")
    trace = synth.poisson_trace(rate, seconds, seed=31)
    pool = {}
    for req in trace:
        key = (req["side"], req["kind"])
        if key not in pool:
            img, msk = synth.request_inputs(req)
            pool[key] = (torch.from_numpy(img).to(dev), torch.from_numpy(msk).to(dev))
    p = fse.fse_params_default(**{**common, "workgroups": 0})
    sides = sorted({r["side"] for r in trace})
    free = {sd: deque(torch.empty((sd, sd), dtype=torch.float32, device=dev) for _ in range(pool_per_side))
            for sd in sides}
    torch.cuda.synchronize()
    srv = fse.fse_serve_create(hbm_budget_bytes=32 << 30, max_slots=4)
    waiting = deque()      # arrived, no free output buffer yet
    inflight = {}          # ticket -> (trace index, output buffer)
    done_at = [None] * len(trace)
    blocks = [0] * len(trace)
    first_out = {}         # side -> output of the first request of that side (kept for the check below)
    backlog = []
    nxt = 0
    t0 = time.perf_counter()
    next_sample = 1.0
    try:
        while nxt < len(trace) or waiting or inflight:
            now = time.perf_counter() - t0
            while nxt < len(trace) and trace[nxt]["t"] <= now:
                waiting.append(nxt)
                nxt += 1
            # submit in arrival order while buffers last (a request whose side
            # has no free buffer holds back the ones behind it only of its side)
            held = deque()
            while waiting:
                i = waiting.popleft()
                sd = trace[i]["side"]
                if free[sd]:
                    out = free[sd].popleft()
                    im, mk = pool[(sd, trace[i]["kind"])]
                    inflight[fse.fse_serve_submit(srv, im, mk, p, out)] = (i, out)
                else:
                    held.append(i)
            waiting = held
            # requests finish roughly in submission order: poll the oldest few
            for tk in list(itertools.islice(inflight, 48)):
                fin, st = fse.fse_serve_poll(srv, tk)
                if fin:
                    i, out = inflight.pop(tk)
                    done_at[i] = time.perf_counter() - t0
                    blocks[i] = st["n_blocks"]
                    sd = trace[i]["side"]
                    if sd not in first_out:
                        first_out[sd] = (i, out)  # not recycled: compared below
                    else:
                        free[sd].append(out)
            if now >= next_sample:
                backlog.append([round(now, 1), nxt - sum(d is not None for d in done_at)])
                next_sample += 1.0
                if len(backlog) % 15 == 0:
                    progress(f"served stream at {rate:g}/s: {now:.0f} s, {backlog[-1][1]} requests waiting or running")
            time.sleep(0.002)
        t_end = time.perf_counter() - t0
    finally:
        fse.fse_serve_destroy(srv)
    lat = np.array([(done_at[i] - trace[i]["t"]) * 1e3 for i in range(len(trace))])
    total_blocks = sum(blocks)
    # the first request of each side against the same request alone
    same = True
    for sd, (i, out) in first_out.items():
        im, mk = pool[(sd, trace[i]["kind"])]
        o = torch.empty_like(im)
        fse.fse_extrapolate(im, mk, p, o)
        torch.cuda.synchronize()
        same = same and bool(torch.equal(o, out))
    res = {"requests": len(trace), "rate_hz": rate, "seconds": seconds, "sides": sides,
           "offered_blocks_per_s": total_blocks / seconds, "value": total_blocks / t_end, "unit": "blocks/s",
           "drain_s": t_end, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "latency_from": "arrival", "output_buffers_per_side": pool_per_side,
           "backlog_requests_per_s": backlog[::max(1, len(backlog) // 20)],
           "bitwise_equal_to_alone": same}
    if plain_sample > 0:
        # the plain per-request path: the first requests one at a time
        torch.cuda.synchronize()
        tp = time.perf_counter()
        nbp = 0
        for r in trace[:plain_sample]:
            im, mk = pool[(r["side"], r["kind"])]
            o = free[r["side"]][0] if free[r["side"]] else torch.empty_like(im)
            fse.fse_extrapolate(im, mk, p, o)
            nbp += fse.fse_last_stats()["n_blocks"]
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        res["plain_per_request"] = {"value": nbp / dtp, "unit": "blocks/s", "requests": plain_sample,
                                    "note": "the trace's first requests, each alone through fse_extrapolate"}
    return res


if __name__ == "__main__":
    main()
