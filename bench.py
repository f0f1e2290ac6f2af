#!/usr/bin/env python3
"""Benchmark of the WD-WENO 2x zoom on one MI355X.

Headline (one JSON line on stdout): output Mpix/s of one 2x doubling of a
1920x1080 RGB float32 frame (planar, [0,1] scale, the polygon scene) to
3840x2160, with the HBM-roofline fraction of the kernel and the FP64 CPU
oracle timed beside it.  A "step" is one weno_zoom2x call on that frame,
inputs resident in HBM.

Extra fields (same line): the uint8 HWC variant of the frame, 512 uneven
images in one persistent launch vs a per-image launch loop, three fused
doublings of a 256x256 pixel-art image replayed from a HIP graph, zooming the
frame to 5760x3240 (two doublings and the tensor resampler), and
forward+backward of a 16x3x512x512 float32 batch.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only-main | --only-zoom-to | --only-u8 | --only-fwd-bwd | --only-cascade]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# FP32 VALU peak without packed math (the library is compiled with packed FP32 off):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6432
ALU_PEAK_PACKED_TFLOPS = 157.2864
# algorithmic FP32 operations per output quad per channel (FMA = 2, rcp = 1):
# x point 74, each + point 64, second differences of phase 2 12
FLOPS_PER_QUAD = 214
KERNEL_SOURCES = ["paper_2312_00229_amd/csrc/weno_fwd.h",  # the forward kernel body
                  "paper_2312_00229_amd/csrc/weno_api.hip"]  # its launch: grid, block map, strip shape
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_zoom2x_rgb_f32_1080p.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def strip_comments(src: str) -> str:
    """C++ source without its comments and with each line's blank space
    trimmed, string and character literals kept as written."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (ln.strip() for ln in "".join(out).splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash() -> str:
    """Hash of the headline kernel's code (comments and blank space excluded),
    which the stored traffic figures must match to be used."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def timed(fn, steps, warmup, torch):
    """Average ms per call of fn() over `steps` calls after `warmup`, with HIP
    events on the current stream bracketing the timed region."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def clock_spinup(fn, torch, min_s=0.15, max_s=0.6, chunk=100):
    """Bring the GPU to its sustained clock before anything is measured.  A
    GPU coming out of idle runs its first tens of milliseconds of load at a
    lower clock (the 1080p doubling: ~45 us per launch over the first 100
    launches, 35 us from ~60 ms on), which is the power state, not the
    kernel.  Runs fn in chunks until at least min_s has passed and two
    consecutive chunks agree within 1 % (at most max_s); the W warm-up steps
    and the K timed steps follow as usual.  Returns what it did, for the
    bench line."""
    t0 = time.perf_counter()
    prev = None
    n = 0
    last = None
    while True:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(chunk):
            fn()
        e1.record()
        torch.cuda.synchronize()
        n += chunk
        last = e0.elapsed_time(e1) / chunk
        el = time.perf_counter() - t0
        if el >= max_s or (el >= min_s and prev is not None and abs(last - prev) <= 0.01 * prev):
            break
        prev = last
    return {"launches": n, "seconds": round(time.perf_counter() - t0, 3), "last_chunk_ms": round(last, 5)}


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def host_threads() -> int:
    """OpenMP threads the C oracle runs with (OMP_NUM_THREADS, else all cores)."""
    try:
        return int(os.environ.get("OMP_NUM_THREADS", ""))
    except ValueError:
        return os.cpu_count() or 1


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img_planar, budget_s=10.0):
    """The FP64 oracle on the headline frame, repeated for about `budget_s`
    seconds of host time; the mean rate over the repeats."""
    import oracle

    x64 = img_planar.astype(np.float64)
    runs, t0 = 0, time.perf_counter()
    while True:
        oracle.zoom2x(x64)
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    H, W = img_planar.shape[-2:]
    return {
        "value": round(runs * 4 * H * W / dt / 1e6, 3),
        "unit": "output Mpix/s",
        "cores": host_threads(),
        "kind": "oracle",
        "sample": "the full %dx%d RGB frame, one doubling (3 planes), FP64 C oracle, OpenMP, %d repeats"
                  % (W, H, runs),
        "seconds": round(dt, 3),
        "cpu_model": host_cpu_model(),
        "logical_cpus": os.cpu_count(),
    }


def cpu_baseline_others(batch_imgs):
    """The FP64 oracle on each of the other workloads, whole: the cascade,
    all 512 images of the batch, forward + hand adjoint of the 16x3x512x512
    batch (the adjoint one plane per thread), and the headline frame's first
    plane on one thread."""
    import ctypes

    import oracle
    from workloads import pixel_art, scene_rgb, to_planar_f32

    out = {}
    cores = host_threads()
    plane = to_planar_f32(scene_rgb(1080, 1920, seed=0))[0].astype(np.float64)
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        oracle.zoom2x(plane)
        dt = time.perf_counter() - t0
        gomp.omp_set_num_threads(cores)
        out["one_core_1080p"] = {"value": round(4 * plane.size / dt / 1e6, 3), "unit": "output Mpix/s (one plane)",
                                 "cores": 1, "seconds": round(dt, 3)}
    except OSError as e:
        out["one_core_1080p"] = {"error": str(e)}
    pa = pixel_art(256, 256, seed=1).transpose(2, 0, 1).astype(np.float64) / 255.0
    t0 = time.perf_counter()
    oracle.cascade(pa, 3)
    dt = time.perf_counter() - t0
    out["cascade_256_x8"] = {"value": round(2048 * 2048 / dt / 1e6, 3), "unit": "output Mpix/s", "cores": cores,
                             "seconds": round(dt, 3), "sample": "the whole workload (3 levels, FP64 intermediates)"}
    log("cpu baseline: 512 images ...")
    t0 = time.perf_counter()
    for im in batch_imgs:
        oracle.zoom2x(np.transpose(im, (2, 0, 1)).astype(np.float64) / 255.0)
    dt = time.perf_counter() - t0
    opx = sum(4 * im.shape[0] * im.shape[1] for im in batch_imgs)
    out["batched_512"] = {"value": round(opx / dt / 1e6, 3), "unit": "output Mpix/s", "cores": cores,
                          "seconds": round(dt, 3), "sample": "all %d images" % len(batch_imgs)}
    log("cpu baseline: forward + adjoint of 16x3x512x512 ...")
    x = np.stack([to_planar_f32(scene_rgb(512, 512, seed=100 + i, n_polygons=20)) for i in range(16)]).astype(np.float64)
    g = np.random.default_rng(0).standard_normal((16, 3, 1024, 1024))
    t0 = time.perf_counter()
    oracle.zoom2x(x)
    oracle.backward(x, g)
    dt = time.perf_counter() - t0
    out["fwd_bwd_16x3x512"] = {"value": round(16 * 1024 * 1024 / dt / 1e6, 3), "unit": "output Mpix/s",
                               "cores": cores, "seconds": round(dt, 3),
                               "sample": "the whole batch (forward: OpenMP over rows; hand adjoint: one plane per "
                                         "thread)"}
    return out


def copy_calibration(torch, dev):
    """Three plain 256 MiB device copies: the reference for the HBM byte counters."""
    a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 3 x %d bytes read + written" % (a.numel() * 4))


def zoom_to_extra(wz, torch, x, dev, steps):
    """Zoom to any size, 1080p RGB f32 -> 5760x3240 (scale 3): two doublings
    to the nested 7679x4319 grid, then the tensor resampler (Section 3.3);
    the resampler alone is also timed on a grid of that size."""
    H, W = x.shape[-2:]
    OH3, OW3 = 3 * H, 3 * W
    ws_zt = torch.empty(wz.zoom_to_workspace_bytes(x, OH3, OW3), dtype=torch.uint8, device=dev)
    ms_zt = timed(lambda: wz.zoom_to(x, OH3, OW3, workspace=ws_zt), steps, 20, torch)
    xg = torch.rand((3, 4 * (H - 1) + 1, 4 * (W - 1) + 1), device=dev)
    ws_rs = torch.empty(max(1, wz.resample_workspace_bytes(xg, OH3, OW3)), dtype=torch.uint8, device=dev)
    ms_rs = timed(lambda: wz.resample(xg, OH3, OW3, workspace=ws_rs), steps, 20, torch)
    rs_bytes = 4 * (xg.numel() + 3 * OH3 * OW3)
    log("zoom_to 1080p -> 5760x3240: %.4f ms (resample stage %.4f ms)" % (ms_zt, ms_rs))
    return {"ms": round(ms_zt, 4), "Mpix_per_s": round(OH3 * OW3 / (ms_zt * 1e-3) / 1e6, 1),
            "resample_stage_ms": round(ms_rs, 4),
            "resample_stage_GBps_algorithmic": round(rs_bytes / (ms_rs * 1e-3) / 1e9, 1),
            "resample_stage_hbm_frac": round(rs_bytes / (ms_rs * 1e-3) / 8e12, 3),
            "resample_stage_algorithmic_bytes": rs_bytes}


def fwd_bwd_batch(torch, dev):
    """The differentiation workload: 16 polygon scenes of 3x512x512 float32
    (seeds 100..115), a standard-normal dL/dU and the forward's output."""
    from workloads import scene_rgb, to_planar_f32

    xb = torch.tensor(np.stack([to_planar_f32(scene_rgb(512, 512, seed=100 + i, n_polygons=20))
                                for i in range(16)]), device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    gy = torch.randn((16, 3, 1024, 1024), device=dev, generator=gen)
    return xb, gy, torch.empty_like(gy)


def cascade_extra(wz, torch, dev, steps, warmup):
    """256^2 RGB pixel art (uint8 HWC), three doublings to 2048^2 uint8 HWC
    (float32 intermediates), from a HIP graph and launched directly."""
    from workloads import pixel_art

    pa = pixel_art(256, 256, seed=1)
    xp = torch.tensor(pa, device=dev).permute(2, 0, 1)
    ws = torch.empty(wz.cascade_workspace_bytes(xp, 3), dtype=torch.uint8, device=dev)
    out = torch.empty((2048, 2048, 3), dtype=torch.uint8, device=dev).permute(2, 0, 1)

    def casc():
        wz.zoom2x_cascade(xp, 3, workspace=ws, out=out)

    casc()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        casc()
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(g):
        casc()
    ms_g = timed(g.replay, steps, warmup, torch)
    ms_e = timed(casc, steps, warmup, torch)
    log("cascade: graph %.4f ms eager %.4f ms" % (ms_g, ms_e))
    return {"ms_graph": round(ms_g, 5), "ms_eager": round(ms_e, 5),
            "Mpix_per_s_graph": round(2048 * 2048 / (ms_g * 1e-3) / 1e6, 1),
            "Mpix_per_s_eager": round(2048 * 2048 / (ms_e * 1e-3) / 1e6, 1)}


def only_fwd_bwd(wz, torch, dev, steps, warmup):
    xb, gy, yb = fwd_bwd_batch(torch, dev)

    def fwdbwd():
        wz.zoom2x_(xb, yb)
        wz.zoom2x_backward(xb, gy)

    ms = timed(fwdbwd, steps, warmup, torch)
    return {"workload": "forward + adjoint, 16x3x512x512 float32", "ms_fwd_bwd": round(ms, 4),
            "Mpix_per_s_fwd_bwd": round(16 * 1024 * 1024 / (ms * 1e-3) / 1e6, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # The GPU clock ramps up over the first tens of milliseconds of sustained
    # load (a 1080p doubling takes ~46 us from idle, ~41 us once warm): the
    # default warm-up (~0.13 s of launches) reaches the steady clock first.
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=3000)
    ap.add_argument("--only-main", action="store_true", help="time only the headline kernel (for profilers)")
    ap.add_argument("--only-zoom-to", action="store_true",
                    help="time only zoom_to 1080p -> 5760x3240 and its resampler (for profilers)")
    ap.add_argument("--only-u8", action="store_true",
                    help="time only the same 1080p frame as uint8 HWC -> uint8 HWC (for profilers)")
    ap.add_argument("--only-fwd-bwd", action="store_true",
                    help="time only forward + adjoint of the 16x3x512^2 float32 batch (for profilers)")
    ap.add_argument("--only-cascade", action="store_true",
                    help="time only the 256^2 pixel-art cascade of three doublings (for profilers)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2312_00229_amd as wz
    from workloads import batch, batch_shapes, pixel_art, scene_rgb, to_planar_f32

    special = args.only_u8 or args.only_fwd_bwd or args.only_zoom_to or args.only_main or args.only_cascade
    if not special:
        # the 512 uneven images (polygon scenes, seeds 2000 + i), generated in
        # worker processes before anything touches the GPU
        log("generating the 512 batch images ...")
        t0 = time.perf_counter()
        batch_imgs = batch(512, seed=2, workers=max(1, min(16, os.cpu_count() or 1)))
        log("generated in %.1f s" % (time.perf_counter() - t0))

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # ---------------- headline: 1080p RGB fp32 -> 2160p ----------------
    H, W = 1080, 1920
    img = scene_rgb(H, W, seed=0)
    planar = to_planar_f32(img)
    x = torch.tensor(planar, device=dev)
    y = torch.empty((3, 2 * H, 2 * W), dtype=torch.float32, device=dev)
    if args.only_u8:
        if args.copy_calib:
            copy_calibration(torch, dev)
        x8 = torch.tensor(img, device=dev).permute(2, 0, 1)
        y8 = torch.empty((2 * H, 2 * W, 3), dtype=torch.uint8, device=dev).permute(2, 0, 1)
        ms8 = timed(lambda: wz.zoom2x_(x8, y8), args.steps, args.warmup, torch)
        print(json.dumps({"workload": "zoom2x 1920x1080 RGB uint8 HWC -> 3840x2160 uint8 HWC", "ms": round(ms8, 5),
                          "Mpix_per_s": round(4 * H * W / (ms8 * 1e-3) / 1e6, 1)}), flush=True)
        return
    if args.only_fwd_bwd:
        print(json.dumps(only_fwd_bwd(wz, torch, dev, args.steps, min(args.warmup, 300))), flush=True)
        return
    if args.only_cascade:
        print(json.dumps(cascade_extra(wz, torch, dev, args.steps, args.warmup)), flush=True)
        return
    if args.only_zoom_to:
        if args.copy_calib:
            copy_calibration(torch, dev)
        print(json.dumps(zoom_to_extra(wz, torch, x, dev, args.steps)), flush=True)
        return
    spin = clock_spinup(lambda: wz.zoom2x_(x, y), torch)
    log("clock spin-up: %d launches in %.2f s (last %.4f ms)" % (spin["launches"], spin["seconds"],
                                                                 spin["last_chunk_ms"]))
    log("headline: zoom2x RGB fp32 %dx%d, steps %d warmup %d" % (W, H, args.steps, args.warmup))
    ms = timed(lambda: wz.zoom2x_(x, y), args.steps, args.warmup, torch)
    out_px = 4 * H * W
    value = out_px / (ms * 1e-3) / 1e6
    alg_bytes = 3 * H * W * 4 + 3 * 4 * H * W * 4
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    alg_flops = FLOPS_PER_QUAD * 3 * H * W
    tflops = alg_flops / (ms * 1e-3) / 1e12
    traffic = measured_traffic()
    rows, cols, tail = wz.launch_shape(x)
    result = {
        "metric": "output Mpix/s + % HBM roofline (2x WENO zoom, RGB fp32); fwd+bwd Mpix/s",
        "value": round(value, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        # before the W warm-up steps: launches until the GPU holds its sustained clock
        "clock_spinup": spin,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "zoom2x 1920x1080 RGB fp32 planar -> 3840x2160, polygon scene (seed 0)",
            "launch": {"rows_per_strip": rows, "cols_per_lane": cols, "tail_rows": tail},
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(tflops, 2),
            "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(tflops / ALU_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "algorithmic_flops_per_launch": alg_flops,
            # the part's FP32 vector peak counting packed (two-wide) FP32 instructions,
            # which the library does not use
            "peak_with_packed_fp32": ALU_PEAK_PACKED_TFLOPS,
            "frac_of_packed_peak": round(tflops / ALU_PEAK_PACKED_TFLOPS, 4),
        },
        "hbm_roofline": {
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "algorithmic_bytes_per_launch": alg_bytes,
        },
    }
    if args.copy_calib:
        copy_calibration(torch, dev)
    if args.only_main:
        print(json.dumps(result), flush=True)
        return

    extras = {}
    # The other workloads are timed with at least 300 warm-up and 300 timed
    # calls whatever the headline's K and W (a few dozen calls of a
    # microsecond-scale launch are mostly noise), fewer for the long ones.
    xsteps, xwarm = max(args.steps, 300), max(args.warmup, 300)
    # ---------------- the headline launch replayed from a HIP graph ----------------
    # (no host launch cost between kernels; the back-to-back stream launches
    # above hide it already, which the two figures show)
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        wz.zoom2x_(x, y)
    torch.cuda.current_stream().wait_stream(gs)
    gh = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gh):
        for _ in range(20):
            wz.zoom2x_(x, y)
    ms_gh = timed(gh.replay, xsteps // 20, xwarm // 20, torch) / 20
    extras["headline_graph_replay"] = {"ms": round(ms_gh, 5), "Mpix_per_s": round(out_px / (ms_gh * 1e-3) / 1e6, 1),
                                       "launches_per_graph": 20}
    log("headline from a graph: %.4f ms per launch" % ms_gh)
    del gh

    # ---------------- a frame whose working set exceeds the 256 MB MALL ----------------
    H8, W8 = 4320, 7680
    x8k = torch.tensor(to_planar_f32(scene_rgb(H8, W8, seed=3, n_polygons=40)), device=dev)
    y8k = torch.empty((3, 2 * H8, 2 * W8), dtype=torch.float32, device=dev)
    ms8k = timed(lambda: wz.zoom2x_(x8k, y8k), max(30, args.steps // 10), 30, torch)
    px8k = 4 * H8 * W8
    extras["zoom2x_rgb_f32_7680x4320"] = {
        "ms": round(ms8k, 4), "Mpix_per_s": round(px8k / (ms8k * 1e-3) / 1e6, 1),
        "GBps_algorithmic": round(15 * px8k / (ms8k * 1e-3) / 1e9, 1),
        "TFLOPs_algorithmic": round(FLOPS_PER_QUAD * 3 * H8 * W8 / (ms8k * 1e-3) / 1e12, 2)}
    log("7680x4320 RGB fp32: %.4f ms" % ms8k)
    del x8k, y8k

    # ---------------- uint8 HWC variant of the same frame ----------------
    x8 = torch.tensor(img, device=dev).permute(2, 0, 1)
    y8 = torch.empty((2 * H, 2 * W, 3), dtype=torch.uint8, device=dev).permute(2, 0, 1)
    ms8 = timed(lambda: wz.zoom2x_(x8, y8), xsteps, xwarm, torch)
    extras["u8_hwc_1080p"] = {"ms": round(ms8, 5), "Mpix_per_s": round(out_px / (ms8 * 1e-3) / 1e6, 1),
                              "GBps_algorithmic": round((3 * H * W + 12 * H * W) / (ms8 * 1e-3) / 1e9, 1)}
    log("u8 HWC 1080p: %.4f ms" % ms8)

    # ---------------- batched: 512 uneven images ----------------
    shapes = batch_shapes(512, seed=2)
    imgs = batch_imgs
    xs = [torch.tensor(im, device=dev).permute(2, 0, 1) for im in imgs]
    ys = [torch.empty((2 * h, 2 * w, 3), dtype=torch.uint8, device=dev).permute(2, 0, 1) for (h, w) in shapes]
    # the persistent plan takes the autotuned strip shape (plans capture the
    # launch configuration when made); the per-image loop runs the plain
    # kernel in its automatic configuration
    from paper_2312_00229_amd.autotune import tune_batched

    b_rows, b_cols, _ = tune_batched(xs, ys, reps=3, use_cache=False)
    plan = wz.BatchedZoom(xs, ys)
    wz.set_launch_config(0, 0)
    bsteps = max(10, xsteps // 20)
    ms_b = timed(plan.run, bsteps, 2, torch)
    ys_loop = [torch.empty_like(t) for t in ys]

    def loop():
        for a, b in zip(xs, ys_loop):
            wz.zoom2x_(a, b)

    ms_l = timed(loop, bsteps, 2, torch)
    identical = all(torch.equal(a, b) for a, b in zip(ys, ys_loop))
    del ys_loop
    bpx = sum(4 * h * w for h, w in shapes)
    extras["batched_512_u8"] = {
        "ms_persistent": round(ms_b, 4), "ms_launch_loop": round(ms_l, 4),
        "Mpix_per_s_persistent": round(bpx / (ms_b * 1e-3) / 1e6, 1),
        "Mpix_per_s_launch_loop": round(bpx / (ms_l * 1e-3) / 1e6, 1),
        "tuned_launch": {"rows_per_strip": b_rows, "cols_per_lane": b_cols},
        "outputs_identical_to_loop": identical,
        "content": "polygon scenes (seeds 2000 + i), sizes U{32..1024}^2 (seed 2)",
    }
    log("batched: persistent %.3f ms (rows %d, cols %d), loop %.3f ms, identical %s"
        % (ms_b, b_rows, b_cols, ms_l, identical))

    extras["cascade_256_x8_u8"] = cascade_extra(wz, torch, dev, xsteps, xwarm)

    extras["zoom_to_rgb_f32_1080p_to_5760x3240"] = zoom_to_extra(wz, torch, x, dev, max(30, args.steps // 10))

    # ---------------- forward + backward, 16 x 3 x 512 x 512 ----------------
    try:
        xb, gy, yb = fwd_bwd_batch(torch, dev)

        def fwd():
            wz.zoom2x_(xb, yb)

        def fwdbwd():
            wz.zoom2x_(xb, yb)
            wz.zoom2x_backward(xb, gy)

        def fwdbwd_loop():   # the same work as 16 per-image calls
            for i in range(16):
                wz.zoom2x_(xb[i], yb[i])
                wz.zoom2x_backward(xb[i], gy[i])

        ms_f = timed(fwd, xsteps, 30, torch)
        ms_fb = timed(fwdbwd, xsteps // 3, 30, torch)
        ms_fbl = timed(fwdbwd_loop, max(30, args.steps // 10), 3, torch)
        gx_batch = wz.zoom2x_backward(xb, gy)
        same = all(torch.equal(gx_batch[i], wz.zoom2x_backward(xb[i], gy[i])) for i in range(16))
        opx = 16 * 1024 * 1024
        extras["fwd_bwd_16x3x512"] = {"ms_fwd": round(ms_f, 4), "ms_fwd_bwd": round(ms_fb, 4),
                                      "ms_fwd_bwd_per_image_loop": round(ms_fbl, 4),
                                      "Mpix_per_s_fwd": round(opx / (ms_f * 1e-3) / 1e6, 1),
                                      "Mpix_per_s_fwd_bwd": round(opx / (ms_fb * 1e-3) / 1e6, 1),
                                      "Mpix_per_s_fwd_bwd_per_image_loop": round(opx / (ms_fbl * 1e-3) / 1e6, 1),
                                      "gradients_identical_to_loop": same}
        log("fwd %.3f ms, fwd+bwd %.3f ms (per-image loop %.3f ms)" % (ms_f, ms_fb, ms_fbl))
    except wz.WenoError as e:
        extras["fwd_bwd_16x3x512"] = {"error": str(e)}

    result["extras"] = extras
    if not args.no_cpu:
        log("cpu baseline (FP64 oracle) ...")
        result["cpu_baseline"] = cpu_baseline(planar)
        result["cpu_baseline"]["others"] = cpu_baseline_others(imgs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
