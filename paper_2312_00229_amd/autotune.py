"""Launch-configuration autotuner for the forward kernels.

The knobs are the strip height (input rows one wave walks, `rows_per_strip`)
and the columns of quads each lane owns (`cols_per_lane`, 1 or 2).  Taller
strips amortise the 9-row pipeline fill, shorter ones give more waves to fill
the 256 CUs; two columns per lane halve the halo overhead per wave but double
its registers.  Every configuration computes every quad with the same
arithmetic, so outputs are bit-identical across configurations; the tuner
checks that too (a cheap guard against a broken configuration).  The
automatic configuration (the library's cost model, which alone can add
one-column tail strips) is one of the candidates, recorded as (0, 0), so
tuning never leaves a shape slower than the default.

`tune_backward` picks the adjoint kernel's strip height (its own setting;
it always runs one column per lane; the automatic height is a candidate,
recorded as 0), checking that the gradient stays bit-identical.  `tune_batched` does the same for a
batched plan (the persistent kernel over a
work queue): plans capture the configuration when they are made, so it builds
one plan per candidate, checks that all outputs stay bit-identical and leaves
the fastest configuration applied for the plans made afterwards.

Results are cached in a JSON file (env WENO_TUNE_CACHE, default
~/.cache/weno_zoom_tune.json) keyed by device name, dtypes, channel count and
a size class of the image (of the batch's total size for batched plans).
Before timing, the GPU is kept busy for a moment: its clock ramps up over the
first tens of milliseconds of load, which would otherwise penalise the
configurations measured first.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import (BatchedZoom, get_backward_launch_config, get_launch_config, set_backward_launch_config,
               set_launch_config, zoom2x_, zoom2x_backward)

ROWS = (8, 12, 16, 20, 24, 27, 32, 40, 48, 64, 96)
ROWS_BATCHED = (16, 24, 32, 48, 64, 96, 128, 192)
ROWS_BACKWARD = (16, 24, 32, 48, 64, 96, 128, 171, 256)
COLS = (1, 2)


def _cache_path() -> str:
    return os.environ.get("WENO_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "weno_zoom_tune.json"))


def _key(x: torch.Tensor, out: torch.Tensor) -> str:
    h, w = x.shape[-2:]
    planes = int(x.numel() // (h * w))
    cls = "%dx%d" % (2 ** max(0, round(math.log2(max(h, 1)))), 2 ** max(0, round(math.log2(max(w, 1)))))
    return "%s|%s->%s|p%d|%s" % (torch.cuda.get_device_name(x.device), x.dtype, out.dtype, planes, cls)


def _warm(fn, seconds: float = 0.1):
    """Keep the GPU busy with fn() for about `seconds` (clock ramp-up)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def _load_cache(use_cache: bool):
    path = _cache_path()
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}
    return {}


def _store_cache(cache):
    path = _cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, path)


def _time(fn, reps: int) -> float:
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(x: torch.Tensor, out: torch.Tensor, reps: int = 30, use_cache: bool = True, verbose: bool = False):
    """Pick and apply the fastest (rows_per_strip, cols_per_lane) for zooming x
    into out, (0, 0) being the automatic configuration.  Returns (rows, cols,
    {config: ms})."""
    key = _key(x, out)
    cache = _load_cache(use_cache)
    if use_cache and key in cache:
        rows, cols = cache[key]["best"]
        set_launch_config(rows, cols)
        return rows, cols, cache[key].get("times", {})
    prev = get_launch_config()
    times = {}
    ref = None
    _warm(lambda: zoom2x_(x, out))
    for rows, cols in [(0, 0)] + [(r, c) for c in COLS for r in ROWS]:
        set_launch_config(rows, cols)
        zoom2x_(x, out)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            set_launch_config(*prev)
            raise RuntimeError("launch configuration (%d, %d) changed the result" % (rows, cols))
        times["%d,%d" % (rows, cols)] = _time(lambda: zoom2x_(x, out), reps)
        if verbose:
            print("rows %4d cols %d: %.4f ms" % (rows, cols, times["%d,%d" % (rows, cols)]), flush=True)
    best = min(times, key=times.get)
    rows, cols = (int(t) for t in best.split(","))
    set_launch_config(rows, cols)
    if use_cache:
        cache[key] = {"best": [rows, cols], "times": times}
        _store_cache(cache)
    return rows, cols, times


def _batched_key(xs, outs) -> str:
    px = sum(int(x.numel()) for x in xs)
    return "batched|%s|%s->%s|n%d|px2^%d" % (torch.cuda.get_device_name(xs[0].device), xs[0].dtype, outs[0].dtype,
                                             len(xs), round(math.log2(max(px, 1))))


def tune_batched(xs, outs, params=None, reps: int = 5, use_cache: bool = True, verbose: bool = False):
    """Pick and apply the fastest (rows_per_strip, cols_per_lane) for a batched
    plan zooming xs into outs; plans made afterwards capture it.  Returns
    (rows, cols, {config: ms})."""
    key = _batched_key(xs, outs)
    cache = _load_cache(use_cache)
    if use_cache and key in cache:
        rows, cols = cache[key]["best"]
        set_launch_config(rows, cols)
        return rows, cols, cache[key].get("times", {})
    prev = get_launch_config()
    times = {}
    ref = None
    for cols in COLS:
        for rows in ROWS_BATCHED:
            set_launch_config(rows, cols)
            plan = BatchedZoom(xs, outs, params)
            if ref is None:
                _warm(plan.run)
            plan.run()
            torch.cuda.synchronize()
            if ref is None:
                ref = [o.clone() for o in outs]
            elif not all(torch.equal(o, r) for o, r in zip(outs, ref)):
                set_launch_config(*prev)
                raise RuntimeError("launch configuration (%d, %d) changed the result" % (rows, cols))
            times["%d,%d" % (rows, cols)] = _time(plan.run, reps)
            if verbose:
                print("batched rows %4d cols %d: %.4f ms" % (rows, cols, times["%d,%d" % (rows, cols)]), flush=True)
    del ref
    best = min(times, key=times.get)
    rows, cols = (int(t) for t in best.split(","))
    set_launch_config(rows, cols)
    if use_cache:
        cache[key] = {"best": [rows, cols], "times": times}
        _store_cache(cache)
    return rows, cols, times


def tune_backward(x, grad_y, reps: int = 5, use_cache: bool = True, verbose: bool = False):
    """Pick and apply the fastest strip height for the adjoint of zooming x
    (gradient grad_y of the output), 0 being the automatic height; the
    forward's configuration is left alone.  Returns (rows, {rows: ms})."""
    h, w = x.shape[-2:]
    planes = int(x.numel() // (h * w))
    cls = "%dx%d" % (2 ** max(0, round(math.log2(max(h, 1)))), 2 ** max(0, round(math.log2(max(w, 1)))))
    key = "backward|%s|p%d|%s" % (torch.cuda.get_device_name(x.device), planes, cls)
    cache = _load_cache(use_cache)
    if use_cache and key in cache:
        rows = cache[key]["best"]
        set_backward_launch_config(rows)
        return rows, cache[key].get("times", {})
    prev = get_backward_launch_config()
    times = {}
    ref = None
    for rows in (0,) + ROWS_BACKWARD:
        set_backward_launch_config(rows)
        if ref is None:
            _warm(lambda: zoom2x_backward(x, grad_y))
        g = zoom2x_backward(x, grad_y)
        torch.cuda.synchronize()
        if ref is None:
            ref = g
        elif not torch.equal(g, ref):
            set_backward_launch_config(prev)
            raise RuntimeError("adjoint strip height %d changed the gradient" % rows)
        times[str(rows)] = _time(lambda: zoom2x_backward(x, grad_y), reps)
        if verbose:
            print("backward rows %4d: %.4f ms" % (rows, times[str(rows)]), flush=True)
    best = min(times, key=times.get)
    rows = int(best)
    set_backward_launch_config(rows)
    if use_cache:
        cache[key] = {"best": rows, "times": times}
        _store_cache(cache)
    return rows, times
