"""Seeded synthetic inputs shaped like the paper's test material.

This module holds no part of the zooming method: only scene generators and
sample grids.  Both the test-suite (oracle and GPU sides) and the benchmark
draw their inputs from here, with numpy's PCG64 generator (`default_rng`).

  smooth_f / smooth_grid   smooth test function on [0,1]^2 (accuracy runs)
  scene_rgb                polygons over a colour gradient plus noise, the
                           stand-in for natural / vector photographs
  pixel_art                blocky palette image with one-pixel lines, the
                           stand-in for pixel-art inputs
  batch_shapes / batch     many RGB images of uneven sizes
The paper's own images (a photo suite, a vector drawing, pixel-art sprites)
are not available; these scenes only imitate their shapes and structure.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# smooth function on [0,1]^2
# --------------------------------------------------------------------------
def smooth_f(x, y):
    return np.sin(2 * np.pi * x) * np.cos(3 * np.pi * y) + 0.5 * np.exp(
        -20.0 * ((x - 0.4) ** 2 + (y - 0.6) ** 2)
    )


def smooth_grid(n: int, margin: int = 0):
    """f sampled at x_i = i/(n-1), i in [-margin, n+margin) (rows = x)."""
    k = np.arange(-margin, n + margin)
    x = k / (n - 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    return smooth_f(X, Y)


# --------------------------------------------------------------------------
# polygon scene (RGB, uint8, HWC)
# --------------------------------------------------------------------------
def _fill_polygon(img, verts, colour):
    """Even-odd fill of pixel centres inside a closed polygon (in place)."""
    H, W = img.shape[:2]
    ys, xs = verts[:, 0], verts[:, 1]
    r0 = max(int(math.floor(ys.min())), 0)
    r1 = min(int(math.ceil(ys.max())) + 1, H)
    c0 = max(int(math.floor(xs.min())), 0)
    c1 = min(int(math.ceil(xs.max())) + 1, W)
    if r0 >= r1 or c0 >= c1:
        return
    py = np.arange(r0, r1)[:, None] + 0.5
    px = np.arange(c0, c1)[None, :] + 0.5
    inside = np.zeros((r1 - r0, c1 - c0), dtype=bool)
    nv = len(verts)
    for a in range(nv):
        y0, x0 = verts[a]
        y1, x1 = verts[(a + 1) % nv]
        if y0 == y1:
            continue
        crosses = (py >= min(y0, y1)) & (py < max(y0, y1))
        xint = x0 + (py - y0) * (x1 - x0) / (y1 - y0)
        inside ^= crosses & (px < xint)
    img[r0:r1, c0:c1][inside] = colour


def scene_rgb(H: int, W: int, seed: int = 0, n_polygons: int = 40, noise_sigma: float = 2.0) -> np.ndarray:
    """Linear colour gradient along a random angle, `n_polygons` star-shaped
    polygons (3-8 vertices, radius U[0.02, 0.25] min(H, W), constant random
    colours, painted in order), Gaussian noise, clipped and rounded half to
    even.  Returns uint8 (H, W, 3)."""
    rng = np.random.default_rng(seed)
    c_a = rng.uniform(0, 255, 3)
    c_b = rng.uniform(0, 255, 3)
    ang = rng.uniform(0, 2 * np.pi)
    yy, xx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    proj = yy * math.sin(ang) + xx * math.cos(ang)
    t = (proj - proj.min()) / max(proj.max() - proj.min(), 1e-12)
    img = (1 - t)[..., None] * c_a + t[..., None] * c_b
    s = min(H, W)
    for _ in range(n_polygons):
        nv = int(rng.integers(3, 9))
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        radius = rng.uniform(0.02, 0.25) * s
        angles = np.sort(rng.uniform(0, 2 * np.pi, nv))
        radii = radius * rng.uniform(0.3, 1.0, nv)
        verts = np.stack([cy + radii * np.sin(angles), cx + radii * np.cos(angles)], axis=1)
        _fill_polygon(img, verts, rng.uniform(0, 255, 3))
    img = img + rng.normal(0.0, noise_sigma, img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# pixel art (RGB, uint8, HWC)
# --------------------------------------------------------------------------
def pixel_art(H: int = 256, W: int = 256, seed: int = 1, block: int = 8, n_lines: int = 32) -> np.ndarray:
    """16-colour palette; each block x block cell takes a palette colour;
    `n_lines` one-pixel DDA lines (no anti-aliasing) at angles U[0, 180) deg,
    lengths U[16, 256]."""
    rng = np.random.default_rng(seed)
    palette = rng.integers(0, 256, (16, 3)).astype(np.uint8)
    cells = rng.integers(0, 16, ((H + block - 1) // block, (W + block - 1) // block))
    idx = np.repeat(np.repeat(cells, block, axis=0), block, axis=1)[:H, :W]
    img = palette[idx].copy()
    for _ in range(n_lines):
        ang = math.radians(rng.uniform(0, 180))
        length = rng.uniform(16, 256)
        y0, x0 = rng.uniform(0, H), rng.uniform(0, W)
        colour = palette[int(rng.integers(0, 16))]
        steps = int(math.ceil(length))
        for k in range(steps + 1):
            y = int(math.floor(y0 + k * math.sin(ang)))
            x = int(math.floor(x0 + k * math.cos(ang)))
            if 0 <= y < H and 0 <= x < W:
                img[y, x] = colour
    return img


# --------------------------------------------------------------------------
# uneven batches
# --------------------------------------------------------------------------
def batch_shapes(count: int = 512, seed: int = 2, lo: int = 32, hi: int = 1024):
    """(H, W) pairs drawn independently from U{lo..hi}."""
    rng = np.random.default_rng(seed)
    hs = rng.integers(lo, hi + 1, count)
    ws = rng.integers(lo, hi + 1, count)
    return [(int(h), int(w)) for h, w in zip(hs, ws)]


def _scene_job(args):
    h, w, seed, n_polygons = args
    return scene_rgb(h, w, seed=seed, n_polygons=n_polygons)


def batch(count: int = 512, seed: int = 2, lo: int = 32, hi: int = 1024, n_polygons: int = 40, workers: int = 1):
    """Images of `batch_shapes`, content as `scene_rgb` with seed 1000*seed + i
    (generated in `workers` processes when > 1; the same images either way)."""
    jobs = [(h, w, 1000 * seed + i, n_polygons) for i, (h, w) in enumerate(batch_shapes(count, seed, lo, hi))]
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor

        with ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_scene_job, jobs, chunksize=4))
    return [_scene_job(j) for j in jobs]


def to_planar_f32(img_u8: np.ndarray) -> np.ndarray:
    """uint8 (H, W, C) -> float32 (C, H, W) on the [0,1] scale."""
    return np.ascontiguousarray(np.transpose(img_u8, (2, 0, 1)).astype(np.float32) / np.float32(255.0))


def random_plane(n: int, m: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """Small random test planes: 'uniform' [0,1], 'steps' (piecewise constant
    with jumps), 'binary' {0,1} (many exact ties in the weights)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random((n, m))
    if kind == "steps":
        base = rng.random((max(1, n // 4 + 1), max(1, m // 4 + 1)))
        return np.repeat(np.repeat(base, 4, 0), 4, 1)[:n, :m].copy()
    if kind == "binary":
        return (rng.random((n, m)) < 0.5).astype(np.float64)
    raise ValueError(kind)


def two_level_u8(h, w, seed, channels=None):
    """uint8 samples drawn from {96, 112, 128, 144} (multiples of 16): under
    equal weights every interpolated value is a small dyadic fraction on the
    0..255 scale, and many of them lie exactly halfway between two codes, so
    the rounding rule is visible.  (h, w) or (h, w, channels)."""
    rng = np.random.default_rng(seed)
    shape = (h, w) if channels is None else (h, w, channels)
    return (96 + 16 * rng.integers(0, 4, shape)).astype(np.uint8)
