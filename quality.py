#!/usr/bin/env python3
"""Image-quality harness: the paper's upsampling protocol on synthetic images.

Protocol (Section 4, natural-image tests): the reference image is cropped so
that (size - 1) is divisible by the scale factor d, downsampled to
(size - 1)/d + 1 samples per axis, and upsampled back to the reference size
d (down - 1) + 1 by each method; PSNR and MSSIM compare the result with the
reference.  Downsampling keeps every d-th pixel (the paper gives the sizes
but not the filter; nested grid nodes keep the reference's samples).

Methods: WD-WENO (k doublings on nested grids, d = 2^k), tensor WENO (the
separable resampler of eq. tensor, the paper's comparator in its vector-image
table), and torch bicubic / bilinear interpolation with aligned corners.

Metrics: PSNR on the [0,1] scale; MSSIM = mean of the SSIM map of Wang et
al. (11x11 Gaussian window, sigma 1.5, K1 = 0.01, K2 = 0.03, dynamic range 1),
per channel, averaged over channels.

Inputs are the synthetic stand-ins of workloads.py (polygon scenes at the
photo suite's 768 x 512 size, pixel art); the paper's images are not
available, so its table values are context only.

Usage: python quality.py [--d 2 4] [--images 4]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import torch
import torch.nn.functional as F

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def psnr(ref: torch.Tensor, img: torch.Tensor) -> float:
    mse = float(torch.mean((ref.double() - img.double()) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(1.0 / mse)


def _gauss_window(size=11, sigma=1.5, dtype=torch.float64, device="cpu"):
    x = torch.arange(size, dtype=dtype, device=device) - (size - 1) / 2.0
    g = torch.exp(-(x * x) / (2 * sigma * sigma))
    g = g / g.sum()
    return g[:, None] * g[None, :]


def ssim_map(a: torch.Tensor, b: torch.Tensor, size=11, sigma=1.5, k1=0.01, k2=0.03, L=1.0) -> torch.Tensor:
    """SSIM map of two (C, H, W) images ('valid' window positions only)."""
    a = a.double().unsqueeze(1)
    b = b.double().unsqueeze(1)
    w = _gauss_window(size, sigma, device=a.device)[None, None]
    mu_a = F.conv2d(a, w)
    mu_b = F.conv2d(b, w)
    saa = F.conv2d(a * a, w) - mu_a * mu_a
    sbb = F.conv2d(b * b, w) - mu_b * mu_b
    sab = F.conv2d(a * b, w) - mu_a * mu_b
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    return ((2 * mu_a * mu_b + c1) * (2 * sab + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) * (saa + sbb + c2))


def mssim(ref: torch.Tensor, img: torch.Tensor) -> float:
    return float(ssim_map(ref, img).mean())


def protocol(img_chw: torch.Tensor, d: int):
    """img_chw: float (C, H, W) on [0,1], on the GPU.  Returns {method: (psnr, mssim)}."""
    import paper_2312_00229_amd as wz

    k = int(round(math.log2(d)))
    assert 2 ** k == d, "d must be a power of two"
    C, H, W = img_chw.shape
    h_ref = (H - 1) // d * d + 1
    w_ref = (W - 1) // d * d + 1
    ref = img_chw[:, :h_ref, :w_ref].contiguous()
    down = ref[:, ::d, ::d].contiguous()
    outs = {
        "wd_weno": wz.zoom_to(down, h_ref, w_ref),
        "tensor_weno": wz.resample(down, h_ref, w_ref),
        "bicubic": F.interpolate(down[None], size=(h_ref, w_ref), mode="bicubic", align_corners=True)[0],
        "bilinear": F.interpolate(down[None], size=(h_ref, w_ref), mode="bilinear", align_corners=True)[0],
    }
    res = {}
    for name, out in outs.items():
        out = out.clamp(0.0, 1.0)
        res[name] = (round(psnr(ref, out), 4), round(mssim(ref, out), 4))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--d", type=int, nargs="+", default=[2, 4])
    ap.add_argument("--images", type=int, default=4)
    args = ap.parse_args()
    import numpy as np

    from workloads import pixel_art, scene_rgb, to_planar_f32

    sets = {
        "polygon scenes 768x512": [to_planar_f32(scene_rgb(512, 768, seed=300 + i)) for i in range(args.images)],
        "pixel art 256x256": [to_planar_f32(pixel_art(256, 256, seed=400 + i)) for i in range(args.images)],
    }
    table = {}
    for set_name, imgs in sets.items():
        for d in args.d:
            acc = {}
            for im in imgs:
                r = protocol(torch.tensor(im, device="cuda"), d)
                for m, (p, s) in r.items():
                    acc.setdefault(m, []).append((p, s))
            table["%s, d=%d" % (set_name, d)] = {
                m: {"psnr": round(float(np.mean([v[0] for v in vals])), 3),
                    "mssim": round(float(np.mean([v[1] for v in vals])), 4)}
                for m, vals in acc.items()
            }
    print(json.dumps(table, indent=1))


if __name__ == "__main__":
    main()
