"""Pins of the quality harness's metrics (CPU): PSNR from its definition,
SSIM against a per-window brute force of Wang et al.'s formula."""
import math

import numpy as np
import torch

import quality


def test_psnr_definition():
    a = torch.zeros(3, 8, 8, dtype=torch.float64)
    b = torch.full((3, 8, 8), 0.1, dtype=torch.float64)
    assert abs(quality.psnr(a, b) - 20.0) <= 1e-9      # 10 log10(1 / 0.01)
    assert quality.psnr(a, a) == math.inf


def _ssim_brute(a, b, size=11, sigma=1.5, k1=0.01, k2=0.03):
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-x * x / (2 * sigma * sigma))
    w = np.outer(g, g)
    w /= w.sum()
    H, W = a.shape
    out = np.empty((H - size + 1, W - size + 1))
    c1, c2 = k1 ** 2, k2 ** 2
    for i in range(out.shape[0]):
        for j in range(out.shape[1]):
            pa = a[i:i + size, j:j + size]
            pb = b[i:i + size, j:j + size]
            ma, mb = (w * pa).sum(), (w * pb).sum()
            va = (w * (pa - ma) ** 2).sum()
            vb = (w * (pb - mb) ** 2).sum()
            cab = (w * (pa - ma) * (pb - mb)).sum()
            out[i, j] = ((2 * ma * mb + c1) * (2 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2))
    return out


def test_ssim_matches_brute_force():
    rng = np.random.default_rng(0)
    a = rng.random((16, 19))
    b = np.clip(a + 0.1 * rng.standard_normal(a.shape), 0, 1)
    got = quality.ssim_map(torch.tensor(a)[None], torch.tensor(b)[None])[0, 0].numpy()
    assert np.abs(got - _ssim_brute(a, b)).max() <= 1e-12


def test_ssim_identity_and_symmetry():
    rng = np.random.default_rng(1)
    a = torch.tensor(rng.random((3, 20, 20)))
    b = torch.tensor(rng.random((3, 20, 20)))
    assert abs(quality.mssim(a, a) - 1.0) <= 1e-12
    assert abs(quality.mssim(a, b) - quality.mssim(b, a)) <= 1e-12
    assert quality.mssim(a, b) < 1.0
