"""Seeded random cases across the parameter space, each against the FP64
oracle: sizes from 1 to 300, batches of one or two, one or three channels,
planar or channel-interleaved layouts, float32 or uint8 at either end, beta
in {1, 1.5, 2}, automatic or forced launch shapes; the adjoint on float32;
the resampler up and down.  The bars are those of the targeted tests:
float32 within 1e-5 of max(1, |ref|), uint8 codes equal up to counted
rounding ties, the adjoint within the bar of conftest.check_adjoint."""
import numpy as np
import pytest
import torch

import oracle
from conftest import check_adjoint, check_u8
from oracle import resample as R

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.default_rng(seed)
    h = int(rng.integers(1, 301)) if rng.random() < 0.8 else int(rng.integers(1, 8))
    w = int(rng.integers(1, 301)) if rng.random() < 0.8 else int(rng.integers(1, 8))
    return rng, h, w, int(rng.integers(1, 3)), [1, 3][int(rng.integers(0, 2))]


def _tensor(a, interleaved):
    """(N, C, H, W) numpy array -> device tensor, planar or with the channel
    dim innermost in memory (NHWC viewed as NCHW)."""
    if interleaved:
        return torch.tensor(np.ascontiguousarray(np.transpose(a, (0, 2, 3, 1))), device="cuda").permute(0, 3, 1, 2)
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _empty(shape, dtype, interleaved):
    n, c, h, w = shape
    if interleaved:
        return torch.empty((n, h, w, c), dtype=dtype, device="cuda").permute(0, 3, 1, 2)
    return torch.empty(shape, dtype=dtype, device="cuda")


@pytest.mark.parametrize("seed", range(40))
def test_random_forward(gpu, seed):
    rng, h, w, n, c = _case(seed)
    in_u8, out_u8 = bool(rng.random() < 0.5), bool(rng.random() < 0.5)
    interleaved = c == 3 and bool(rng.random() < 0.5)
    beta = [1.0, 1.5, 2.0][int(rng.integers(0, 3))]
    cfg = [(0, 0), (4, 1), (8, 2), (27, 2), (13, 1)][int(rng.integers(0, 5))]
    if in_u8:
        codes = rng.integers(0, 256, size=(n, c, h, w)).astype(np.uint8)
        x = _tensor(codes, interleaved)
        V = codes.astype(np.float64) / 255.0
    else:
        V32 = rng.random((n, c, h, w), dtype=np.float32)
        x = _tensor(V32, interleaved)
        V = V32.astype(np.float64)
    out = _empty((n, c, 2 * h, 2 * w), torch.uint8 if out_u8 else torch.float32, interleaved)
    try:
        gpu.set_launch_config(*cfg)
        gpu.zoom2x_(x, out, beta=beta)
    finally:
        gpu.set_launch_config(0, 0)
    ref = oracle.zoom2x(V, beta=beta)
    got = out.cpu().numpy()
    what = (seed, h, w, n, c, in_u8, out_u8, interleaved, beta, cfg)
    if out_u8:
        check_u8(got, ref, str(what), max_tie_frac=5e-5)
    else:
        assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), what


@pytest.mark.parametrize("seed", range(100, 112))
def test_random_backward(gpu, seed):
    rng, h, w, n, c = _case(seed)
    h, w = min(h, 120), min(w, 160)
    beta = [1.0, 1.5, 2.0][int(rng.integers(0, 3))]
    rows = [0, 4, 7, 19][int(rng.integers(0, 4))]
    V = rng.random((n, c, h, w), dtype=np.float32)
    G = rng.standard_normal((n, c, 2 * h, 2 * w)).astype(np.float32)
    try:
        gpu.set_backward_launch_config(rows)
        got = gpu.zoom2x_backward(torch.tensor(V, device="cuda"), torch.tensor(G, device="cuda"),
                                  gpu.Params(beta=beta)).cpu().numpy()
    finally:
        gpu.set_backward_launch_config(0)
    check_adjoint(got, V, G, str((seed, h, w, n, c, beta, rows)), beta=beta)


@pytest.mark.parametrize("seed", range(200, 216))
def test_random_resample(gpu, seed):
    rng, h, w, n, c = _case(seed)
    oh = int(rng.integers(1, 2 * h + 40))
    ow = int(rng.integers(1, 2 * w + 40))
    V = rng.random((n, c, h, w), dtype=np.float32)
    got = gpu.resample(torch.tensor(V, device="cuda"), oh, ow).cpu().numpy()
    ref = R.tensor_resample(V.astype(np.float64), oh, ow)
    assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), (seed, h, w, n, c, oh, ow)
