"""Seeded random cases across the parameter space, each against the FP64
oracle: sizes from 1 to 300, batches of one or two, one or three channels,
planar or channel-interleaved layouts, float32 or uint8 at either end, beta
in {1, 1.5, 2}, automatic or forced launch shapes (and automatic shapes over
many planes and widths, one-column tail strips among them, against a forced
one); the adjoint on float32;
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


def _has_tail(w):
    """The width leaves a last strip column one one-column strip can hold."""
    own2, own1 = 118, 55
    sx = -(-w // own2)
    return sx >= 2 and w - (sx - 1) * own2 <= own1


@pytest.mark.parametrize("seed", range(300, 330))
def test_random_automatic_launch_shapes(gpu, seed):
    # Automatic launch shapes over many planes and widths (one-dimensional
    # grids with one-column tail strips among them) against a forced shape
    # without tail strips, bit for bit, and the oracle on the last plane's
    # tail columns.
    rng = np.random.default_rng(seed)
    planes = int(rng.integers(1, 49))
    h = int(rng.integers(4, 400))
    tails = [w for w in range(120, 1200) if _has_tail(w)]
    w = int(rng.choice(tails)) if rng.random() < 0.8 else int(rng.integers(4, 1200))
    u8 = rng.random() < 0.3
    a = rng.random((planes, h, w))
    x = torch.tensor((a * 255).round().astype(np.uint8) if u8 else a.astype(np.float32), device="cuda")
    gpu.set_launch_config(0, 0)
    rows, cols, tail = gpu.launch_shape(x)
    y = gpu.zoom2x(x).cpu().numpy()
    gpu.set_launch_config(16, 1)
    y2 = gpu.zoom2x(x).cpu().numpy()
    gpu.set_launch_config(0, 0)
    print("seed %d: %d x %d x %d %s, shape %s" % (seed, planes, h, w, "u8" if u8 else "f32", (rows, cols, tail)))
    assert np.array_equal(y, y2)
    V = (x[-1].cpu().numpy().astype(np.float64) / 255.0) if u8 else x[-1].cpu().numpy().astype(np.float64)
    c0 = max(0, w - 70)
    ref = oracle.window_zoom2x(V, 0, min(h, 40), c0, w)
    got = y[-1, :2 * min(h, 40), 2 * c0:]
    if u8:
        check_u8(got, ref, "seed %d" % seed)
    else:
        assert np.abs(got - ref).max() <= 1e-5


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
