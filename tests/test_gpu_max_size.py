"""Planes at the size limit.  Buffer offsets are 32-bit: every plane spans
less than 2^31 bytes, and idle lanes address 2^31 + a row offset, which must
stay out of range without wrapping.  An 11585 x 11585 float32 plane doubles
to 23170 x 23170 floats (2,147,395,600 bytes, just under 2^31); a
23170 x 23170 uint8 plane doubles to the same byte count.  Sampled windows
-- the four corners, the last rows and columns, interior points -- are
checked against the oracle on windows of the input, in the automatic launch
configuration (the benchmark's).  The resampler is checked at both limits: upsampling into a
23170 x 23170 float plane and downsampling out of one, on sampled rows and
columns."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mca
from conftest import check_u8

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _windows(H, W, k=16):
    return [(0, 0), (0, W - k), (H - k, 0), (H - k, W - k), (H // 2 + 7, W // 3), (H - k, W // 2), (H // 3, W - k)]


def test_forward_f32_largest_plane(gpu):
    H = W = 11585
    gpu.set_launch_config(0, 0)
    xs = np.random.default_rng(31).random((H, W), dtype=np.float32)
    x = torch.from_numpy(xs).cuda()
    y = gpu.zoom2x(x)
    assert y.numel() * 4 < 2 ** 31
    for r0, c0 in _windows(H, W):
        ref = oracle.window_zoom2x(xs, r0, r0 + 16, c0, c0 + 16)
        got = y[2 * r0: 2 * r0 + 32, 2 * c0: 2 * c0 + 32].cpu().numpy()
        assert np.abs(got - ref).max() <= TOL, (r0, c0)
    del x, y
    torch.cuda.empty_cache()


def test_forward_u8_largest_plane(gpu):
    H = W = 23170
    gpu.set_launch_config(0, 0)
    img = np.random.default_rng(32).integers(0, 256, (H, W), dtype=np.uint8)
    x = torch.from_numpy(img).cuda()
    y = gpu.zoom2x(x)
    assert y.numel() < 2 ** 31
    planes = None
    for r0, c0 in _windows(H, W):
        wr0, wc0 = max(0, r0 - 6), max(0, c0 - 6)
        sub = img[wr0: min(H, r0 + 22), wc0: min(W, c0 + 22)].astype(np.float64) / 255.0
        ref = oracle.window_zoom2x(sub, r0 - wr0, r0 - wr0 + 16, c0 - wc0, c0 - wc0 + 16)
        got = y[2 * r0: 2 * r0 + 32, 2 * c0: 2 * c0 + 32].cpu().numpy()
        check_u8(got, ref, "largest u8 plane window (%d, %d)" % (r0, c0))
        assert np.array_equal(got[0::2, 0::2], img[r0: r0 + 16, c0: c0 + 16])
    del x, y
    torch.cuda.empty_cache()


def test_backward_largest_plane(gpu):
    H = W = 11585
    gpu.set_launch_config(0, 0)
    rng = np.random.default_rng(33)
    xs = rng.random((H, W), dtype=np.float32)
    x = torch.from_numpy(xs).cuda()
    g = torch.empty((2 * H, 2 * W), device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(34)
    g.normal_(generator=gen)
    gx = gpu.zoom2x_backward(x, g)
    M = 12
    for r0, c0 in _windows(H, W, 12):
        r1, c1 = r0 + 12, c0 + 12
        wr0, wr1 = max(0, r0 - M), min(H, r1 + M)
        wc0, wc1 = max(0, c0 - M), min(W, c1 + M)
        Vw = xs[wr0:wr1, wc0:wc1].astype(np.float64)
        Gw = g[2 * wr0: 2 * wr1, 2 * wc0: 2 * wc1].cpu().numpy().astype(np.float64)
        ref_w = oracle.backward(Vw, Gw)
        bar, spread = mca.adjoint_bar(Vw, Gw, ref_w)
        ref = ref_w[r0 - wr0: r1 - wr0, c0 - wc0: c1 - wc0]
        got = gx[r0:r1, c0:c1].cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref_w).max()
        print("largest plane adjoint window (%d, %d): rel err %.2e, bar %.2e" % (r0, c0, err, bar))
        assert err <= bar, (r0, c0)
    del x, g, gx
    torch.cuda.empty_cache()


def _resample_samples(xs, OH, OW, rows, cols):
    """Oracle outputs of the tensor resampler of the float32 plane xs at
    (rows x cols): each sampled output row from its four clamped tap rows
    (the 1D spline on a 4-row array at local position 1 + t), then along it."""
    from oracle import resample as R

    H, W = xs.shape
    px, py = R.grid_positions(H, OH), R.grid_positions(W, OW)
    out = np.empty((len(rows), len(cols)))
    for k, r in enumerate(rows):
        i = min(max(int(np.floor(px[r])), 0), max(H - 2, 0))
        taps = xs[[min(max(j, 0), H - 1) for j in (i - 1, i, i + 1, i + 2)]].astype(np.float64)
        z = R.weno1d_eval(taps, [1.0 + (px[r] - i)], axis=-2)[0]
        out[k] = R.weno1d_eval(z, py[cols])
    return out


@pytest.mark.parametrize("shape,out", [((15447, 15447), (23170, 23170)),    # output plane just under 2^31 bytes
                                       ((23170, 23170), (11585, 11585))])   # input plane just under 2^31 bytes
def test_resample_largest_planes(gpu, shape, out):
    xs = np.random.default_rng(35).random(shape, dtype=np.float32)
    x = torch.from_numpy(xs).cuda()
    y = gpu.resample(x, *out)
    assert max(x.numel(), y.numel()) * 4 < 2 ** 31
    OH, OW = out
    rows = [0, 1, OH // 2 + 3, OH - 2, OH - 1]
    cols = list(range(0, 130)) + list(range(OW // 2 - 65, OW // 2 + 65)) + list(range(OW - 130, OW))
    ref = _resample_samples(xs, OH, OW, rows, cols)
    got = y[rows][:, cols].cpu().numpy()
    assert np.abs(got - ref).max() <= TOL
    del x, y
    torch.cuda.empty_cache()
