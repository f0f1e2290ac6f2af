"""GPU parity of the adjoint kernel (weno_zoom2x_backward through the C ABI)
against the oracle's hand adjoint (itself pinned to torch FP64 autograd and
central finite differences in the CPU suite).

Bar (conftest.check_adjoint): max |got - ref| <= bar * max |ref| with bar =
max(1e-5, 4 x the spread that Monte Carlo arithmetic at FP32 unit roundoff
gives the oracle's own gradient at that input, oracle.mca).  Well-conditioned
inputs keep the 1e-5 bar (the kernel reaches ~1e-6); next to flat regions the
gradient divides by t = eps + D close to eps and FP32 rounding of the formulas
alone moves it by up to ~1e-4, which the bar follows.  The whole 16x3x512^2
batch is checked in test_gpu_full_size.py."""
import numpy as np
import pytest
import torch

import oracle
from conftest import check_adjoint
from workloads import random_plane, scene_rgb, to_planar_f32

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


SHAPES = [(1, 1), (1, 9), (9, 1), (2, 3), (7, 77), (40, 39), (65, 120), (130, 37), (64, 38), (3, 200),
          # strip layout boundaries: one strip up to 37 columns, two (21 | W - 21) for 38..42, first + last
          # (42 + up to 41) up to 83, then middle strips of 46 (84: 42 | 41 | 1, 129: 42 | 46 | 41,
          # 130: 42 | 46 | 41 | 1, 175/176: four or five strips)
          (6, 37), (5, 38), (6, 42), (5, 43), (11, 83), (11, 84), (9, 85), (12, 129), (6, 130), (5, 131),
          (4, 175), (3, 176), (4, 177)]


@pytest.mark.parametrize("shape", SHAPES)
def test_backward_matches_oracle(gpu, shape):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    V = random_plane(*shape, seed=5, kind="steps") * 0.7 + 0.3 * rng.random(shape)
    G = rng.standard_normal((2 * shape[0], 2 * shape[1]))
    got = gpu.zoom2x_backward(_t(V), _t(G)).cpu().numpy()
    check_adjoint(got, V, G, "shape %s" % (shape,))


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 2.0, 3.0])
@pytest.mark.parametrize("kind", ["uniform", "binary", "steps"])
def test_backward_beta(gpu, beta, kind):
    rng = np.random.default_rng(int(beta * 10) + 1)
    V = random_plane(33, 71, seed=9, kind=kind)
    G = rng.standard_normal((66, 142))
    p = gpu.Params(beta=beta)
    got = gpu.zoom2x_backward(_t(V), _t(G), p).cpu().numpy()
    check_adjoint(got, V, G, "beta %.1f %s" % (beta, kind), beta=beta)


@pytest.mark.parametrize("kind", ["binary", "steps"])
def test_backward_beta0_without_eps(gpu, kind):
    # beta = 0, k_eps = 0: constant weights, so the adjoint is the transpose
    # of a linear map and must stay finite where indicators vanish
    rng = np.random.default_rng(5)
    V = random_plane(29, 63, seed=13, kind=kind)
    G = rng.standard_normal((58, 126))
    got = gpu.zoom2x_backward(_t(V), _t(G), gpu.Params(beta=0.0, k_eps=0.0)).cpu().numpy()
    assert np.isfinite(got).all()
    check_adjoint(got, V, G, "beta 0 without eps %s" % kind, beta=0.0, keps=0.0)


@pytest.mark.parametrize("nbw,h", [(0.25, 1.0), (0.0, 1.0), (-1.0, 0.25)])
def test_backward_parameters(gpu, nbw, h):
    rng = np.random.default_rng(3)
    V = random_plane(20, 50, seed=2, kind="steps") * 0.5 + 0.5 * rng.random((20, 50))
    G = rng.standard_normal((40, 100))
    got = gpu.zoom2x_backward(_t(V), _t(G), gpu.Params(nbw=nbw, h=h)).cpu().numpy()
    check_adjoint(got, V, G, "nbw %g h %g" % (nbw, h), nbw=None if nbw < 0 else nbw, h=h)


def test_backward_batch_and_strides(gpu):
    rng = np.random.default_rng(4)
    V = rng.random((2, 3, 21, 45)).astype(np.float32)
    G = rng.standard_normal((2, 3, 42, 90)).astype(np.float32)
    got = gpu.zoom2x_backward(_t(V), _t(G)).cpu().numpy()
    check_adjoint(got, V, G, "batch 2x3")
    # channels-interleaved input view
    x_hwc = _t(np.transpose(V[0], (1, 2, 0))).permute(2, 0, 1)
    got2 = gpu.zoom2x_backward(x_hwc, _t(G[0])).cpu().numpy()
    check_adjoint(got2, V[0], G[0], "HWC view")


def test_backward_into_callers_output(gpu):
    rng = np.random.default_rng(12)
    x = _t(rng.random((3, 40, 70)))
    g = _t(rng.standard_normal((3, 80, 140)))
    ref = gpu.zoom2x_backward(x, g)
    out = torch.full((40, 70, 3), float("nan"), device="cuda").permute(2, 0, 1)   # any strides
    assert gpu.zoom2x_backward(x, g, out=out) is out
    assert torch.equal(out, ref)
    with pytest.raises(ValueError):
        gpu.zoom2x_backward(x, g, out=torch.empty((3, 40, 71), device="cuda"))


def test_backward_deterministic(gpu):
    rng = np.random.default_rng(5)
    x = _t(rng.random((3, 100, 150)))
    g = _t(rng.standard_normal((3, 200, 300)))
    a = gpu.zoom2x_backward(x, g)
    b = gpu.zoom2x_backward(x, g)
    assert torch.equal(a, b)


def test_backward_independent_of_strip_height(gpu):
    """Every strip recomputes its warm-up rows exactly, so the result does not
    depend on where the bands start: bit-identical for every strip height."""
    rng = np.random.default_rng(15)
    x = _t(rng.random((2, 150, 100)))
    g = _t(rng.standard_normal((2, 300, 200)))
    ref = gpu.zoom2x_backward(x, g)
    try:
        for rows in (4, 5, 8, 13, 32, 64, 149):
            gpu.set_backward_launch_config(rows)
            assert torch.equal(gpu.zoom2x_backward(x, g), ref), rows
        # the forward's launch configuration does not reach the adjoint
        gpu.set_backward_launch_config(0)
        gpu.set_launch_config(8, 1)
        assert torch.equal(gpu.zoom2x_backward(x, g), ref)
    finally:
        gpu.set_backward_launch_config(0)
        gpu.set_launch_config(0, 0)


@pytest.mark.parametrize("H", [1, 2, 3, 5, 6, 9])
def test_backward_short_planes_every_band_layout(gpu, H):
    """Planes barely taller than a band: the top band is 4 rows shorter than
    the others (at least 1 row) and the bottom band takes what is left, so
    these heights give one to four bands of uneven size; every layout gives
    the same bits, and they match the oracle."""
    rng = np.random.default_rng(40 + H)
    V = rng.random((2, H, 70))
    G = rng.standard_normal((2, 2 * H, 140))
    x, g = _t(V), _t(G)
    ref = gpu.zoom2x_backward(x, g)
    check_adjoint(ref.cpu().numpy(), V, G, "short plane H=%d" % H)
    try:
        for rows in (4, 5, 6, 7, 8, 12):
            gpu.set_backward_launch_config(rows)
            assert torch.equal(gpu.zoom2x_backward(x, g), ref), (H, rows)
    finally:
        gpu.set_backward_launch_config(0)


def test_autograd_function(gpu):
    rng = np.random.default_rng(6)
    V = rng.random((3, 24, 31))
    x = _t(V).requires_grad_(True)
    y = gpu.WenoZoom2x.apply(x)
    G = rng.standard_normal(y.shape)
    (y * _t(G)).sum().backward()
    check_adjoint(x.grad.cpu().numpy(), V, G, "autograd function")


def test_finite_differences_fp64_16x16(gpu):
    # directional derivative of the FP64 oracle forward along a random
    # direction equals <grad, direction> of the GPU gradient
    rng = np.random.default_rng(7)
    V = rng.random((16, 16))
    G = rng.standard_normal((32, 32))
    D = rng.standard_normal((16, 16))
    eps = 1e-6
    fd = ((oracle.zoom2x(V + eps * D) - oracle.zoom2x(V - eps * D)) * G).sum() / (2 * eps)
    got = gpu.zoom2x_backward(_t(V), _t(G)).cpu().numpy().astype(np.float64)
    assert abs((got * D).sum() - fd) <= 1e-4 * max(1.0, abs(fd))


def test_inverse_problem_recovers_input(gpu):
    # recoverable inverse problem: target = zoom2x(x*); fit x from 0.5 with Adam
    torch.manual_seed(0)
    xs = torch.rand((3, 32, 32), device="cuda")
    target = gpu.zoom2x(xs)
    x = torch.full_like(xs, 0.5).requires_grad_(True)
    opt = torch.optim.Adam([x], lr=1e-2)
    first = None
    for it in range(300):
        opt.zero_grad()
        loss = torch.mean((gpu.WenoZoom2x.apply(x) - target) ** 2)
        loss.backward()
        opt.step()
        if first is None:
            first = float(loss.detach())
    assert float(loss.detach()) < 1e-3 * first
    assert float((x.detach() - xs).abs().max()) < 0.05


def _fit(gpu, target, shape, steps=200, lr=1e-2):
    x = torch.full(shape, 0.5, device="cuda").requires_grad_(True)
    opt = torch.optim.Adam([x], lr=lr)
    losses = []
    for _ in range(steps):
        opt.zero_grad()
        loss = torch.mean((gpu.WenoZoom2x.apply(x) - target) ** 2)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    return x.detach(), losses


def test_inverse_problem_full_size(gpu):
    """The differentiation workload at its full size: a 3 x 256 x 256 input
    fitted from 0.5 with Adam (lr 1e-2, 200 steps) so that its 2x zoom
    matches a 512 x 512 target.  (a) Recoverable: the target is the zoom of
    the polygon scene rendered at 256^2, which the fit must recover.  (b) The
    same scene rendered directly at 512^2 (the generator places polygons
    relative to the image size): the fit must beat the zoom of the 256^2
    rendering, the natural low-resolution candidate."""
    x_star = _t(to_planar_f32(scene_rgb(256, 256, seed=100)))
    target = gpu.zoom2x(x_star)
    x, losses = _fit(gpu, target, x_star.shape)
    err = float((x - x_star).abs().max())
    print("recoverable: loss %.3e -> %.3e, max |x - x*| %.4f" % (losses[0], losses[-1], err))
    assert losses[-1] < 1e-5 * losses[0]     # measured 5.6e-2 -> 4.6e-9
    assert err < 0.03                          # measured 0.0063

    hi = _t(to_planar_f32(scene_rgb(512, 512, seed=100)))
    x, losses = _fit(gpu, hi, x_star.shape)
    naive = float(torch.mean((gpu.zoom2x(x_star) - hi) ** 2))
    print("rendered: loss %.3e -> %.3e (zoom of the 256^2 rendering: %.3e)" % (losses[0], losses[-1], naive))
    assert losses[-1] < 0.7 * naive            # measured 5.8e-4 against 1.5e-3
