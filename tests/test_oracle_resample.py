"""Pins of the arbitrary-resolution oracle (Section 2's 1D WENO, eq.
wenoSpline, eq. tensor, Section 3.3)."""
import numpy as np
import pytest

import oracle
from oracle import resample as R


def _poly_eval(coef, t):
    return np.polyval(coef, t)


def test_ideal_weights_from_the_cubic():
    # brute force: the cubic through nodes -1..2 and the two quadratics by
    # polynomial fits; C_0 solves C_0 p_i + (1 - C_0) p_{i+1} = q
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = rng.standard_normal(4)
        t = rng.uniform(0.05, 0.95)
        q = _poly_eval(np.polyfit([-1, 0, 1, 2], v, 3), t)
        p0 = _poly_eval(np.polyfit([-1, 0, 1], v[:3], 2), t)
        p1 = _poly_eval(np.polyfit([0, 1, 2], v[1:], 2), t)
        c0 = (q - p1) / (p0 - p1)
        assert abs(c0 - R.ideal_weights(t)[0]) <= 1e-9


def test_indicator_by_quadrature():
    rng = np.random.default_rng(1)
    xg, wg = np.polynomial.legendre.leggauss(3)
    for _ in range(10):
        c = rng.standard_normal(3)
        t0, t1 = (0.0, 1.0) if rng.random() < 0.5 else (-1.0, 0.0)
        tt = 0.5 * (t1 - t0) * xg + 0.5 * (t1 + t0)
        d1 = c[1] + 2 * c[2] * tt
        quad = 0.5 * (t1 - t0) * np.sum(wg * (d1 ** 2 + (2 * c[2]) ** 2))
        assert abs(quad - R._indicator(c[1], c[2], t0, t1)) <= 1e-12


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
def test_nodes_and_quadratics(beta):
    x = np.linspace(-1.0, 2.0, 13)
    rng = np.random.default_rng(2)
    pos = np.concatenate([np.arange(13.0), rng.uniform(0, 12, 25)])
    quad = 0.3 * x * x - x + 0.2
    u = R.weno1d_eval(quad, pos, beta=beta, h=x[1] - x[0])
    exact = np.interp(pos, np.arange(13), quad)  # at nodes
    assert np.abs(u[:13] - quad).max() == 0.0 or np.abs(u[:13] - quad).max() <= 1e-15
    xp = -1.0 + pos * (x[1] - x[0])
    interior = (pos >= 1) & (pos <= 11)
    assert np.abs(u - (0.3 * xp * xp - xp + 0.2))[interior].max() <= 1e-12


def test_cubics_linear_scheme_and_midpoint_taps():
    x = np.arange(10.0)
    cub = 0.01 * x ** 3 - 0.2 * x * x + x
    pos = np.array([1.5, 2.25, 4.7, 7.9])
    u = R.weno1d_eval(cub, pos, beta=0.0)
    assert np.abs(u - (0.01 * pos ** 3 - 0.2 * pos ** 2 + pos)).max() <= 1e-12
    v = np.random.default_rng(3).standard_normal(8)
    mid = R.weno1d_eval(v, [3.5], beta=0.0)[0]
    assert abs(mid - (-v[2] + 9 * v[3] + 9 * v[4] - v[5]) / 16) <= 1e-14


def test_fourth_order_1d():
    f = lambda x: np.sin(3 * x) + 0.3 * np.cos(7 * x)
    errs = []
    for n in (32, 64, 128, 256):
        h = 1.0 / (n - 1)
        pad = 3
        xs = (np.arange(-pad, n + pad)) * h
        pos = pad + np.arange(n - 1) + 0.37
        u = R.weno1d_eval(f(xs), pos, beta=2.0, h=h)
        errs.append(np.abs(u - f((pos - pad) * h)).max())
    order = np.log2(errs[-2] / errs[-1]) * np.log(2) / np.log(255 / 127)
    assert 3.8 <= order <= 4.3


def test_tensor_reproduces_biquadratics_and_identity():
    H, W = 9, 11
    i = np.arange(H)[:, None] * 1.0
    j = np.arange(W)[None, :] * 1.0
    f = lambda a, b: 0.1 * a * a * b - 0.05 * a * b * b + a - 2 * b + 0.01 * a * a * b * b
    V = f(i, j)
    out = R.tensor_resample(V, 17, 5)
    pi = R.grid_positions(H, 17)[:, None]
    pj = R.grid_positions(W, 5)[None, :]
    inner = np.ix_((pi[:, 0] >= 1) & (pi[:, 0] <= H - 2), (pj[0] >= 1) & (pj[0] <= W - 2))
    assert np.abs(out - f(pi, pj))[inner].max() <= 1e-10
    rng = np.random.default_rng(4)
    Z = rng.random((6, 7))
    assert np.array_equal(R.tensor_resample(Z, 6, 7), Z)


def test_zoom_to_nested_grid_is_the_doubling():
    rng = np.random.default_rng(5)
    V = rng.random((7, 9))
    # target exactly the nested grid after one doubling: resampling copies
    U = R.zoom_to(V, 13, 17)
    ref = oracle.zoom2x(V)[:13, :17]
    assert np.abs(U - ref).max() <= 1e-14
    # three-quarter scale is plain resampling; triple scale needs two doublings
    assert R.zoom_to(V, 5, 6).shape == (5, 6)
    assert R.zoom_to(V, 21, 27).shape == (21, 27)
