"""FP64 oracle for the arbitrary-resolution path (arXiv 2312.00229, Section 3.3).

TEST INFRASTRUCTURE ONLY (callers: tests, smoke check, CPU baseline).

1D WENO interpolation (Section 2, eqs. Tocnost .. IzrazOmega): on
[x_i, x_{i+1}] with local coordinate t = (x - x_i)/h in [0, 1], the two
quadratics
    p_i     through v_{i-1}, v_i, v_{i+1}     (nodes t = -1, 0, 1)
    p_{i+1} through v_i, v_{i+1}, v_{i+2}     (nodes t = 0, 1, 2)
are blended with
    alpha_s = C_s(t) / (eps + SI_s)^beta,  omega_s = alpha_s / (alpha_0 + alpha_1),
where the ideal weights C_0, C_1 are the linear functions with
C_0 p_i + C_1 p_{i+1} = the cubic through the four nodes (eq.
PolinomZaVelikiStencil), and the indicator is
    SI_s = sum_{l=1,2} int_{x_i}^{x_{i+1}} h^{2l-1} (d^l p_{i+s} / dx^l)^2 dx.
Everything here is computed from those definitions: the ideal weights by
solving for the cubic, the indicator by integrating the quadratic's
derivatives.  eps = K_eps h^2 with h the input spacing.

The WENO spline w(V, x) (eq. wenoSpline) evaluates that interpolant at any
x in [0, n-1]; samples beyond the ends are clamped.  The tensor WENO
resampler (eq. tensor) applies it along the rows, then along the columns.
An output grid of n* samples spans the input grid end to end: output sample
j sits at x_j = j (n-1)/(n*-1).  Arbitrary-size zooming (Section 3.3)
doubles k times with the 2D method and resamples the (2^k (n-1) + 1) grid.
"""
from __future__ import annotations

import numpy as np


def _quad_coeffs(vm, v0, vp):
    """Quadratic through (-1, vm), (0, v0), (1, vp) as c0 + c1 t + c2 t^2."""
    c0 = v0
    c1 = (vp - vm) / 2.0
    c2 = (vp - 2.0 * v0 + vm) / 2.0
    return c0, c1, c2


def _indicator(c1, c2, t0, t1):
    """int_{t0}^{t1} (p')^2 + (p'')^2 dt for p = c0 + c1 t + c2 t^2 (the h
    powers of the definition cancel against dx = h dt and d/dx = d/dt / h)."""
    def F(t):  # antiderivative of (c1 + 2 c2 t)^2 + (2 c2)^2
        return c1 * c1 * t + 2.0 * c1 * c2 * t * t + (4.0 / 3.0) * c2 * c2 * t ** 3 + 4.0 * c2 * c2 * t
    return F(t1) - F(t0)


def ideal_weights(t):
    """C_0(t), C_1(t): the cubic through nodes -1, 0, 1, 2 equals
    C_0 p_i + C_1 p_{i+1}.  Both quadratics agree at t = 0, 1, so
    p_{i+1} - p_i = kappa t (t - 1) and q - p_i = D t (t + 1)(t - 1) with q, p_i,
    p_{i+1} matching at t = 2: kappa * 2 = D * 6.  Hence
    C_1 = (q - p_i)/(p_{i+1} - p_i) = (t + 1)/3, C_0 = 1 - C_1."""
    c1 = (t + 1.0) / 3.0
    return 1.0 - c1, c1


def weno1d_eval(V, x, beta=2.0, keps=1e-8, h=1.0, axis=-1):
    """w(V, x) along `axis` of V at the (1-D array of) positions x, in units
    of the grid index (0 .. n-1)."""
    V = np.moveaxis(np.asarray(V, dtype=np.float64), axis, -1)
    n = V.shape[-1]
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(V.shape[:-1] + (len(x),))
    eps = keps * h * h
    for k, xk in enumerate(x):
        i = int(np.floor(xk))
        i = min(max(i, 0), max(n - 2, 0))
        t = xk - i
        idx = [min(max(j, 0), n - 1) for j in (i - 1, i, i + 1, i + 2)]
        vm1, v0, v1, v2 = (V[..., j] for j in idx)
        a0, a1, a2 = _quad_coeffs(vm1, v0, v1)          # p_i in t
        b0, b1, b2 = _quad_coeffs(v0, v1, v2)           # p_{i+1} in s = t - 1
        p0 = a0 + a1 * t + a2 * t * t
        s = t - 1.0
        p1 = b0 + b1 * s + b2 * s * s
        si0 = _indicator(a1, a2, 0.0, 1.0)
        si1 = _indicator(b1, b2, -1.0, 0.0)
        C0, C1 = ideal_weights(t)
        al0 = C0 / (eps + si0) ** beta
        al1 = C1 / (eps + si1) ** beta
        if t == 0.0:
            out[..., k] = v0          # the interpolant passes through its nodes
        elif t == 1.0:
            out[..., k] = v1
        else:
            out[..., k] = (al0 * p0 + al1 * p1) / (al0 + al1)
    return np.moveaxis(out, -1, axis)


def grid_positions(n_in, n_out):
    """End-to-end output positions x_j = j (n_in - 1)/(n_out - 1)."""
    if n_out == 1:
        return np.zeros(1)
    return np.arange(n_out) * ((n_in - 1) / (n_out - 1))


def tensor_resample(V, out_h, out_w, beta=2.0, keps=1e-8, h=1.0):
    """eq. (tensor): every (.., H, W) plane resampled to (out_h, out_w),
    first along the rows (axis -2), then along the columns."""
    V = np.asarray(V, dtype=np.float64)
    H, W = V.shape[-2:]
    Z = weno1d_eval(V, grid_positions(H, out_h), beta, keps, h, axis=-2)
    return weno1d_eval(Z, grid_positions(W, out_w), beta, keps, h, axis=-1)


def zoom_to(V, out_h, out_w, beta=2.0, keps=1e-8, h=1.0):
    """Section 3.3: k doublings, k the least with 2^k (n - 1) + 1 >= the target
    along both axes, then the tensor resampler on the paper's
    (2^k (n-1) + 1) x (2^k (m-1) + 1) grid, on which the spacing is h / 2^k."""
    from . import zoom2x

    V = np.asarray(V, dtype=np.float64)
    H, W = V.shape[-2:]
    k = 0
    # an axis of one sample cannot be refined by doubling; it is only resampled
    while ((H > 1 and (2 ** k) * (H - 1) + 1 < out_h) or (W > 1 and (2 ** k) * (W - 1) + 1 < out_w)) and k < 8:
        k += 1
    U = V
    for lvl in range(k):
        n, m = U.shape[-2:]
        # the paper's nested grids: each level doubles the (2n-1) x (2m-1) grid
        U = zoom2x(U, beta=beta, keps=keps, h=h / 2 ** lvl)[..., : 2 * n - 1, : 2 * m - 1]
    return tensor_resample(U, out_h, out_w, beta=beta, keps=keps, h=h / 2 ** k)
