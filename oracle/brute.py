"""Brute-force mini-oracle for WD-WENO 2x zooming (arXiv 2312.00229, Section 3).

TEST INFRASTRUCTURE ONLY.  Pure-Python loops over every output point, for
tiny images (a few pixels per side).  It restates the method from its
geometric definitions instead of closed forms:

  * points live at x_{i,j} = (i h/2, j h/2) on the fine grid (Section 3);
  * d^gamma is one fine-grid step in direction gamma, eq. (Vektor), so the
    diagonal step has length sqrt(2) h / 2 and the axis step h / 2;
  * the stencil of eq. (p) is {x - d, x + d, x + 3d}; the candidate is the
    quadratic through those three samples, found by solving its 3x3
    Vandermonde system in the arclength s along d, evaluated at s = 0;
  * the smoothness indicator of eq. (2Dsmoothness) integrates the squared
    first and second s-derivatives of that quadratic over [-|d|, |d|] with
    3-point Gauss-Legendre quadrature (exact for the degree-2 integrand),
    weighted by L^(2l-1), L the length of the integration interval (or
    sqrt(2) h with `si_mode=1`);
  * D adds the same-direction indicators of the four neighbours of eq.
    (2DsmoothnessFinal) (phase 1) or eq. (tezine) (phase 2), weighted by
    `nbw` (h^2/8 unless given: the proof of Theorem 1 and Table 1 row 2;
    the definitions print h^2/4);
  * alpha = 0.5 / (eps + D)^beta, eq. (alpha), omega = alpha / sum alpha and
    u = sum omega p, eqs. (IzrazOmega2d) / (2dKombinacija).

Input samples outside the image are clamped to the edge.
"""
from __future__ import annotations

import math

import numpy as np

_GL_NODES, _GL_WEIGHTS = np.polynomial.legendre.leggauss(3)


def _quadratic_through(s_nodes, values):
    """Coefficients (c0, c1, c2) of c0 + c1 s + c2 s^2 through three points."""
    A = np.array([[1.0, s, s * s] for s in s_nodes])
    return np.linalg.solve(A, np.asarray(values, dtype=np.float64))


def _indicator(coef, half, scale):
    c0, c1, c2 = coef
    total = 0.0
    for l in (1, 2):
        acc = 0.0
        for t, wq in zip(_GL_NODES, _GL_WEIGHTS):
            s = half * t
            der = c1 + 2.0 * c2 * s if l == 1 else 2.0 * c2
            acc += wq * half * der * der
        total += scale ** (2 * l - 1) * acc
    return total


class BruteWENO:
    def __init__(self, V, beta=2.0, keps=1e-8, h=1.0, si_mode=0, nbw=None):
        self.V = np.asarray(V, dtype=np.float64)
        self.n, self.m = self.V.shape
        self.beta = float(beta)
        self.h = float(h)
        self.eps = keps * h * h
        self.nbw = h * h / 8.0 if nbw is None else float(nbw)
        self.si_mode = si_mode
        self._val = {}
        self._stencil = {}

    # directions gamma_k = gamma_0 + k pi/2, eq. (defgammak)
    @staticmethod
    def _directions(phase):
        g0 = math.pi / 4 if phase == 1 else 0.0
        return [g0 + k * math.pi / 2 for k in range(4)]

    def _step(self, gamma, phase):
        """d^gamma as a fine-grid step (di, dj) and its length."""
        c, s = math.cos(gamma), math.sin(gamma)
        di = int(round(c)) if phase == 2 else int(math.copysign(1, c))
        dj = int(round(s)) if phase == 2 else int(math.copysign(1, s))
        length = math.hypot(di * self.h / 2.0, dj * self.h / 2.0)
        return di, dj, length

    def value(self, i, j):
        """Value at fine index (i, j) of the padded grid."""
        key = (i, j)
        if key in self._val:
            return self._val[key]
        if i % 2 == 0 and j % 2 == 0:
            I = min(max(i // 2, 0), self.n - 1)
            J = min(max(j // 2, 0), self.m - 1)
            v = self.V[I, J]
        else:
            phase = 1 if (i % 2 == 1 and j % 2 == 1) else 2
            v = self._blend(i, j, phase)
        self._val[key] = v
        return v

    def stencil(self, i, j, phase, k):
        """(candidate p, indicator SI) of direction k at fine point (i, j)."""
        key = (i, j, k)
        if key in self._stencil:
            return self._stencil[key]
        di, dj, length = self._step(self._directions(phase)[k], phase)
        vals = [self.value(i + t * di, j + t * dj) for t in (-1, 1, 3)]
        coef = _quadratic_through([-length, length, 3 * length], vals)
        p = coef[0]
        scale = 2.0 * length if self.si_mode == 0 else math.sqrt(2.0) * self.h
        si = _indicator(coef, length, scale)
        self._stencil[key] = (p, si)
        return p, si

    def _neighbours(self, phase):
        if phase == 1:
            return [(0, 2), (2, 0), (0, -2), (-2, 0)]
        return [(1, 1), (-1, -1), (-1, 1), (1, -1)]

    def omegas(self, i, j):
        phase = 1 if (i % 2 == 1 and j % 2 == 1) else 2
        alphas, ps = [], []
        for k in range(4):
            p, si = self.stencil(i, j, phase, k)
            D = si + self.nbw * sum(self.stencil(i + a, j + b, phase, k)[1] for a, b in self._neighbours(phase))
            alphas.append(0.5 / (self.eps + D) ** self.beta)
            ps.append(p)
        tot = sum(alphas)
        return [a / tot for a in alphas], ps

    def _blend(self, i, j, phase):
        w, ps = self.omegas(i, j)
        return sum(wk * pk for wk, pk in zip(w, ps))

    def zoom(self):
        U = np.empty((2 * self.n, 2 * self.m))
        for i in range(2 * self.n):
            for j in range(2 * self.m):
                U[i, j] = self.value(i, j)
        return U


def zoom2x(V, **kw):
    """2n x 2m result for one (n, m) plane."""
    return BruteWENO(V, **kw).zoom()
