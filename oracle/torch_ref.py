"""WD-WENO 2x zooming as vectorised torch FP64 CPU ops (arXiv 2312.00229, Section 3).

TEST INFRASTRUCTURE ONLY: the autograd reference for the hand adjoint.  It
restates the two phases on the coarse index grid (every field is a tensor of
positions) rather than on the fine grid of the C oracle:

  X(I, J)  phase-1 point at (I + 1/2, J + 1/2), four diagonal stencils;
  A(I, J)  phase-2 point at (I + 1/2, J), vertical stencils on originals,
           horizontal stencils on X;
  B(I, J)  phase-2 point at (I, J + 1/2), horizontal stencils on originals,
           vertical stencils on X.

`rounding` (optional): a function applied to every intermediate the
formulas produce (candidates, stencil differences, indicators, eps + D,
weights, their sum, blends).  Passing a random relative perturbation of the
size of a unit roundoff makes this Monte Carlo arithmetic (D. S. Parker,
"Monte Carlo arithmetic: exploiting randomness in floating-point
arithmetic", 1997): the spread of the results, and of their autograd
gradients, over a few draws estimates how far rounding at that precision can
move any evaluation of these formulas.

Candidate of a stencil (a, b, c) at nodes -1, 1, 3 evaluated at 0:
(3a + 6b - c)/8.  Indicator with the interval-length scale:
(b - a)^2 + 13/12 (a - 2b + c)^2 (the integral of eq. 2Dsmoothness worked out
in closed form).  Clamp-to-edge padding through index gathers, so autograd
folds gradients of padded reads onto the source pixels.
"""
from __future__ import annotations

import torch

M = 6  # coarse margin of the padded input


def _exact(x):
    return x


def zoom2x(V: torch.Tensor, beta=2.0, keps=1e-8, h=1.0, nbw=None, rounding=None) -> torch.Tensor:
    """V: (..., n, m) float64 -> (..., 2n, 2m)."""
    r = rounding or _exact

    def _cand(a, b, c):
        return r((3.0 * a + 6.0 * b - c) / 8.0)

    def _si(a, b, c):
        return r(r(b - a) ** 2 + (13.0 / 12.0) * r(a - 2.0 * b + c) ** 2)

    def _blend(ps, Ds, eps, beta):
        alphas = [r(0.5 / r(eps + D) ** beta) for D in Ds]
        tot = r(alphas[0] + alphas[1] + alphas[2] + alphas[3])
        return r(sum(a * p for a, p in zip(alphas, ps)) / tot)

    n, m = V.shape[-2:]
    eps = keps * h * h
    w = h * h / 8.0 if nbw is None else nbw
    ri = torch.arange(-M, n + M).clamp(0, n - 1)
    ci = torch.arange(-M, m + M).clamp(0, m - 1)
    Vp = V.index_select(-2, ri).index_select(-1, ci)  # Vp[..., I+M, J+M]

    def v(di, dj, r0, r1, c0, c1):
        """V(I+di, J+dj) for I in [r0, r1), J in [c0, c1)."""
        return Vp[..., r0 + di + M: r1 + di + M, c0 + dj + M: c1 + dj + M]

    # ---- phase 1 on X(I, J), I, J in [-4, n+3) (indicators) ----
    lo, hr, hc = -4, n + 3, m + 3

    def tri_x(r0, r1, c0, c1):
        g = lambda a, b: v(a, b, r0, r1, c0, c1)
        return [
            (g(0, 0), g(1, 1), g(2, 2)),      # gamma = pi/4   (down-right)
            (g(1, 0), g(0, 1), g(-1, 2)),     # gamma = 3pi/4  (up-right)
            (g(1, 1), g(0, 0), g(-1, -1)),    # gamma = 5pi/4  (up-left)
            (g(0, 1), g(1, 0), g(2, -1)),     # gamma = 7pi/4  (down-left)
        ]

    SIx = [_si(*t) for t in tri_x(lo, hr, lo, hc)]
    # X on [-3, n+2): own indicator plus (I+-1, J), (I, J+-1) neighbours
    def sx(k, di, dj):
        return SIx[k][..., 1 + di: SIx[k].shape[-2] - 1 + di, 1 + dj: SIx[k].shape[-1] - 1 + dj]

    Px = [_cand(*t) for t in tri_x(lo + 1, hr - 1, lo + 1, hc - 1)]
    Dx = [sx(k, 0, 0) + w * (sx(k, 1, 0) + sx(k, -1, 0) + sx(k, 0, 1) + sx(k, 0, -1)) for k in range(4)]
    X = _blend(Px, Dx, eps, beta)          # X[..., I+3, J+3] for I in [-3, n+2)
    XM = 3

    def x(di, dj, r0, r1, c0, c1):
        return X[..., r0 + di + XM: r1 + di + XM, c0 + dj + XM: c1 + dj + XM]

    # ---- phase 2 indicators, A and B on [-1, n+1) ----
    r0, r1, c0, c1 = -1, n + 1, -1, m + 1

    def tri_a(r0, r1, c0, c1):
        gv = lambda a, b: v(a, b, r0, r1, c0, c1)
        gx = lambda a, b: x(a, b, r0, r1, c0, c1)
        return [
            (gv(0, 0), gv(1, 0), gv(2, 0)),      # gamma = 0     (down, originals)
            (gx(0, -1), gx(0, 0), gx(0, 1)),     # gamma = pi/2  (right, x points)
            (gv(1, 0), gv(0, 0), gv(-1, 0)),     # gamma = pi    (up, originals)
            (gx(0, 0), gx(0, -1), gx(0, -2)),    # gamma = 3pi/2 (left, x points)
        ]

    def tri_b(r0, r1, c0, c1):
        gv = lambda a, b: v(a, b, r0, r1, c0, c1)
        gx = lambda a, b: x(a, b, r0, r1, c0, c1)
        return [
            (gx(-1, 0), gx(0, 0), gx(1, 0)),     # gamma = 0     (down, x points)
            (gv(0, 0), gv(0, 1), gv(0, 2)),      # gamma = pi/2  (right, originals)
            (gx(0, 0), gx(-1, 0), gx(-2, 0)),    # gamma = pi    (up, x points)
            (gv(0, 1), gv(0, 0), gv(0, -1)),     # gamma = 3pi/2 (left, originals)
        ]

    SIa = [_si(*t) for t in tri_a(r0, r1, c0, c1)]   # SIa[k][..., I+1, J+1]
    SIb = [_si(*t) for t in tri_b(r0, r1, c0, c1)]
    Pa = [_cand(*t) for t in tri_a(0, n, 0, m)]
    Pb = [_cand(*t) for t in tri_b(0, n, 0, m)]

    def sa(k, di, dj):
        return SIa[k][..., 1 + di: 1 + di + n, 1 + dj: 1 + dj + m]

    def sb(k, di, dj):
        return SIb[k][..., 1 + di: 1 + di + n, 1 + dj: 1 + dj + m]

    # eq. (tezine): the +-1 diagonal fine neighbours of A(I,J) are B(I, J-1),
    # B(I, J), B(I+1, J-1), B(I+1, J); those of B(I,J) are A(I-1, J), A(I, J),
    # A(I-1, J+1), A(I, J+1).
    Da = [sa(k, 0, 0) + w * (sb(k, 0, -1) + sb(k, 0, 0) + sb(k, 1, -1) + sb(k, 1, 0)) for k in range(4)]
    Db = [sb(k, 0, 0) + w * (sa(k, -1, 0) + sa(k, 0, 0) + sa(k, -1, 1) + sa(k, 0, 1)) for k in range(4)]
    A = _blend(Pa, Da, eps, beta)
    B = _blend(Pb, Db, eps, beta)
    Xo = x(0, 0, 0, n, 0, m)

    top = torch.stack([V, B], dim=-1).reshape(V.shape[:-1] + (2 * m,))
    bot = torch.stack([A, Xo], dim=-1).reshape(V.shape[:-1] + (2 * m,))
    return torch.stack([top, bot], dim=-2).reshape(V.shape[:-2] + (2 * n, 2 * m))
