"""Properties the paper fixes, checked on the FP64 oracle.

- originals kept at even/even fine indices (Section 3);
- every candidate is exact on quadratics along its line, so bivariate
  polynomials of total degree <= 2 are reproduced for any beta; with beta = 0
  the weights are equal and each pair of parallel candidates is the cubic
  through four collinear samples (eq. Ideal2DPolynomial), so degree <= 3 is
  reproduced (Proposition 1);
- omega >= 0 and sum omega = 1 (eqs. IzrazOmega2d, IzrazOmega2dRavno);
- constants, offsets and the symmetries of the direction sets."""
import numpy as np
import pytest

from workloads import random_plane

M = 6  # ghost margin, beyond the -4..+5 footprint of a quad


def _ghost(oracle_mod, fn, n, m, h=1.0, **kw):
    """zoom of samples fn(x, y) taken on an input grid extended by M samples;
    returns (result on the 2n x 2m grid, exact fn at the fine positions)."""
    i = np.arange(-M, n + M) * h
    j = np.arange(-M, m + M) * h
    V = fn(i[:, None], j[None, :])
    U = oracle_mod.zoom2x(V, h=h, **kw)[2 * M: 2 * M + 2 * n, 2 * M: 2 * M + 2 * m]
    fi = np.arange(2 * n) * h / 2
    fj = np.arange(2 * m) * h / 2
    return U, fn(fi[:, None], fj[None, :])


QUADRATICS = [
    lambda x, y: 0.3 + 0 * x + 0 * y,
    lambda x, y: 0.7 * x - 0.2 * y + 0.1,
    lambda x, y: x * x - 0.5 * x * y + 0.25 * y * y + x,
    lambda x, y: -0.4 * x * y + 0.9 * y * y - y,
]
CUBICS = [
    lambda x, y: x ** 3 - 2 * x * x * y + 0.5 * y ** 3,
    lambda x, y: 0.2 * x * y * y - 0.7 * x ** 3 + x * y,
]


@pytest.mark.parametrize("k", range(len(QUADRATICS)))
@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0, 3.0])
def test_reproduces_quadratics_any_beta(oracle_mod, k, beta):
    U, exact = _ghost(oracle_mod, QUADRATICS[k], 7, 9, h=0.25, beta=beta)
    assert np.abs(U - exact).max() <= 1e-12


@pytest.mark.parametrize("k", range(len(CUBICS)))
def test_reproduces_cubics_linear_scheme(oracle_mod, k):
    U, exact = _ghost(oracle_mod, CUBICS[k], 8, 6, h=0.5, beta=0.0)
    assert np.abs(U - exact).max() <= 1e-12


def test_cubics_not_reproduced_by_nonlinear_scheme(oracle_mod):
    # beta > 0 moves the weights off 1/4: degree 3 is no longer exact (the
    # pins above would not catch a weight that silently stayed ideal).
    U, exact = _ghost(oracle_mod, CUBICS[0], 8, 6, h=0.5, beta=2.0)
    assert np.abs(U - exact).max() > 1e-6


def test_pair_identity_beta0(oracle_mod):
    # beta = 0: x point = mean of the two diagonal 4-point cubics (-1, 9, 9, -1)/16
    V = random_plane(8, 8, seed=11)
    U = oracle_mod.zoom2x(V, beta=0.0)
    for I in range(1, 6):
        for J in range(1, 6):
            d1 = (-V[I - 1, J - 1] + 9 * V[I, J] + 9 * V[I + 1, J + 1] - V[I + 2, J + 2]) / 16
            d2 = (-V[I - 1, J + 2] + 9 * V[I, J + 1] + 9 * V[I + 1, J] - V[I + 2, J - 1]) / 16
            assert abs(U[2 * I + 1, 2 * J + 1] - 0.5 * (d1 + d2)) <= 1e-14


def test_originals_kept(oracle_mod):
    V = random_plane(9, 7, seed=5, kind="steps")
    U = oracle_mod.zoom2x(V)
    assert np.array_equal(U[0::2, 0::2], V)


@pytest.mark.parametrize("c", [0.0, 0.5, 1.0, 123.25])
def test_constants(oracle_mod, c):
    U = oracle_mod.zoom2x(np.full((5, 8), c))
    assert np.abs(U - c).max() <= 1e-15 * max(1.0, abs(c)) * 8


def test_offset_equivariance(oracle_mod):
    V = random_plane(9, 11, seed=6, kind="steps")
    a = oracle_mod.zoom2x(V) + 0.375
    b = oracle_mod.zoom2x(V + 0.375)
    assert np.abs(a - b).max() <= 1e-12


def test_transpose_equivariance(oracle_mod):
    V = random_plane(7, 10, seed=8)
    a = oracle_mod.zoom2x(V.T)
    b = oracle_mod.zoom2x(V).T
    assert np.abs(a - b).max() <= 1e-14


@pytest.mark.parametrize("axis", [0, 1])
def test_flip_equivariance_on_paper_grid(oracle_mod, axis):
    # on the (2n-1) x (2m-1) grid of Section 3, clamp padding is symmetric
    V = random_plane(8, 9, seed=9, kind="steps")
    n, m = V.shape
    a = oracle_mod.zoom2x(np.flip(V, axis))[: 2 * n - 1, : 2 * m - 1]
    b = np.flip(oracle_mod.zoom2x(V)[: 2 * n - 1, : 2 * m - 1], axis)
    assert np.abs(a - b).max() <= 1e-14


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
def test_weights_convex(oracle_mod, beta):
    V = random_plane(6, 7, seed=10, kind="binary")
    W = oracle_mod.weights(V, beta=beta)
    new = np.ones(W.shape[:2], bool)
    new[0::2, 0::2] = False
    assert (W >= 0).all()
    assert np.abs(W[new].sum(-1) - 1).max() <= 1e-14
    if beta == 0.0:
        assert np.abs(W[new] - 0.25).max() <= 1e-15


def test_weights_avoid_a_step(oracle_mod):
    # a vertical step edge: at + points just left of it the candidate that
    # reaches across the step gets a vanishing weight for beta = 2
    V = np.zeros((12, 12))
    V[:, 6:] = 1.0
    W = oracle_mod.weights(V, beta=2.0)
    # B(I, 4) at fine (2I, 9): right stencil uses columns 4, 5, 6 (crosses)
    w = W[10, 9]
    # axis directions k: 0 down, 1 right, 2 up, 3 left
    assert w[1] < 1e-10
    assert w[0] + w[2] > 0.999  # the vertical candidates along the edge dominate
