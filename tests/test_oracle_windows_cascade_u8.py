"""Pins of the oracle's helpers that the full-size GPU checks rely on.

- window_zoom2x: a block of output quads computed on a window of the input
  equals the same block of the whole-plane result, bit for bit, at every
  border and in the interior;
- the footprint of a quad: quad (I, J) reads exactly the inputs of rows and
  columns I-4 .. I+5, J-4 .. J+5 (79 of those 100 samples: the four corners
  of the square are outside every stencil and neighbour set, Section 3 stencil
  and neighbour bookkeeping), so inputs outside it leave the quad bit-identical
  and inputs inside it move it;
- cascade (eq. zoomfactor): every level reproduces bivariate polynomials of
  total degree <= 2, so three levels do too; the originals of each level are
  kept, so level L's samples at multiples of 2^L are the input;
- uint8 quantisation: round half to even, clamp; the comparison helper counts a
  one-code difference at a k + 1/2 value as a tie and any other difference as
  an error.
"""
import numpy as np
import pytest

from conftest import check_u8, u8_compare
from workloads import pixel_art, random_plane, two_level_u8


@pytest.mark.parametrize("win", [
    (0, 10, 0, 12),        # top-left corner
    (0, 7, 20, 33),        # top edge
    (15, 29, 40, 47),      # bottom-right corner
    (10, 20, 0, 5),        # left edge
    (8, 19, 14, 31),       # interior
    (0, 29, 0, 47),        # the whole plane
])
@pytest.mark.parametrize("beta", [1.0, 2.0])
def test_window_equals_full_plane(oracle_mod, win, beta):
    V = np.stack([random_plane(29, 47, seed=s, kind=k) for s, k in ((1, "steps"), (2, "uniform"))])
    full = oracle_mod.zoom2x(V, beta=beta)
    r0, r1, c0, c1 = win
    got = oracle_mod.window_zoom2x(V, r0, r1, c0, c1, beta=beta)
    assert got.shape == (2, 2 * (r1 - r0), 2 * (c1 - c0))
    assert np.array_equal(got, full[:, 2 * r0: 2 * r1, 2 * c0: 2 * c1])


def test_quad_footprint(oracle_mod):
    n = m = 22
    I, J = 10, 11
    V = random_plane(n, m, seed=4, kind="uniform")
    base = oracle_mod.zoom2x(V)[2 * I: 2 * I + 2, 2 * J: 2 * J + 2]
    moved = np.zeros((n, m), bool)
    for r in range(n):
        for c in range(m):
            W = V.copy()
            W[r, c] += 0.37
            q = oracle_mod.zoom2x(W)[2 * I: 2 * I + 2, 2 * J: 2 * J + 2]
            moved[r, c] = not np.array_equal(q, base)
    rows, cols = np.nonzero(moved)
    assert rows.min() == I - 4 and rows.max() == I + 5
    assert cols.min() == J - 4 and cols.max() == J + 5
    assert moved.sum() == 79
    # the missing samples of the 10 x 10 square are its four corners
    sq = moved[I - 4: I + 6, J - 4: J + 6]
    assert not sq[0, 0] and not sq[0, -1] and not sq[-1, 0] and not sq[-1, -1]


QUADRATICS = [
    lambda x, y: 0.3 + 0 * x + 0 * y,
    lambda x, y: 0.7 * x - 0.2 * y + 0.1,
    lambda x, y: 0.02 * (x * x - 0.5 * x * y + 0.25 * y * y) + 0.1 * x,
    lambda x, y: 0.01 * (-0.4 * x * y + 0.9 * y * y) - 0.05 * y,
]


@pytest.mark.parametrize("k", range(len(QUADRATICS)))
@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
def test_cascade_reproduces_quadratics(oracle_mod, k, beta):
    n, m, L = 30, 34, 3
    f = QUADRATICS[k]
    x = np.arange(n, dtype=np.float64)
    y = np.arange(m, dtype=np.float64)
    V = f(x[:, None], y[None, :])
    U = oracle_mod.cascade(V, L, beta=beta)
    assert U.shape == (8 * n, 8 * m)
    s = 2 ** L
    fx = np.arange(s * n) / s
    fy = np.arange(s * m) / s
    E = np.abs(U - f(fx[:, None], fy[None, :]))
    # clamped borders break exactness within 4 + 2 + 1 input rows/columns
    # above/left and 5.5 + 2.75 + 1.4 below/right; keep a margin of 11
    inner = E[11 * s: (n - 11) * s, 11 * s: (m - 11) * s]
    assert inner.size > 0
    assert inner.max() <= 1e-11, inner.max()


def test_cascade_one_level_is_the_doubling(oracle_mod):
    V = random_plane(13, 17, seed=5, kind="steps")
    assert np.array_equal(oracle_mod.cascade(V, 1), oracle_mod.zoom2x(V))


@pytest.mark.parametrize("L", [2, 3])
def test_cascade_keeps_originals_of_every_level(oracle_mod, L):
    img = pixel_art(16, 20, seed=3, block=4, n_lines=3)
    V = np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0
    U = oracle_mod.cascade(V, L)
    assert np.array_equal(U[:, :: 2 ** L, :: 2 ** L], V)
    # level L-1's result sits at the even samples of level L
    prev = oracle_mod.cascade(V, L - 1)
    assert np.array_equal(U[:, ::2, ::2], prev)


def test_cascade_halves_spacing(oracle_mod):
    # level l works on spacing h / 2^l: with an explicit neighbour weight the
    # second level equals a doubling with h/2 (the project's reading of the
    # paper's "successive application", parity unpinned by the paper)
    V = random_plane(9, 11, seed=6, kind="steps")
    two = oracle_mod.cascade(V, 2, h=2.0)
    ref = oracle_mod.zoom2x(oracle_mod.zoom2x(V, h=2.0), h=1.0)
    assert np.array_equal(two, ref)
    other = oracle_mod.zoom2x(oracle_mod.zoom2x(V, h=2.0), h=2.0)
    assert not np.array_equal(two, other)


def test_quantize_half_even_and_clamp(oracle_mod):
    x = np.array([0.5, 1.5, 2.5, 3.5, 126.5, 127.5, 254.5, 0.49999, 0.50001, 255.4, 255.5, 300.0, -0.5, -3.0])
    q = oracle_mod.quantize_u8_255(x)
    assert q.tolist() == [0, 2, 2, 4, 126, 128, 254, 0, 1, 255, 255, 255, 0, 0]
    # on the [0,1] scale: 255 u, then the same rule
    assert oracle_mod.quantize_u8(np.array([0.0, 1.0, 2.0 / 255.0, 0.5])).tolist() == [0, 255, 2, 128]


def test_u8_compare_counts_ties_and_errors():
    u = np.array([2.5, 3.5, 10.2, 10.2, 100.0, 7.5]) / 255.0
    exact = np.array([2, 4, 10, 10, 100, 8], dtype=np.uint8)
    assert u8_compare(exact, u) == (0, 0)
    # a one-code difference at k + 1/2 is a tie; elsewhere an error
    assert u8_compare(np.array([3, 4, 10, 10, 100, 8], np.uint8), u) == (1, 0)
    assert u8_compare(np.array([2, 4, 11, 10, 100, 8], np.uint8), u) == (0, 1)
    # two codes away from a tie value is an error, not a tie
    assert u8_compare(np.array([2, 4, 10, 10, 100, 6], np.uint8), u) == (0, 1)


def test_check_u8_bounds_ties():
    # exact halves may round either way in FP32: all allowed here (the GPU
    # test on exact halves pins round half to even without any allowance)
    u = (np.arange(4000) % 200 + 0.5) / 255.0
    up = np.floor(255.0 * u + 0.5).astype(np.uint8)
    assert check_u8(up, u, "exact halves rounded up") > 0
    # values within the tie band of a half but not on it: a flipped code is a
    # counted tie, and more than the allowed fraction fails
    v = (np.arange(4000) % 200 + 0.5 + 1e-4) / 255.0
    codes = np.rint(255.0 * v).astype(np.uint8)
    assert check_u8(codes, v, "near halves") == 0
    one = codes.copy()
    one[7] -= 1
    assert check_u8(one, v, "one flipped") == 1
    with pytest.raises(AssertionError):
        check_u8(codes - 1, v, "all flipped")


def test_two_level_input_has_exact_ties(oracle_mod):
    img = two_level_u8(37, 70, seed=1)
    X = oracle_mod.zoom2x(img.astype(np.float64), beta=0.0)   # 0..255 scale
    frac = X - np.floor(X)
    ties = frac == 0.5
    assert ties.mean() > 0.1
    # the [0,1]-scale result is the same map (beta = 0 is linear)
    assert np.abs(oracle_mod.zoom2x(img / 255.0, beta=0.0) * 255.0 - X).max() <= 1e-10
