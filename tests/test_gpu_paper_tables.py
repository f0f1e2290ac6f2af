"""The GPU kernel reproduces the paper's Table 1 (Section 4, convergence test:
beta = 1, f(x,y) = 1/(x^2+y^2+1) on [-1,1]^2) through the C ABI.

Same readings as the oracle's reproduction: the table's h is the spacing of
the zoomed grid (input spacing 2h); samples outside the domain are f itself,
supplied by padding the input with M ghost samples per side and cropping the
output (a quad reads inputs I-4..I+5, so M = 6 leaves the cropped outputs
independent of the clamped edge), or read in place through the library's
external boundary; neighbour weight h_in^2/8.

FP32 resolves the errors of rows 1-7 (row 7's 2.36e-6 is ~40 ulp of f ~ 1);
the finer rows are below FP32 rounding and are pinned on the oracle only."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_convergence.txt")
M = 6


def _table():
    rows = [[float(t) for t in ln.split()] for ln in open(GOLD) if ln.strip() and not ln.startswith("#")]
    return np.array(rows)


def f1(x, y):
    return 1.0 / (x * x + y * y + 1.0)


def gpu_zoom(gpu, i, boundary="pad"):
    """The zoomed (2n-1)^2 grid of row i: ghost samples by padding and
    cropping, or read in place (boundary "external": the input is the n x n
    view of the padded array)."""
    ht = 2.0 ** (-i)
    hin = 2 * ht
    n = int(round(2 / hin)) + 1
    x = -1 + np.arange(-M, n + M) * hin
    V = torch.tensor(f1(x[:, None], x[None, :]).astype(np.float32), device="cuda")
    kw = dict(beta=1.0, k_eps=1e-8, h=hin, nbw=hin * hin / 8.0)
    if boundary == "pad":
        U = gpu.zoom2x(V, **kw)[2 * M: 2 * M + 2 * n - 1, 2 * M: 2 * M + 2 * n - 1]
    else:
        U = gpu.zoom2x(V[M: M + n, M: M + n], boundary="external", **kw)[: 2 * n - 1, : 2 * n - 1]
    return U.cpu().numpy().astype(np.float64), ht, n


def gpu_linf(gpu, i, boundary="pad"):
    U, ht, n = gpu_zoom(gpu, i, boundary)
    xo = -1 + np.arange(2 * n - 1) * ht
    return np.abs(U - f1(xo[:, None], xo[None, :])).max()


def test_row1_is_12_over_19(gpu):
    # the centre x point of the 2x2 grid {-1, 1}^2 is 7/19, so the error is 12/19
    assert abs(gpu_linf(gpu, 0) - 12.0 / 19.0) <= 1e-6


@pytest.mark.parametrize("i", range(4))
def test_ghost_samples_read_in_place(gpu, i):
    # the library's external boundary reads the ghost samples through the
    # view's strides: the same arithmetic as padding and cropping, bit for bit
    Ue, _, _ = gpu_zoom(gpu, i, "external")
    Up, _, _ = gpu_zoom(gpu, i, "pad")
    assert np.array_equal(Ue, Up)
    if i == 0:
        assert abs(gpu_linf(gpu, 0, "external") - 12.0 / 19.0) <= 1e-6


@pytest.mark.parametrize("i", range(7))
def test_table1_linf_rows(gpu, i):
    tab = _table()
    linf = gpu_linf(gpu, i)
    # the oracle's bar (rows 1, 2 to the printed three digits, rows 3-6
    # within 6 %), widened for row 7 where FP32 rounding is a few % of the error
    tol = 0.006 if i in (0, 1) else (0.06 if i < 6 else 0.15)
    assert abs(linf / tab[i, 1] - 1) <= tol, (i, linf, tab[i, 1])


def test_table1_orders_rows_3_to_6(gpu):
    tab = _table()
    e = [gpu_linf(gpu, i) for i in range(2, 6)]
    for k in range(1, 4):
        order = np.log2(e[k - 1] / e[k])
        assert abs(order - tab[2 + k, 2]) <= 0.25, (k, order, tab[2 + k, 2])
