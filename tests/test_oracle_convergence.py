"""Theorem 1: O(h^4) for smooth data.  The smooth test function on [0,1]^2
sampled at n = 32, 64, 128, 256, ghost samples beyond the domain."""
import numpy as np

from workloads import smooth_f

M = 6


def _err(oracle_mod, n):
    h = 1.0 / (n - 1)
    x = np.arange(-M, n + M) * h
    V = smooth_f(x[:, None], x[None, :])
    U = oracle_mod.zoom2x(V, beta=2.0, h=h)[2 * M: 2 * M + 2 * n - 1, 2 * M: 2 * M + 2 * n - 1]
    xf = np.arange(2 * n - 1) * h / 2
    return np.abs(U - smooth_f(xf[:, None], xf[None, :])).max()


def test_fourth_order_smooth():
    import oracle

    e = [_err(oracle, n) for n in (32, 64, 128, 256)]
    orders = [np.log2(e[k] / e[k + 1]) * 1.0 for k in range(3)]
    # spacing ratio (n-1) / (2n-1) is ~1/2; use the exact ratio
    hs = [1.0 / (n - 1) for n in (32, 64, 128, 256)]
    orders = [np.log(e[k] / e[k + 1]) / np.log(hs[k] / hs[k + 1]) for k in range(3)]
    assert abs(orders[-1] - 4.0) <= 0.1, orders
