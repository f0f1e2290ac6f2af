import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU case")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0.  A GPU test never skips: a missing GPU or
    library is a failure."""
    import torch

    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    import paper_2312_00229_amd as wz
    from paper_2312_00229_amd import _lib

    _lib.lib()  # raises if the library is not built
    return wz


def u8_compare(gpu_codes, oracle_u, tie_band=1e-5):
    """Compare uint8 codes with the FP64 oracle's [0,1] values.

    A mismatch is a counted tie only if the oracle value lies within
    `tie_band` (on the [0,1] scale) of a rounding boundary k + 1/2 (in 255
    units) and the codes differ by one; any other mismatch is an error.
    Returns (n_ties, n_errors)."""
    import oracle

    x = 255.0 * np.asarray(oracle_u, dtype=np.float64)
    ref = oracle.quantize_u8_255(x).astype(np.float64)
    g = np.asarray(gpu_codes, dtype=np.float64)
    bad = g != ref
    frac = x - np.floor(x)
    near = np.abs(frac - 0.5) < 255.0 * tie_band
    tie = bad & near & (np.abs(g - ref) <= 1)
    return int(tie.sum()), int((bad & ~tie).sum())


def check_u8(gpu_codes, oracle_u, label, tie_band=1e-5, max_tie_frac=1e-4):
    """uint8 parity: no error (u8_compare), and a bounded number of counted
    ties.  Oracle values that are halves k + 1/2 up to the oracle's own
    rounding (within 1e-6 of a code, 4e-9 on the [0,1] scale) may round either
    way in FP32 and are all allowed; beyond those, at most
    max(2, max_tie_frac * size) ties.  Prints the counts so that every run
    records them."""
    import oracle

    n = int(np.asarray(gpu_codes).size)
    ties, errors = u8_compare(gpu_codes, oracle_u, tie_band)
    x = 255.0 * np.asarray(oracle_u, dtype=np.float64)
    halves = int((np.abs(x - np.floor(x) - 0.5) <= 1e-6).sum())
    bound = halves + max(2, int(np.ceil(max_tie_frac * n)))
    print("%s: uint8 ties %d of %d (%.2e; %d oracle values are halves), bound %d, errors %d"
          % (label, ties, n, ties / max(1, n), halves, bound, errors))
    assert errors == 0, (label, errors)
    assert ties <= bound, (label, ties, bound)
    return ties


def check_adjoint(got, V32, G, label, mca_slice=None, **kw):
    """Adjoint parity against the FP64 oracle: max |got - ref| <= bar x max |ref|
    with bar = max(1e-5, 4 x the FP32 Monte Carlo arithmetic spread of the
    gradient at this input; oracle.mca).  The spread is taken on
    V32[mca_slice] (a representative part of a large batch) when given."""
    import oracle
    from oracle import mca

    V64 = np.asarray(V32, dtype=np.float32).astype(np.float64)
    G64 = np.asarray(G, dtype=np.float32).astype(np.float64)
    okw = {k: v for k, v in kw.items() if k in ("beta", "keps", "h", "nbw")}
    ref = oracle.backward(V64, G64, **okw)
    sl = slice(None) if mca_slice is None else mca_slice
    bar, spread = mca.adjoint_bar(V64[sl], G64[sl], ref[sl], **okw)
    scale = float(np.abs(ref).max())
    err = float(np.abs(np.asarray(got, dtype=np.float64) - ref).max()) / max(scale, 1e-300)
    print("%s: adjoint rel err %.2e, FP32 Monte Carlo spread %.2e, bar %.2e" % (label, err, spread, bar))
    assert err <= bar, (label, err, bar)
    return err
