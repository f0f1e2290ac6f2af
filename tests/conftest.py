import os
import sys

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
    import numpy as np

    x = 255.0 * np.asarray(oracle_u, dtype=np.float64)
    ref = np.clip(np.rint(x), 0, 255)
    g = np.asarray(gpu_codes, dtype=np.float64)
    bad = g != ref
    frac = x - np.floor(x)
    near = np.abs(frac - 0.5) < 255.0 * tie_band
    tie = bad & near & (np.abs(g - ref) <= 1)
    return int(tie.sum()), int((bad & ~tie).sum())
