"""The C oracle against the brute-force mini-oracle and the torch restatement.

The brute force solves each stencil's Vandermonde system and integrates the
indicator of eq. (2Dsmoothness) by Gauss-Legendre quadrature, point by point;
agreement on every size up to 6x6 pins the closed forms, index bookkeeping
and neighbour sets of the C oracle."""
import numpy as np
import pytest
import torch

from oracle import brute, torch_ref
from workloads import random_plane

SIZES = [(n, m) for n in range(1, 7) for m in range(1, 7) if (n * m) % 3 == 0 or n == m or n == 1]


@pytest.mark.parametrize("n,m", SIZES)
@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0, 0.1])
def test_c_oracle_matches_brute_force(oracle_mod, n, m, beta):
    V = random_plane(n, m, seed=100 * n + m, kind="uniform")
    a = oracle_mod.zoom2x(V, beta=beta)
    b = brute.zoom2x(V, beta=beta)
    assert np.abs(a - b).max() <= 1e-12


@pytest.mark.parametrize("si_mode", [0, 1])
@pytest.mark.parametrize("nbw", [None, 0.25, 0.0])
@pytest.mark.parametrize("kind", ["uniform", "steps", "binary"])
def test_c_oracle_matches_brute_force_variants(oracle_mod, si_mode, nbw, kind):
    V = random_plane(5, 6, seed=7, kind=kind)
    for h in (1.0, 0.25):
        a = oracle_mod.zoom2x(V, beta=2.0, h=h, si_mode=si_mode, nbw=nbw)
        b = brute.zoom2x(V, beta=2.0, h=h, si_mode=si_mode, nbw=nbw)
        assert np.abs(a - b).max() <= 1e-12


@pytest.mark.parametrize("shape", [(1, 1), (2, 9), (9, 2), (13, 17)])
@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
def test_torch_restatement_matches_c_oracle(oracle_mod, shape, beta):
    V = random_plane(*shape, seed=3, kind="steps" if beta else "uniform")
    a = oracle_mod.zoom2x(V, beta=beta)
    c = torch_ref.zoom2x(torch.tensor(V), beta=beta).numpy()
    assert np.abs(a - c).max() <= 1e-12
