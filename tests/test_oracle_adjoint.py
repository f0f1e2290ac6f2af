"""The oracle's hand adjoint against torch FP64 autograd (through the
independent torch restatement) and against central finite differences of
the C forward, borders included."""
import numpy as np
import pytest
import torch

from oracle import torch_ref
from workloads import random_plane


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (16, 16), (9, 14)])
@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
def test_adjoint_matches_autograd(oracle_mod, shape, beta):
    rng = np.random.default_rng(sum(shape))
    V = random_plane(*shape, seed=4, kind="steps") + 0.1 * rng.random(shape)
    G = rng.standard_normal((2 * shape[0], 2 * shape[1]))
    gv = oracle_mod.backward(V, G, beta=beta)
    Vt = torch.tensor(V, requires_grad=True)
    (torch_ref.zoom2x(Vt, beta=beta) * torch.tensor(G)).sum().backward()
    ref = Vt.grad.numpy()
    assert np.abs(gv - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_adjoint_finite_differences(oracle_mod):
    rng = np.random.default_rng(1)
    V = rng.random((16, 16))
    G = rng.standard_normal((32, 32))
    gv = oracle_mod.backward(V, G, beta=2.0)
    step = 1e-6
    for (I, J) in [(0, 0), (0, 15), (15, 0), (7, 8), (3, 12), (15, 15), (1, 1), (8, 0)]:
        Vp = V.copy()
        Vm = V.copy()
        Vp[I, J] += step
        Vm[I, J] -= step
        fd = ((oracle_mod.zoom2x(Vp) - oracle_mod.zoom2x(Vm)) * G).sum() / (2 * step)
        assert abs(fd - gv[I, J]) <= 1e-5 * max(1.0, abs(fd)), (I, J, fd, gv[I, J])


def test_torch_gradcheck_16x16():
    rng = np.random.default_rng(2)
    V = torch.tensor(rng.random((16, 16)), requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: torch_ref.zoom2x(v, beta=2.0), (V,), eps=1e-6, atol=1e-5)


@pytest.mark.parametrize("kind", ["binary", "steps"])
def test_adjoint_beta0_is_the_transpose(oracle_mod, kind):
    # beta = 0 makes every weight 0.5 / t^0 = 0.5, so the doubling is a
    # linear map A and its adjoint is exactly A^T: <A d, g> = <d, A^T g> for
    # any d, with no finite-difference error.  k_eps = 0 leaves the
    # indicators of flat regions at 0, where the weights must stay constant.
    rng = np.random.default_rng(7)
    V = random_plane(11, 14, seed=3, kind=kind)
    D = rng.standard_normal(V.shape)
    G = rng.standard_normal((22, 28))
    gv = oracle_mod.backward(V, G, beta=0.0, keps=0.0)
    assert np.isfinite(gv).all()
    lhs = (oracle_mod.zoom2x(D, beta=0.0, keps=0.0) * G).sum()
    assert abs(lhs - (D * gv).sum()) <= 1e-12 * max(1.0, abs(lhs))
    # and eps plays no part in it
    assert np.array_equal(gv, oracle_mod.backward(V, G, beta=0.0, keps=1e-8))
