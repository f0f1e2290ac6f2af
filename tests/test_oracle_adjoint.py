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


def test_backward_of_many_planes_is_per_plane(oracle_mod):
    # the multi-plane entry runs the planes on separate threads: same numbers
    rng = np.random.default_rng(2)
    V = rng.random((5, 17, 23))
    G = rng.standard_normal((5, 34, 46))
    many = oracle_mod.backward(V, G)
    for c in range(5):
        assert np.array_equal(many[c], oracle_mod.backward(V[c], G[c]))


def test_mca_spread_measures_fp32_conditioning(oracle_mod):
    """Monte Carlo arithmetic at FP32 unit roundoff (oracle.mca): small where
    the gradient is well conditioned, large next to flat regions where the
    adjoint divides by t = eps + D close to eps (eq. alpha)."""
    from oracle import mca

    rng = np.random.default_rng(1)
    G = rng.standard_normal((66, 142))
    smooth = random_plane(33, 71, seed=9, kind="uniform").astype(np.float32).astype(np.float64)
    steps = random_plane(33, 71, seed=9, kind="steps").astype(np.float32).astype(np.float64)
    s_smooth = mca.adjoint_spread(smooth, G, oracle_mod.backward(smooth, G))
    s_steps = mca.adjoint_spread(steps, G, oracle_mod.backward(steps, G, beta=3.0), beta=3.0)
    assert 1e-8 < s_smooth < 1e-6
    assert s_steps > 1e-5
    bar, spread = mca.adjoint_bar(smooth, G, oracle_mod.backward(smooth, G))
    assert bar == mca.ADJ_FLOOR and spread == s_smooth


def test_mca_rounding_hook_is_the_restatement(oracle_mod):
    # no perturbation: the hooked restatement is the plain one, bit for bit
    V = torch.tensor(random_plane(9, 13, seed=2, kind="steps"))
    a = torch_ref.zoom2x(V)
    b = torch_ref.zoom2x(V, rounding=lambda t: t)
    assert torch.equal(a, b)
    # one unit roundoff per intermediate moves the forward by a few units
    gen = torch.Generator().manual_seed(0)
    from oracle import mca

    c = torch_ref.zoom2x(V, rounding=lambda t: t * (1 + mca.U32 * (2 * torch.rand(t.shape, generator=gen,
                                                                                   dtype=torch.float64) - 1)))
    rel = float((c - a).abs().max() / a.abs().max())
    assert 1e-9 < rel < 1e-6
