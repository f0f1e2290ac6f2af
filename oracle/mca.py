"""Monte Carlo arithmetic on the oracle: how far rounding at FP32 precision
can move the WD-WENO adjoint, and the parity bar for an FP32 adjoint derived
from it.

TEST INFRASTRUCTURE ONLY (like the rest of this package).

Monte Carlo arithmetic (D. S. Parker, "Monte Carlo arithmetic: exploiting
randomness in floating-point arithmetic", 1997) replaces each rounding of a
computation by a random relative perturbation of the size of the unit
roundoff; the spread of the results over a few draws estimates the rounding
error any evaluation of the same formulas at that precision can suffer.  Here
every intermediate of the forward formulas of the vectorised restatement
(torch_ref: candidates, stencil differences, indicators, eps + D, weights,
their sum, blends) is multiplied by 1 + u or 1 - u (u the FP32 unit
roundoff, the sign drawn at random per element), and the FP64 autograd
gradient is taken through the perturbed evaluation.  Full-size (rather than
uniformly distributed) perturbations make the largest deviation over four
draws stable to within a factor of about 1.5 from seed to seed.

Where the gradient is well conditioned the spread is ~1e-7 of its largest
entry; next to flat regions (t = eps + D close to eps, eq. alpha) it grows to
1e-5 .. 1e-3, because du/dt = -beta omega (p - u) / t divides by t there.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24       # unit roundoff of FP32
ADJ_FLOOR = 1e-5       # bar where the gradient is well conditioned (relative to max |ref|)
ADJ_MCA_FACTOR = 2.0   # margin over the spread (kernel errors measured at <= 0.9 of it)


def adjoint_spread(V, G, ref, draws=4, seed=0, beta=2.0, keps=1e-8, h=1.0, nbw=None) -> float:
    """Largest distance of `draws` Monte Carlo arithmetic gradients from the
    exact adjoint `ref` (dL/dV for dL/dU = G at V), relative to max |ref|."""
    import torch

    from . import torch_ref

    gen = torch.Generator().manual_seed(seed)

    def rnd(t):
        sign = 2.0 * torch.randint(0, 2, t.shape, generator=gen).to(torch.float64) - 1.0
        return t * (1.0 + U32 * sign)

    V64 = torch.tensor(np.asarray(V, dtype=np.float64))
    G64 = torch.tensor(np.asarray(G, dtype=np.float64))
    worst = 0.0
    for _ in range(draws):
        x = V64.clone().requires_grad_(True)
        (torch_ref.zoom2x(x, beta=beta, keps=keps, h=h, nbw=nbw, rounding=rnd) * G64).sum().backward()
        worst = max(worst, float(np.abs(x.grad.numpy() - ref).max()))
    return worst / max(float(np.abs(ref).max()), 1e-300)


def adjoint_bar(V, G, ref, **kw):
    """(bar, spread): the parity bar of an FP32 adjoint, max |got - ref| <=
    bar * max |ref|, with bar = max(ADJ_FLOOR, ADJ_MCA_FACTOR * spread)."""
    spread = adjoint_spread(V, G, ref, **kw)
    return max(ADJ_FLOOR, ADJ_MCA_FACTOR * spread), spread
