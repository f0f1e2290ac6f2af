"""Sample magnitudes.  The method is defined for any real samples, but the
FP32 kernels square indicator sums: the doubling's weights 1/t^2 leave the
normal FP32 range once t = eps + D exceeds ~1e19 (samples ~1e9), and the
resampler's beta = 2 weights E0^2 / (E0^2 + k E1^2) overflow once E0 exceeds
~1.8e19 (samples ~8e8).  The supported range is |samples| <= 1e8; these
tests pin parity with the FP64 oracle across it, relative to the output's
magnitude, from 1e-6 to 1e8."""
import numpy as np
import pytest
import torch

import oracle
from oracle import resample as R
from conftest import check_adjoint
from workloads import random_plane

pytestmark = pytest.mark.gpu
SCALES = [1e-6, 1e-2, 1.0, 1e4, 1e8]


def _f32(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _plane(h, w, seed, scale):
    V = random_plane(h, w, seed=seed, kind="steps") * 0.7 + 0.3 * random_plane(h, w, seed=seed + 1, kind="uniform")
    return (V * scale).astype(np.float32)


def _close(got, ref, rel=1e-5):
    assert np.isfinite(got).all()
    return np.abs(got - ref).max() <= rel * np.abs(ref).max()


@pytest.mark.parametrize("scale", SCALES)
def test_doubling_across_magnitudes(gpu, scale):
    gpu.set_launch_config(0, 0)
    V = _plane(37, 150, seed=11, scale=scale)
    got = gpu.zoom2x(_f32(V)).cpu().numpy()
    assert _close(got, oracle.zoom2x(V.astype(np.float64))), scale


@pytest.mark.parametrize("scale", SCALES)
@pytest.mark.parametrize("out", [(23, 101), (80, 333)])
def test_resample_across_magnitudes(gpu, scale, out):
    V = _plane(41, 170, seed=13, scale=scale)
    got = gpu.resample(_f32(V), *out).cpu().numpy()
    assert _close(got, R.tensor_resample(V.astype(np.float64), *out)), (scale, out)


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e4])
def test_adjoint_across_magnitudes(gpu, scale):
    """The map is homogeneous of degree one where eps is negligible, so the
    gradient keeps its magnitude across sample scales; parity with the FP64
    hand adjoint within the bar of conftest.check_adjoint."""
    V = _plane(29, 90, seed=17, scale=scale)
    G = np.random.default_rng(17).standard_normal((58, 180)).astype(np.float32)
    got = gpu.zoom2x_backward(_f32(V), _f32(G)).cpu().numpy()
    assert np.isfinite(got).all()
    check_adjoint(got, V, G, "adjoint at scale %g" % scale)
