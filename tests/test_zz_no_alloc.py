"""GPU: weno_zoom2x_batched_noalloc (the batched doubling without a caller
workspace: image table and queue head in the library's fixed device array)
against weno_zoom2x_batched with a workspace, bit for bit, on consecutive
calls of shrinking size, at the maximum image count, and against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2312_00229_amd import _lib
from workloads import batch_shapes, scene_rgb

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _inputs(n, seed, lo, hi):
    shapes = batch_shapes(n, seed=seed, lo=lo, hi=hi)
    rng = np.random.default_rng(seed)
    xs = []
    for i, (h, w) in enumerate(shapes):
        if i % 3 == 2:   # float32 planar among the uint8 HWC images
            xs.append(torch.tensor(rng.random((3, h, w)).astype(np.float32), device="cuda"))
        else:
            xs.append(torch.tensor(scene_rgb(h, w, seed=seed + i, n_polygons=4), device="cuda").permute(2, 0, 1))
    return xs


@pytest.mark.parametrize("cfg", [(0, 0), (16, 1)])
def test_noalloc_matches_workspace_call_twice(gpu, cfg):
    gpu.set_launch_config(*cfg)
    try:
        for n, seed, hi in ((40, 5, 400), (7, 6, 90)):        # the second call is smaller
            xs = _inputs(n, seed, 1, hi)
            print("noalloc call: %d images up to %d px, launch config %s" % (n, hi, cfg), flush=True)
            got = gpu.zoom2x_batched_noalloc(xs)
            ref = gpu.zoom2x_batched(xs)
            torch.cuda.synchronize()
            for x, a, b in zip(xs, got, ref):
                assert a.shape == b.shape and a.dtype == b.dtype
                assert torch.equal(a, b)
            # and the float32 images against the oracle
            for x, a in zip(xs, got):
                if x.dtype == torch.float32:
                    ref = oracle.zoom2x(x.cpu().numpy().astype(np.float64))
                    assert np.abs(a.cpu().numpy() - ref).max() <= TOL
    finally:
        gpu.set_launch_config(0, 0)


def test_noalloc_float_against_oracle(gpu):
    rng = np.random.default_rng(9)
    shapes = [(1, 1), (5, 130), (67, 3), (64, 64)]
    xs = [torch.tensor(rng.random((2, h, w)).astype(np.float32), device="cuda") for h, w in shapes]
    ys = gpu.zoom2x_batched_noalloc(xs)
    torch.cuda.synchronize()
    for x, y in zip(xs, ys):
        ref = oracle.zoom2x(x.cpu().numpy().astype(np.float64))
        assert np.abs(y.cpu().numpy() - ref).max() <= TOL


def test_noalloc_maximum_count_and_beyond(gpu):
    n = _lib.WENO_NOALLOC_MAX_IMAGES
    rng = np.random.default_rng(11)
    base = torch.tensor(rng.random((n, 3, 5)).astype(np.float32), device="cuda")
    xs = [base[i] for i in range(n)]
    print("noalloc call: %d images of 3 x 5" % n, flush=True)
    got = gpu.zoom2x_batched_noalloc(xs)
    ref = gpu.zoom2x_batched(xs)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(got, ref))
    with pytest.raises(_lib.WenoError):
        gpu.zoom2x_batched_noalloc(xs + [base[0]])
