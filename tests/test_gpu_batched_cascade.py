"""GPU: one persistent launch over many uneven images (bit-identical to the
per-image kernel) and the three-level cascade against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from workloads import batch_shapes, pixel_art, scene_rgb

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.mark.parametrize("cfg", [(64, 2), (16, 1)])
def test_batched_bit_identical_to_single(gpu, cfg):
    gpu.set_launch_config(*cfg)
    shapes = batch_shapes(24, seed=3, lo=1, hi=300)
    imgs = [scene_rgb(h, w, seed=100 + i, n_polygons=5) for i, (h, w) in enumerate(shapes)]
    xs = [torch.tensor(im, device="cuda").permute(2, 0, 1) for im in imgs]
    ys = gpu.zoom2x_batched(xs)
    torch.cuda.synchronize()
    for x, y in zip(xs, ys):
        ref = gpu.zoom2x(x)
        assert torch.equal(y, ref)


def test_batched_f32_against_oracle(gpu):
    gpu.set_launch_config(64, 2)
    shapes = [(1, 1), (3, 200), (130, 4), (64, 64), (129, 257)]
    rng = np.random.default_rng(1)
    xs = [torch.tensor(rng.random((2, h, w)).astype(np.float32), device="cuda") for h, w in shapes]
    plan = gpu.BatchedZoom(xs, [torch.empty((2, 2 * h, 2 * w), device="cuda") for h, w in shapes])
    for _ in range(3):  # the plan can be run again; the queue head is reset by a kernel
        ys = plan.run()
    torch.cuda.synchronize()
    for x, y in zip(xs, ys):
        ref = oracle.zoom2x(x.cpu().numpy().astype(np.float64))
        assert np.abs(y.cpu().numpy() - ref).max() <= TOL


@pytest.mark.parametrize("hw", [(32, 32), (21, 37)])   # odd widths use pitched intermediates
def test_cascade_three_levels(gpu, hw):
    gpu.set_launch_config(64, 2)
    img = pixel_art(*hw, seed=1, block=8, n_lines=4)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    yf = gpu.zoom2x_cascade(x, 3, out_dtype=torch.float32).permute(1, 2, 0).cpu().numpy()
    ref = oracle.cascade(np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0, 3)
    assert np.abs(np.transpose(yf, (2, 0, 1)) - ref).max() <= TOL
    y8 = gpu.zoom2x_cascade(x, 3).permute(1, 2, 0).cpu().numpy()
    from conftest import check_u8

    check_u8(np.transpose(y8, (2, 0, 1)), ref, "cascade %s" % (hw,))


def test_cascade_graph_replay(gpu):
    gpu.set_launch_config(64, 2)
    img = pixel_art(48, 40, seed=2, block=8, n_lines=5)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    eager = gpu.zoom2x_cascade(x, 3)
    ws = torch.empty(gpu.cascade_workspace_bytes(x, 3), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gpu.zoom2x_cascade(x, 3, workspace=ws)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = gpu.zoom2x_cascade(x, 3, workspace=ws)
    for _ in range(4):
        res.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, eager)


def test_cascade_into_callers_output(gpu):
    rng = np.random.default_rng(21)
    x = torch.tensor(rng.integers(0, 256, size=(37, 53, 3), dtype=np.uint8), device="cuda").permute(2, 0, 1)
    ref = gpu.zoom2x_cascade(x, 2)
    out = torch.empty((148, 212, 3), dtype=torch.uint8, device="cuda").permute(2, 0, 1)
    assert gpu.zoom2x_cascade(x, 2, out=out) is out
    assert torch.equal(out, ref)
    # planar float32 output of the same cascade
    ref_f = gpu.zoom2x_cascade(x, 2, out_dtype=torch.float32)
    out_f = torch.empty((3, 148, 212), dtype=torch.float32, device="cuda")
    gpu.zoom2x_cascade(x, 2, out=out_f, out_dtype=torch.float32)
    assert torch.equal(out_f, ref_f)
    with pytest.raises(ValueError):
        gpu.zoom2x_cascade(x, 2, out=torch.empty((3, 148, 211), dtype=torch.uint8, device="cuda"))


def _chain(gpu, x, levels, beta, out_dtype):
    """The cascade as separate doublings through the public single-level call:
    level l on spacing 2^-l (the default neighbour weight follows h^2/8)."""
    cur = x
    for lvl in range(levels):
        last = lvl == levels - 1
        cur = gpu.zoom2x(cur, gpu.Params(beta=beta, h=2.0 ** -lvl),
                         out_dtype=(out_dtype if last else torch.float32))
    return cur


@pytest.mark.parametrize("levels,hw,beta", [(2, (40, 56), 2.0), (3, (32, 32), 2.0), (3, (21, 37), 1.0),
                                            (4, (9, 13), 1.5), (3, (256, 256), 2.0), (2, (1, 70), 2.0)])
def test_cascade_equals_separate_doublings(gpu, levels, hw, beta):
    # the cascade (planar float32 intermediates in its workspace) against one
    # public doubling per level with the spacing halved: bit-identical, for
    # float32 and uint8 outputs
    img = pixel_art(*hw, seed=3, block=4, n_lines=5)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    ws = torch.empty(gpu.cascade_workspace_bytes(x, levels), dtype=torch.uint8, device="cuda")
    for out_dtype in (torch.float32, torch.uint8):
        y = gpu.zoom2x_cascade(x, levels, gpu.Params(beta=beta), out_dtype=out_dtype, workspace=ws)
        ref = _chain(gpu, x, levels, beta, out_dtype)
        assert torch.equal(y, ref), (levels, hw, beta, out_dtype)


def test_cascade_many_planes_f32(gpu):
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.random((5, 3, 23, 130), dtype=np.float32), device="cuda")
    ws = torch.empty(gpu.cascade_workspace_bytes(x, 3), dtype=torch.uint8, device="cuda")
    for _ in range(3):
        y = gpu.zoom2x_cascade(x, 3, workspace=ws)
        assert torch.equal(y, _chain(gpu, x, 3, 2.0, torch.float32))
