"""Execution contract of the C ABI on the GPU: calls are asynchronous on the
caller's stream, enqueue kernels only (so they can be captured into a HIP
graph and replayed), and may come from several host threads at once.
Every graph is replayed several times with eager work and synchronisations in
between, and every replay is checked against the eager result."""
import threading

import numpy as np
import pytest
import torch

from workloads import random_plane, scene_rgb

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                                   # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = fn()
    return g, res


def test_single_doubling_graph_replay(gpu):
    gpu.set_launch_config(0, 0)
    x = torch.tensor(random_plane(77, 150, seed=5, kind="steps").astype(np.float32), device="cuda")
    eager = gpu.zoom2x(x)
    out = torch.empty_like(eager)
    g, _ = _capture(lambda: gpu.zoom2x_(x, out))
    for k in range(4):
        out.fill_(float("nan"))
        _ = gpu.zoom2x(x * 0.5)                # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k


def test_batched_plan_graph_replay(gpu):
    gpu.set_launch_config(0, 0)
    shapes = [(40, 61), (7, 130), (90, 33), (1, 1), (64, 64)]
    xs = [torch.tensor(scene_rgb(h, w, seed=70 + i, n_polygons=5), device="cuda").permute(2, 0, 1)
          for i, (h, w) in enumerate(shapes)]
    refs = [gpu.zoom2x(x) for x in xs]
    outs = [torch.empty_like(r) for r in refs]
    plan = gpu.BatchedZoom(xs, outs)           # the table is uploaded here, outside the capture
    g, _ = _capture(plan.run)
    for k in range(4):
        for o in outs:
            o.zero_()
        plan2 = gpu.zoom2x_batched(xs[:2])     # another plan and launch between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r), k
        del plan2


def test_backward_graph_replay(gpu):
    gpu.set_backward_launch_config(0)
    rng = np.random.default_rng(12)
    x = torch.tensor(rng.random((3, 40, 57), dtype=np.float32), device="cuda")
    gy = torch.tensor(rng.standard_normal((3, 80, 114)).astype(np.float32), device="cuda")
    eager = gpu.zoom2x_backward(x, gy)
    g, res = _capture(lambda: gpu.zoom2x_backward(x, gy))
    for k in range(4):
        res.fill_(float("nan"))
        _ = gpu.zoom2x_backward(x, gy * 2.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, eager), k


@pytest.mark.parametrize("op,shape,out", [("zoom_to", (45, 70), (130, 201)),     # doublings + fused resampler
                                          ("resample", (30, 1500), (17, 70))])  # the two-pass resampler
def test_zoom_to_and_resample_graph_replay(gpu, op, shape, out):
    x = torch.tensor(random_plane(*shape, seed=8, kind="steps").astype(np.float32), device="cuda")
    fn = gpu.zoom_to if op == "zoom_to" else gpu.resample
    size = gpu.zoom_to_workspace_bytes if op == "zoom_to" else gpu.resample_workspace_bytes
    ws = torch.empty(size(x, *out), dtype=torch.uint8, device="cuda")
    eager = fn(x, *out, workspace=ws)
    g, res = _capture(lambda: fn(x, *out, workspace=ws))
    for k in range(4):
        res.fill_(float("nan"))
        ws.fill_(255)                          # stale workspace contents must not matter
        _ = fn(x * 0.5, *out)                  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, eager), k


def test_calls_on_a_side_stream(gpu):
    gpu.set_launch_config(0, 0)
    x = torch.tensor(random_plane(100, 200, seed=9, kind="uniform").astype(np.float32), device="cuda")
    ref = gpu.zoom2x(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        y = gpu.zoom2x(x)
        gx = gpu.zoom2x_backward(x, torch.ones_like(y))
    s.synchronize()
    assert torch.equal(y, ref)
    assert torch.isfinite(gx).all()


def test_stream_handle_is_torchs_current_stream(gpu):
    dev = torch.device("cuda", 0)
    assert gpu._stream(dev) == torch.cuda.current_stream(dev).cuda_stream
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert gpu._stream(dev) == s.cuda_stream
    assert gpu._stream(dev) == torch.cuda.current_stream(dev).cuda_stream


def test_concurrent_host_threads(gpu):
    gpu.set_launch_config(0, 0)
    inputs = [torch.tensor(random_plane(60 + 7 * i, 90 + 11 * i, seed=20 + i, kind="steps").astype(np.float32),
                           device="cuda") for i in range(6)]
    refs = [gpu.zoom2x(x) for x in inputs]
    torch.cuda.synchronize()
    results = [None] * len(inputs)
    errors = []

    def work(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                out = None
                for _ in range(20):
                    out = gpu.zoom2x(inputs[i])
            s.synchronize()
            results[i] = out
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(inputs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for r, ref in zip(results, refs):
        assert torch.equal(r, ref)
