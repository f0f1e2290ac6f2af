"""GPU tests of the launch-configuration autotuner (single images,
batched plans and the adjoint): it picks one of its candidate configurations
(the automatic one among them), applies it, caches it, and every
configuration it tries gives bit-identical outputs."""
import numpy as np
import pytest
import torch

from workloads import random_plane, scene_rgb

pytestmark = pytest.mark.gpu


@pytest.fixture
def tune_cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("WENO_TUNE_CACHE", str(path))
    return path


def test_tune_single_image(gpu, tune_cache):
    from paper_2312_00229_amd import autotune

    x = torch.tensor(random_plane(70, 300, seed=1, kind="steps").astype(np.float32), device="cuda")
    out = torch.empty((140, 600), device="cuda")
    try:
        gpu.set_launch_config(0, 0)
        ref = gpu.zoom2x(x)
        rows, cols, times = autotune.tune(x, out, reps=2)
        # the fixed configurations and the automatic one, (0, 0)
        assert (rows, cols) in {(r, c) for r in autotune.ROWS for c in autotune.COLS} | {(0, 0)}
        assert gpu.get_launch_config() == (rows, cols)
        assert len(times) == len(autotune.ROWS) * len(autotune.COLS) + 1
        assert "0,0" in times
        assert torch.equal(gpu.zoom2x(x), ref)
        assert tune_cache.exists()
        gpu.set_launch_config(0, 0)
        rows2, cols2, _ = autotune.tune(x, out, reps=2)          # served from the cache
        assert (rows2, cols2) == (rows, cols)
    finally:
        gpu.set_launch_config(0, 0)


def test_tune_batched_plan(gpu, tune_cache):
    from paper_2312_00229_amd import autotune

    shapes = [(33, 47), (120, 90), (7, 300), (64, 64), (1, 5), (200, 31)]
    imgs = [scene_rgb(h, w, seed=50 + i, n_polygons=6) for i, (h, w) in enumerate(shapes)]
    xs = [torch.tensor(im, device="cuda").permute(2, 0, 1) for im in imgs]
    outs = [torch.empty((2 * h, 2 * w, 3), dtype=torch.uint8, device="cuda").permute(2, 0, 1) for h, w in shapes]
    try:
        gpu.set_launch_config(0, 0)
        refs = [gpu.zoom2x(x) for x in xs]
        rows, cols, times = autotune.tune_batched(xs, outs, reps=2)
        assert (rows, cols) in {(r, c) for r in autotune.ROWS_BATCHED for c in autotune.COLS}
        assert len(times) == len(autotune.ROWS_BATCHED) * len(autotune.COLS)
        plan = gpu.BatchedZoom(xs, outs)                            # captures the tuned configuration
        assert (plan.plan.rows_per_strip, plan.plan.cols_per_lane) == (rows, cols)
        for o in outs:
            o.zero_()
        plan.run()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
    finally:
        gpu.set_launch_config(0, 0)


def test_tune_backward(gpu, tune_cache):
    from paper_2312_00229_amd import autotune

    rng = np.random.default_rng(3)
    x = torch.tensor(rng.random((2, 3, 96, 130), dtype=np.float32), device="cuda")
    g = torch.tensor(rng.standard_normal((2, 3, 192, 260)).astype(np.float32), device="cuda")
    try:
        gpu.set_backward_launch_config(0)
        gpu.set_launch_config(0, 0)
        ref = gpu.zoom2x_backward(x, g)
        rows, times = autotune.tune_backward(x, g, reps=2)
        assert rows in (0,) + autotune.ROWS_BACKWARD                # 0: the automatic height
        assert len(times) == len(autotune.ROWS_BACKWARD) + 1
        assert gpu.get_backward_launch_config() == rows
        assert gpu.get_launch_config() == (0, 0)                       # the forward is left alone
        assert torch.equal(gpu.zoom2x_backward(x, g), ref)
        gpu.set_backward_launch_config(0)
        assert autotune.tune_backward(x, g, reps=2)[0] == rows        # served from the cache
    finally:
        gpu.set_backward_launch_config(0)
