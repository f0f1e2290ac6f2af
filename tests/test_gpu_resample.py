"""GPU parity of weno_resample and weno_zoom_to (Section 3.3) against the
FP64 oracle."""
import numpy as np
import pytest
import torch

from conftest import check_u8
from oracle import resample as R
from workloads import pixel_art, random_plane, scene_rgb

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _t(a, dtype=np.float32):
    return torch.tensor(np.ascontiguousarray(a, dtype=dtype), device="cuda")


@pytest.mark.parametrize("shape,out", [((9, 11), (17, 5)), ((40, 70), (100, 33)), ((1, 5), (3, 9)), ((64, 64), (64, 64)),
                                       ((130, 97), (257, 401)), ((50, 3), (7, 2)), ((7, 1), (13, 4)), ((1, 1), (3, 5)),
                                       ((6, 2), (1, 1))])
@pytest.mark.parametrize("beta", [2.0, 1.0])
def test_resample_f32(gpu, shape, out, beta):
    V = random_plane(*shape, seed=shape[0], kind="steps") * 0.6 + 0.4 * random_plane(*shape, seed=1)
    got = gpu.resample(_t(V), *out, gpu.Params(beta=beta)).cpu().numpy()
    ref = R.tensor_resample(V.astype(np.float32).astype(np.float64), *out, beta=beta)
    assert np.abs(got - ref).max() <= TOL


def test_resample_u8_hwc(gpu):
    img = scene_rgb(60, 90, seed=3, n_polygons=8)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    y = gpu.resample(x, 133, 211)
    ref = R.tensor_resample(np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0, 133, 211)
    check_u8(y.cpu().numpy(), ref, "resample u8 HWC")


@pytest.mark.parametrize("shape,out", [((7, 9), (13, 17)), ((20, 30), (57, 88)), ((33, 40), (20, 25)),
                                       ((16, 16), (100, 61))])
def test_zoom_to_f32(gpu, shape, out):
    V = random_plane(*shape, seed=7, kind="steps") * 0.5 + 0.5 * random_plane(*shape, seed=8)
    got = gpu.zoom_to(_t(V), *out).cpu().numpy()
    ref = R.zoom_to(V.astype(np.float32).astype(np.float64), *out)
    assert got.shape == ref.shape
    print("zoom_to %s -> %s: max-abs error %.3e" % (shape, out, np.abs(got - ref).max()))
    assert np.abs(got - ref).max() <= TOL


def test_zoom_to_scale3_pixel_art_u8(gpu):
    # the paper's scale-3 example: over-zoom to (4n-3) and resample to 3n
    img = pixel_art(32, 40, seed=6, block=4, n_lines=5)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    y = gpu.zoom_to(x, 96, 120)
    ref = R.zoom_to(np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0, 96, 120)
    check_u8(y.cpu().numpy(), ref, "zoom_to scale 3 pixel art")


def test_quality_protocol_runs(gpu):
    # the paper's crop / downsample / upsample protocol: nested-grid nodes of
    # the WD-WENO result are the downsampled samples themselves
    import quality
    from workloads import to_planar_f32

    img = torch.tensor(to_planar_f32(scene_rgb(129, 193, seed=11, n_polygons=10)), device="cuda")
    res = quality.protocol(img, 2)
    assert set(res) == {"wd_weno", "tensor_weno", "bicubic", "bilinear"}
    for p, s in res.values():
        assert 10.0 < p < 80.0 and 0.0 < s <= 1.0
    up = gpu.zoom_to(img[:, ::2, ::2].contiguous(), 129, 193)
    assert torch.equal(up[:, ::2, ::2], img[:, ::2, ::2])


@pytest.mark.parametrize("pair", ["u8->f32", "f32->u8"])
def test_resample_mixed_dtypes(gpu, pair):
    V = random_plane(37, 53, seed=4, kind="steps") * 0.6 + 0.4 * random_plane(37, 53, seed=5)
    if pair == "u8->f32":
        img = (V * 255.0).round().astype(np.uint8)
        got = gpu.resample(_t(img, np.uint8), 71, 30, out_dtype=torch.float32).cpu().numpy()
        ref = R.tensor_resample(img.astype(np.float64) / 255.0, 71, 30)
        assert np.abs(got - ref).max() <= TOL
    else:
        V32 = V.astype(np.float32)
        got = gpu.resample(_t(V32), 71, 30, out_dtype=torch.uint8).cpu().numpy()
        ref = R.tensor_resample(V32.astype(np.float64), 71, 30)
        check_u8(got, ref, "resample f32->u8")


@pytest.mark.parametrize("shape,out", [((41, 77), (150, 301)), ((25, 33), (97, 40))])
def test_zoom_to_odd_widths_two_levels(gpu, shape, out):
    # two doublings through pitched float intermediates of odd widths
    V = random_plane(*shape, seed=17, kind="steps") * 0.5 + 0.5 * random_plane(*shape, seed=18)
    got = gpu.zoom_to(_t(V), *out).cpu().numpy()
    ref = R.zoom_to(V.astype(np.float32).astype(np.float64), *out)
    print("zoom_to odd widths %s -> %s: max-abs error %.3e" % (shape, out, np.abs(got - ref).max()))
    assert np.abs(got - ref).max() <= TOL


@pytest.mark.parametrize("op", ["resample", "zoom_to"])
def test_beta0_without_eps(gpu, op):
    # beta = 0 allows k_eps = 0: the weights are the ideal C_0, C_1 even where
    # both indicators vanish (flat regions), never 0/0
    V = random_plane(31, 47, seed=23, kind="binary").astype(np.float32)
    p = gpu.Params(beta=0.0, k_eps=0.0)
    if op == "resample":
        got = gpu.resample(_t(V), 45, 70, p).cpu().numpy()
        ref = R.tensor_resample(V.astype(np.float64), 45, 70, beta=0.0, keps=0.0)
    else:
        got = gpu.zoom_to(_t(V), 100, 151, p).cpu().numpy()
        ref = R.zoom_to(V.astype(np.float64), 100, 151, beta=0.0, keps=0.0)
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= TOL


# width ratios 0.58, 1.7, 2.3 (LDS rows of 512 samples per tile), 10.7 (768),
# 14 (1024) and 20.2 (beyond the fused kernel: row pass, then column pass)
@pytest.mark.parametrize("shape,out", [((300, 700), (517, 1201)), ((517, 1201), (300, 700)), ((97, 3001), (40, 1291)),
                                       ((257, 1031), (96, 97)), ((40, 1400), (20, 101)), ((20, 2000), (10, 100))])
def test_resample_many_tiles(gpu, shape, out):
    # several column tiles and row runs per plane, ragged at both ends, 3 planes
    V = np.stack([random_plane(*shape, seed=30 + c, kind="steps") * 0.6 + 0.4 * random_plane(*shape, seed=40 + c)
                  for c in range(3)]).astype(np.float32)
    got = gpu.resample(_t(V), *out).cpu().numpy()
    ref = R.tensor_resample(V.astype(np.float64), *out)
    assert np.abs(got - ref).max() <= TOL


def test_resample_u8_hwc_many_tiles(gpu):
    img = scene_rgb(211, 640, seed=12, n_polygons=12)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    y = gpu.resample(x, 300, 913)
    ref = R.tensor_resample(np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0, 300, 913)
    check_u8(y.cpu().numpy(), ref, "resample u8 HWC many tiles")


def test_resample_nodes_are_copies(gpu):
    # an output grid of 2n - 1 samples puts every other sample on an input
    # node: those are the input values bit for bit
    V = random_plane(123, 301, seed=9, kind="uniform").astype(np.float32)
    got = gpu.resample(_t(V), 245, 601).cpu().numpy()
    assert np.array_equal(got[::2, ::2], V)


@pytest.mark.parametrize("shape,out", [((400, 300), (37, 250)), ((301, 64), (99, 64)), ((64, 40), (16, 40))])
def test_resample_row_window_steps(gpu, shape, out):
    # vertical ratios 11.1, 3.06 and 4.2: consecutive output rows advance the
    # interval by 3 or 4 and more rows, the window steps that reload most or
    # all of its rows
    V = random_plane(*shape, seed=shape[0], kind="steps").astype(np.float32) * 0.7 + 0.3 * random_plane(*shape, seed=3)
    V = V.astype(np.float32)
    got = gpu.resample(_t(V), *out).cpu().numpy()
    ref = R.tensor_resample(V.astype(np.float64), *out)
    assert np.abs(got - ref).max() <= TOL


def test_caller_output_and_workspace(gpu):
    # caller-owned output (here an HWC view) and workspace: same result as
    # the allocating call, and repeated calls reuse them
    V = random_plane(30, 44, seed=2, kind="steps").astype(np.float32)
    x = _t(np.stack([V, V * 0.5, 1.0 - V]))
    ref = gpu.resample(x, 47, 61)
    out = torch.empty((47, 61, 3), device="cuda").permute(2, 0, 1)
    ws = torch.empty(gpu.resample_workspace_bytes(x, 47, 61), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        out.fill_(float("nan"))
        assert gpu.resample(x, 47, 61, workspace=ws, out=out) is out
        assert torch.equal(out, ref)
    ref2 = gpu.zoom_to(x, 100, 150)
    out2 = torch.empty_like(ref2)
    ws2 = torch.empty(gpu.zoom_to_workspace_bytes(x, 100, 150), dtype=torch.uint8, device="cuda")
    assert torch.equal(gpu.zoom_to(x, 100, 150, workspace=ws2, out=out2), ref2)
    with pytest.raises(ValueError):
        gpu.resample(x, 47, 61, out=torch.empty((3, 47, 60), device="cuda"))
