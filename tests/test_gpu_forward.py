"""GPU parity of the forward kernel (weno_zoom2x through the C ABI) against
the FP64 oracle.

Bar: FP32 outputs within 1e-5 max-abs of the oracle on [0,1]-scaled data;
originals bit-exact; uint8 codes equal except counted rounding ties."""
import numpy as np
import pytest
import torch

import oracle
from conftest import check_u8
from workloads import pixel_art, random_plane, scene_rgb, smooth_grid, to_planar_f32, two_level_u8

pytestmark = pytest.mark.gpu
TOL = 1e-5
CONFIGS = [(64, 2), (64, 1), (8, 2), (16, 1), (128, 2)]


def _set(gpu, cfg):
    gpu.set_launch_config(*cfg)


def _f32(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (5, 130), (130, 5), (64, 64), (67, 250), (200, 131), (9, 119), (9, 120),
          (31, 237)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("cfg", CONFIGS)
def test_forward_matches_oracle_f32(gpu, shape, cfg):
    _set(gpu, cfg)
    V = random_plane(*shape, seed=shape[0] * 1000 + shape[1], kind="steps") * 0.7 + 0.3 * random_plane(
        *shape, seed=7, kind="uniform")
    V32 = V.astype(np.float32)
    U = gpu.zoom2x(_f32(V32)).cpu().numpy()
    ref = oracle.zoom2x(V32.astype(np.float64))
    assert U.shape == ref.shape
    assert np.abs(U - ref).max() <= TOL
    assert np.array_equal(U[0::2, 0::2], V32)  # originals bit-exact


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0, 0.5, 3.0])
@pytest.mark.parametrize("kind", ["uniform", "binary", "steps"])
def test_forward_beta(gpu, beta, kind):
    _set(gpu, (64, 2))
    V = random_plane(53, 141, seed=int(beta * 10) + 3, kind=kind).astype(np.float32)
    U = gpu.zoom2x(_f32(V), beta=beta).cpu().numpy()
    ref = oracle.zoom2x(V.astype(np.float64), beta=beta)
    assert np.abs(U - ref).max() <= TOL


@pytest.mark.parametrize("kind", ["binary", "steps"])
def test_forward_beta0_without_eps(gpu, kind):
    # beta = 0 allows k_eps = 0; flat regions then have zero indicators and
    # the weights must still be the constant 0.5 / t^0 (0^0 = 1), not NaN
    _set(gpu, (64, 2))
    V = random_plane(37, 90, seed=21, kind=kind).astype(np.float32)
    U = gpu.zoom2x(_f32(V), beta=0.0, k_eps=0.0).cpu().numpy()
    ref = oracle.zoom2x(V.astype(np.float64), beta=0.0, keps=0.0)
    assert np.isfinite(U).all()
    assert np.abs(U - ref).max() <= TOL


@pytest.mark.parametrize("nbw,h,keps", [(0.25, 1.0, 1e-8), (0.0, 1.0, 1e-8), (-1.0, 0.5, 1e-6), (-1.0, 2.0, 1e-8)])
def test_forward_parameters(gpu, nbw, h, keps):
    _set(gpu, (64, 2))
    V = random_plane(40, 70, seed=11, kind="steps").astype(np.float32)
    U = gpu.zoom2x(_f32(V), beta=2.0, k_eps=keps, h=h, nbw=nbw).cpu().numpy()
    ref = oracle.zoom2x(V.astype(np.float64), beta=2.0, keps=keps, h=h, nbw=None if nbw < 0 else nbw)
    assert np.abs(U - ref).max() <= TOL


def test_smooth_function_64(gpu):
    # the smooth accuracy case: 64 x 64 samples of the test function, 2x
    _set(gpu, (64, 2))
    V = smooth_grid(64).astype(np.float32)
    h = 1.0 / 63
    U = gpu.zoom2x(_f32(V), h=h).cpu().numpy()
    ref = oracle.zoom2x(V.astype(np.float64), h=h)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(U - ref).max() <= TOL * scale


@pytest.mark.parametrize("cfg", [(64, 2), (16, 1)])
def test_u8_hwc_scene(gpu, cfg, request):
    _set(gpu, cfg)
    img = scene_rgb(97, 263, seed=5, n_polygons=12)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)      # HWC memory, (C, H, W) view
    y = gpu.zoom2x(x)                                            # uint8, HWC-strided
    assert y.stride()[0] == 1
    codes = y.permute(1, 2, 0).cpu().numpy()                     # (2H, 2W, C)
    ref = oracle.zoom2x(np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0)
    check_u8(np.transpose(codes, (2, 0, 1)), ref, "u8 HWC scene %s" % (cfg,))
    assert np.array_equal(codes[0::2, 0::2], img)


@pytest.mark.parametrize("cfg", [(64, 2), (16, 1)])
@pytest.mark.parametrize("layout", ["plane", "hwc"])
def test_u8_exact_ties_round_half_even(gpu, cfg, layout):
    # beta = 0 on samples that are multiples of 16: every new point is a small
    # dyadic fraction, computed exactly in FP32 and FP64, and a large share of
    # them lie exactly on k + 1/2.  The codes must be those of round half to
    # even, with no tie allowance.
    _set(gpu, cfg)
    if layout == "plane":
        img = two_level_u8(53, 141, seed=7)
        x = torch.tensor(img, device="cuda")
        got = gpu.zoom2x(x, beta=0.0).cpu().numpy()
        X = oracle.zoom2x(img.astype(np.float64), beta=0.0)        # 0..255 scale
    else:
        img = two_level_u8(41, 75, seed=8, channels=3)
        x = torch.tensor(img, device="cuda").permute(2, 0, 1)
        got = np.transpose(gpu.zoom2x(x, beta=0.0).permute(1, 2, 0).cpu().numpy(), (2, 0, 1))
        X = oracle.zoom2x(np.transpose(img, (2, 0, 1)).astype(np.float64), beta=0.0)
    n_ties = int((X - np.floor(X) == 0.5).sum())
    print("exact k+1/2 values: %d of %d" % (n_ties, X.size))
    assert n_ties > 0.1 * X.size
    assert np.array_equal(got, oracle.quantize_u8_255(X))


def test_u8_to_f32_and_f32_to_u8(gpu):
    _set(gpu, (64, 2))
    img = pixel_art(40, 56, seed=4, block=4, n_lines=6)
    x8 = torch.tensor(img, device="cuda").permute(2, 0, 1)
    ref = oracle.zoom2x(np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0)
    yf = gpu.zoom2x(x8, out_dtype=torch.float32).permute(1, 2, 0).cpu().numpy()
    assert np.abs(np.transpose(yf, (2, 0, 1)) - ref).max() <= TOL
    xf = _f32(np.transpose(img, (2, 0, 1)) / 255.0)
    y8 = gpu.zoom2x(xf, out_dtype=torch.uint8).cpu().numpy()
    check_u8(y8, ref, "pixel art f32->u8")


def test_strided_views(gpu):
    _set(gpu, (64, 2))
    base = random_plane(90, 300, seed=12, kind="steps").astype(np.float32)
    t = _f32(base)
    view = t[3:80:2, 5:290:3]          # non-contiguous rows and columns
    U = gpu.zoom2x(view).cpu().numpy()
    ref = oracle.zoom2x(view.cpu().numpy().astype(np.float64))
    assert np.abs(U - ref).max() <= TOL
    # non-contiguous output
    out_big = torch.zeros((2 * view.shape[0], 4 * view.shape[1]), device="cuda")
    out = out_big[:, ::2]
    gpu.zoom2x_(view, out)
    assert np.abs(out.cpu().numpy() - ref).max() <= TOL
    assert float(out_big[:, 1::2].abs().max()) == 0.0


def test_batch_of_planes_nchw(gpu):
    _set(gpu, (32, 2))
    V = np.stack([random_plane(33, 47, seed=s, kind="steps") for s in range(6)]).reshape(2, 3, 33, 47).astype(np.float32)
    U = gpu.zoom2x(_f32(V)).cpu().numpy()
    ref = oracle.zoom2x(V.astype(np.float64))
    assert np.abs(U - ref).max() <= TOL


def test_constant_plane(gpu):
    _set(gpu, (64, 2))
    for c in (0.0, 0.25, 1.0):
        U = gpu.zoom2x(torch.full((37, 91), c, device="cuda")).cpu().numpy()
        assert np.abs(U - c).max() <= 1e-6 * max(c, 1.0)


def test_launch_configs_bit_identical(gpu):
    img = scene_rgb(150, 333, seed=9, n_polygons=10)
    x = _f32(np.transpose(img, (2, 0, 1)) / 255.0)
    outs = []
    for cfg in [(8, 1), (64, 1), (8, 2), (64, 2), (256, 2)]:
        _set(gpu, cfg)
        outs.append(gpu.zoom2x(x).cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _blocks(planes, H, W, rows, cols):
    own = 118 if cols == 2 else 55
    strips = -(-W // own) * -(-H // rows)
    return planes * -(-strips // 4)


@pytest.mark.parametrize("dtype", ["f32", "u8_hwc"])
def test_paced_and_unpaced_launches_bit_identical(gpu, dtype):
    # A launch whose workgroups all fit on the device at once runs paced (wave
    # priorities, rows written through the L2); one of several rounds does
    # not.  Same arithmetic, so the outputs must match bit for bit, and the
    # oracle.  1080p RGB: 27-row two-column strips give 510 workgroups (one
    # round: at most three per compute unit); 4-row strips give thousands.
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    img = scene_rgb(1080, 1920, seed=4, n_polygons=30)
    if dtype == "f32":
        x = _f32(to_planar_f32(img))
    else:
        x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    outs = {}
    for cfg in [(27, 2), (4, 2), (4, 1), (0, 0)]:
        _set(gpu, cfg)
        outs[cfg] = gpu.zoom2x(x).cpu().numpy()
    _set(gpu, (0, 0))
    assert _blocks(3, 1080, 1920, 27, 2) <= 3 * cus
    assert _blocks(3, 1080, 1920, 4, 2) > 3 * cus and _blocks(3, 1080, 1920, 4, 1) > 5 * cus
    for cfg, o in outs.items():
        assert np.array_equal(o, outs[(27, 2)]), cfg
    # and the oracle on a band of rows across the first strip boundaries
    planes = np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0
    ref = oracle.window_zoom2x(planes, 20, 60, 100, 260)
    got = outs[(4, 2)][:, 40:120, 200:520]
    if dtype == "f32":
        assert np.abs(got - ref).max() <= TOL
    else:
        check_u8(got, ref, "paced/unpaced u8 band")


@pytest.mark.parametrize("shape", [(3, 512, 512), (48, 512, 512), (3, 480, 640), (1, 2048, 2048), (3, 96, 173)])
@pytest.mark.parametrize("dtypes", ["f32->f32", "u8->u8", "u8->f32", "f32->u8"])
def test_tail_strips(gpu, shape, dtypes):
    # Planar images whose last strip column holds no more than a one-column
    # strip owns: the automatic launch walks it in one-column strips of
    # taller bands and numbers its waves across the planes.  Must match a
    # launch without tail strips bit for bit, and the oracle.
    _set(gpu, (0, 0))
    rng = np.random.default_rng(shape[1] * 7 + shape[2])
    img = (rng.random(shape) * 0.6 + np.linspace(0, 0.4, shape[2])[None, None, :]).astype(np.float32)
    src_u8 = dtypes.startswith("u8")
    x = torch.tensor(np.rint(img * 255).astype(np.uint8) if src_u8 else img, device="cuda")
    out_dtype = torch.uint8 if dtypes.endswith("u8") else torch.float32
    rows, cols, tail = gpu.launch_shape(x)
    if shape != (3, 96, 173):
        assert cols == 2 and tail > 0, (rows, cols, tail)
    y = gpu.zoom2x(x, out_dtype=out_dtype)
    _set(gpu, (rows, 2))
    assert gpu.launch_shape(x) == (rows, 2, 0)
    y2 = gpu.zoom2x(x, out_dtype=out_dtype)
    _set(gpu, (0, 0))
    a, b = y.cpu().numpy(), y2.cpu().numpy()
    assert np.array_equal(a, b), shape
    V = (x.cpu().numpy().astype(np.float64) / 255.0) if src_u8 else img.astype(np.float64)
    if shape[0] * shape[1] * shape[2] <= 3 * 512 * 512:
        ref = oracle.zoom2x(V)
    else:   # the last planes, on a window over the tail columns and the band boundaries
        V = V[-2:]
        a = a[-2:]
        c0 = shape[2] - 150
        ref = oracle.window_zoom2x(V, 0, 160, c0, shape[2])
        a = a[:, :320, 2 * c0:]
    if dtypes.endswith("u8"):
        check_u8(a, ref, "tail strips %s %s" % (shape, dtypes))
    else:
        assert np.abs(a - ref).max() <= TOL


def test_interleaved_and_planar_layouts_bit_identical(gpu):
    # HWC images launch on a grid padded to a multiple of the XCD count (the
    # same strip of every channel on one XCD) and take their own strip height
    # from the cost model; planar copies of the same data do neither.  Same
    # arithmetic per plane, so the results must match bit for bit.
    _set(gpu, (0, 0))
    for (h, w) in [(1080, 1920), (333, 517), (64, 4000)]:
        img = scene_rgb(h, w, seed=h + w, n_polygons=12)
        hwc = torch.tensor(img, device="cuda").permute(2, 0, 1)
        planar = hwc.contiguous()
        a = gpu.zoom2x(hwc).cpu().numpy()
        b = gpu.zoom2x(planar).cpu().numpy()
        assert np.array_equal(a, b), (h, w)
        af = gpu.zoom2x(hwc, out_dtype=torch.float32).cpu().numpy()
        bf = gpu.zoom2x(planar, out_dtype=torch.float32).cpu().numpy()
        assert np.array_equal(af, bf), (h, w)


def test_full_size_1080p_sampled(gpu):
    # 1920 x 1080 RGB uint8 scene (and its planar float32 /255 version),
    # zoomed to 3840 x 2160 in the benchmark's launch configuration (the
    # automatic one); sampled windows (including all four corners and edges)
    # checked against the oracle computed on windows of the input.
    _set(gpu, (0, 0))
    img = scene_rgb(1080, 1920, seed=0)
    x = torch.tensor(img, device="cuda").permute(2, 0, 1)
    y8 = gpu.zoom2x(x).permute(1, 2, 0).cpu().numpy()
    xf = _f32(to_planar_f32(img))
    yf = gpu.zoom2x(xf).cpu().numpy()
    planes = np.transpose(img, (2, 0, 1)).astype(np.float64) / 255.0
    rng = np.random.default_rng(0)
    windows = [(0, 0), (0, 1920 - 24), (1080 - 24, 0), (1080 - 24, 1920 - 24)]
    windows += [(int(rng.integers(0, 1080 - 24)), int(rng.integers(0, 1920 - 24))) for _ in range(6)]
    total_ties = 0
    for (r0, c0) in windows:
        ref = oracle.window_zoom2x(planes, r0, r0 + 24, c0, c0 + 24)
        got_f = yf[:, 2 * r0: 2 * r0 + 48, 2 * c0: 2 * c0 + 48]
        assert np.abs(got_f - ref).max() <= TOL, (r0, c0)
        got8 = np.transpose(y8[2 * r0: 2 * r0 + 48, 2 * c0: 2 * c0 + 48], (2, 0, 1))
        total_ties += check_u8(got8, ref, "1080p u8 window (%d, %d)" % (r0, c0))
    n_out = 3 * 48 * 48 * len(windows)
    print("1080p u8 windows: %d ties of %d" % (total_ties, n_out))
    assert total_ties <= 1e-3 * n_out
    assert np.array_equal(y8[0::2, 0::2], img)


@pytest.mark.parametrize("cfg", [(8, 2), (16, 1)])
@pytest.mark.parametrize("W", [131, 132, 1, 57])
@pytest.mark.parametrize("dtypes", ["f32->f32", "u8->u8", "u8->f32", "f32->u8"])
def test_padded_output_rows_untouched(gpu, cfg, W, dtypes):
    """Planar outputs inside a wider buffer (contiguous columns, padded rows),
    for every dtype pair: every output is written, matches the oracle, and the
    padding past each row keeps its bytes.  Covers the fixed-layout kernels
    (float rows with vector stores -- odd widths end in a half store -- and
    byte rows, whose lanes outside the image store nothing) and, where the
    padded float rows are not 16-byte aligned, the runtime-flag path."""
    _set(gpu, cfg)
    H, pad = 21, 6
    src_t, dst_t = dtypes.split("->")
    V = random_plane(H, W, seed=W, kind="steps") * 0.6 + 0.4 * random_plane(H, W, seed=3, kind="uniform")
    if src_t == "u8":
        img = (V * 255.0).round().astype(np.uint8)
        x = torch.tensor(img, device="cuda")
        ref = oracle.zoom2x(img.astype(np.float64) / 255.0)
    else:
        V32 = V.astype(np.float32)
        x = _f32(V32)
        ref = oracle.zoom2x(V32.astype(np.float64))
    if dst_t == "u8":
        big = torch.full((2 * H, 2 * W + pad), 201, dtype=torch.uint8, device="cuda")
    else:
        big = torch.full((2 * H, 2 * W + pad), -7.0, device="cuda")
    out = big[:, : 2 * W]
    gpu.zoom2x_(x, out)
    got = out.cpu().numpy()
    if dst_t == "u8":
        check_u8(got, ref, "padded rows %s W=%d %s" % (cfg, W, dtypes))
        assert bool((big[:, 2 * W:] == 201).all())
    else:
        assert np.abs(got - ref).max() <= TOL
        assert bool((big[:, 2 * W:] == -7.0).all())


@pytest.mark.parametrize("shape", [(9, 11), (40, 141), (3, 300)])
def test_external_boundary_f32(gpu, shape):
    # the input is a view into a larger array; its 4 rows/columns before and
    # 5 after are the samples beyond the plane: the result is the doubling of
    # that (H + 9) x (W + 9) region, cropped
    _set(gpu, (0, 0))
    H, W = shape
    E = random_plane(H + 12, W + 15, seed=H + W, kind="steps").astype(np.float32)
    r0, c0 = 5, 7   # the view starts at E[r0, c0]; rows r0-4 .. r0+H+4 are read
    Et = _f32(E)
    U = gpu.zoom2x(Et[r0:r0 + H, c0:c0 + W], boundary="external").cpu().numpy()
    region = E[r0 - 4:r0 + H + 5, c0 - 4:c0 + W + 5]
    ref = oracle.zoom2x(region.astype(np.float64))[8:8 + 2 * H, 8:8 + 2 * W]
    assert np.abs(U - ref).max() <= TOL
    assert np.array_equal(U[0::2, 0::2], E[r0:r0 + H, c0:c0 + W])
    # and bit for bit the library's own doubling of the region, cropped
    full = gpu.zoom2x(_f32(region)).cpu().numpy()[8:8 + 2 * H, 8:8 + 2 * W]
    assert np.array_equal(U, full)


def test_external_boundary_with_tail_strips(gpu):
    # three 512x512 planes viewed inside larger ones (ghost samples read in
    # place), launched with one-column tail strips for the last 40 columns
    _set(gpu, (0, 0))
    H = W = 512
    E = np.stack([random_plane(H + 12, W + 15, seed=70 + k, kind="steps") for k in range(3)]).astype(np.float32)
    r0, c0 = 5, 7
    Et = _f32(E)
    view = Et[:, r0:r0 + H, c0:c0 + W]
    assert gpu.launch_shape(view)[2] > 0
    U = gpu.zoom2x(view, boundary="external").cpu().numpy()
    region = E[:, r0 - 4:r0 + H + 5, c0 - 4:c0 + W + 5]
    full = gpu.zoom2x(_f32(region)).cpu().numpy()[:, 8:8 + 2 * H, 8:8 + 2 * W]
    assert np.array_equal(U, full)
    ref = oracle.window_zoom2x(region[1].astype(np.float64), 4, 60, W + 4 - 60, W + 4)
    assert np.abs(U[1, :112, 2 * (W - 60):] - ref).max() <= TOL


def test_external_boundary_u8_hwc_and_batched(gpu):
    _set(gpu, (0, 0))
    img = scene_rgb(70, 130, seed=4, n_polygons=6)
    big = torch.tensor(img, device="cuda")
    r0, c0, H, W = 6, 9, 50, 111
    view = big[r0:r0 + H, c0:c0 + W].permute(2, 0, 1)
    y = gpu.zoom2x(view, boundary="external").cpu().numpy()
    region = big[r0 - 4:r0 + H + 5, c0 - 4:c0 + W + 5].permute(2, 0, 1).contiguous()
    full = gpu.zoom2x(region).cpu().numpy()[:, 8:8 + 2 * H, 8:8 + 2 * W]
    assert np.array_equal(y, full)
    # the batched entry point reads the same ghost samples
    outs = [torch.empty((2 * H, 2 * W, 3), dtype=torch.uint8, device="cuda").permute(2, 0, 1) for _ in range(2)]
    gpu.BatchedZoom([view, view], outs, gpu.Params(boundary="external")).run()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), y)
