"""C ABI checks that need no GPU: the library loads, exports every function
include/weno_zoom.h declares, and rejects bad arguments on the host before
anything is enqueued (no device memory is touched: the pointers below are
never dereferenced because validation fails first)."""
import ctypes
import os
import re

import pytest

from paper_2312_00229_amd import _lib
from paper_2312_00229_amd._lib import WenoBatchPlan, WenoParams, WenoTensor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "weno_zoom.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(weno_\w+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("weno_zoom2x", "weno_zoom2x_batched", "weno_zoom2x_backward", "weno_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) <= set(_lib._SIGS)


def _t(ptr=0x1000, dtype=_lib.WENO_F32, n=1, c=1, h=4, w=5, contiguous=True):
    return WenoTensor(ptr, dtype, n, c, h, w, c * h * w, h * w, w, 1)


def _p(beta=2.0, keps=1e-8, h=1.0, nbw=-1.0):
    return WenoParams(beta, keps, h, nbw)


def call_zoom(src, dst, p):
    return _lib.lib().weno_zoom2x(ctypes.byref(src) if src else None, ctypes.byref(dst) if dst else None,
                                  ctypes.byref(p) if p else None, None)


def test_null_and_size_errors():
    src, dst, p = _t(), _t(ptr=0x100000, h=8, w=10), _p()
    assert call_zoom(None, dst, p) == _lib.WENO_EINVAL
    assert call_zoom(src, None, p) == _lib.WENO_EINVAL
    assert call_zoom(src, dst, None) == _lib.WENO_EINVAL
    assert call_zoom(_t(ptr=0), dst, p) == _lib.WENO_EINVAL
    assert call_zoom(_t(h=0), dst, p) == _lib.WENO_EINVAL
    assert call_zoom(src, _t(ptr=0x100000, h=8, w=9), p) == _lib.WENO_EINVAL   # not 2x
    assert call_zoom(src, _t(ptr=0x100000, c=2, h=8, w=10), p) == _lib.WENO_EINVAL


def test_plane_size_limits():
    # buffer offsets are 32-bit: every plane must span less than 2^31 bytes
    p = _p()
    big = 23171                     # a float plane of big^2 elements spans > 2^31 bytes
    assert call_zoom(_t(h=big, w=big), _t(ptr=1 << 40, h=2 * big, w=2 * big), p) == _lib.WENO_EINVAL
    # source fine (1 GiB), destination over the limit (4 GiB)
    assert call_zoom(_t(h=16384, w=16384), _t(ptr=1 << 40, h=32768, w=32768), p) == _lib.WENO_EINVAL
    # uint8 destination just over the limit: 2*23171 squared bytes
    u8 = _lib.WENO_U8
    assert call_zoom(_t(dtype=u8, h=big, w=big), _t(ptr=1 << 40, dtype=u8, h=2 * big, w=2 * big), p) == _lib.WENO_EINVAL
    # at most 65535 planes (one grid dimension)
    assert call_zoom(_t(n=65536, h=2, w=2), _t(ptr=1 << 40, n=65536, h=4, w=4), p) == _lib.WENO_EINVAL
    assert call_zoom(_t(n=256, c=256, h=2, w=2), _t(ptr=1 << 40, n=256, c=256, h=4, w=4), p) == _lib.WENO_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_dtype_error():
    assert call_zoom(_t(dtype=7), _t(ptr=0x100000, h=8, w=10), _p()) == _lib.WENO_EDTYPE


def test_overlap_error():
    src = _t(ptr=0x100000, h=4, w=5)
    dst = _t(ptr=0x100000 + 40, h=8, w=10)
    assert call_zoom(src, dst, _p()) == _lib.WENO_EOVERLAP


@pytest.mark.parametrize("p", [_p(beta=-1.0), _p(h=0.0), _p(keps=-1.0), _p(beta=float("nan")),
                               _p(keps=0.0), _p(beta=10.0, keps=1e-30)])
def test_parameter_errors(p):
    assert call_zoom(_t(), _t(ptr=0x100000, h=8, w=10), p) == _lib.WENO_EINVAL


def _plan_status(p):
    # the batched plan checks the parameters first and the workspace size
    # after them: ENOSPC (with a workspace of 0 bytes) means they passed
    L = _lib.lib()
    src = (WenoTensor * 1)(_t())
    dst = (WenoTensor * 1)(_t(ptr=0x100000, h=8, w=10))
    return L.weno_zoom2x_batched_plan(src, dst, 1, ctypes.byref(p), 0x300000, 0, None, ctypes.byref(WenoBatchPlan()))


def test_weight_sum_limit():
    # four weights t^-beta at the smallest scaled t of any kernel, (3/13) eps
    # (the adjoint's; the doubling's is eps/4), must sum below FP32's range:
    # 4 ((3/13) eps)^-beta < 2^126
    assert _plan_status(_p(beta=64.0, keps=0.35)) == _lib.WENO_EINVAL     # each weight ~2^232
    assert _plan_status(_p(beta=64.0, keps=1.1)) == _lib.WENO_EINVAL      # ~2^126.6
    assert _plan_status(_p(beta=64.0, keps=1.2)) == _lib.WENO_ENOSPC      # ~2^118.5: accepted
    assert _plan_status(_p(beta=2.0, keps=1e-8)) == _lib.WENO_ENOSPC
    assert _plan_status(_p(beta=4.0, keps=1e-8)) == _lib.WENO_ENOSPC     # 2^114.8
    assert _plan_status(_p(beta=5.0, keps=1e-8)) == _lib.WENO_EINVAL     # 2^143.5


def test_batched_noalloc_errors():
    L = _lib.lib()
    src = (WenoTensor * 2)(_t(), _t(ptr=0x2000))
    dst = (WenoTensor * 2)(_t(ptr=0x100000, h=8, w=10), _t(ptr=0x200000, h=8, w=10))
    p = _p()
    assert L.weno_zoom2x_batched_noalloc(src, dst, 0, ctypes.byref(p), None) == _lib.WENO_EINVAL
    assert L.weno_zoom2x_batched_noalloc(None, dst, 2, ctypes.byref(p), None) == _lib.WENO_EINVAL
    assert L.weno_zoom2x_batched_noalloc(src, dst, _lib.WENO_NOALLOC_MAX_IMAGES + 1, ctypes.byref(p),
                                         None) == _lib.WENO_ENOSPC
    assert L.weno_zoom2x_batched_noalloc(src, dst, 2, None, None) == _lib.WENO_EINVAL
    bad = (WenoTensor * 2)(_t(ptr=0x100000, h=8, w=10), _t(ptr=0x200000, h=8, w=9))
    assert L.weno_zoom2x_batched_noalloc(src, bad, 2, ctypes.byref(p), None) == _lib.WENO_EINVAL
    overlap = (WenoTensor * 2)(_t(ptr=0x100000, h=8, w=10), _t(ptr=0x100000 + 64, h=8, w=10))
    assert L.weno_zoom2x_batched_noalloc(src, overlap, 2, ctypes.byref(p), None) == _lib.WENO_EOVERLAP
    assert "fixed scratch" in _lib.status_string(_lib.WENO_ENOSPC)


def test_beta_zero_allows_zero_eps_validation():
    # beta = 0 gives equal weights, eps never enters; validation alone (a
    # shape error is planted so nothing is launched)
    assert call_zoom(_t(), _t(ptr=0x100000, h=8, w=9), _p(beta=0.0, keps=0.0)) == _lib.WENO_EINVAL


def test_batched_errors():
    L = _lib.lib()
    src = (WenoTensor * 2)(_t(), _t(ptr=0x2000))
    dst = (WenoTensor * 2)(_t(ptr=0x100000, h=8, w=10), _t(ptr=0x200000, h=8, w=10))
    plan = WenoBatchPlan()
    p = _p()
    ws = L.weno_zoom2x_batched_workspace(2)
    assert ws >= 256 and ws % 256 == 0
    assert L.weno_zoom2x_batched_plan(src, dst, 0, ctypes.byref(p), 0x300000, ws, None, ctypes.byref(plan)) == _lib.WENO_EINVAL
    assert L.weno_zoom2x_batched_plan(src, dst, 2, ctypes.byref(p), 0x300000, ws - 1, None, ctypes.byref(plan)) == _lib.WENO_ENOSPC
    assert L.weno_zoom2x_batched_plan(src, dst, 2, ctypes.byref(p), 0x300010, ws, None, ctypes.byref(plan)) == _lib.WENO_EINVAL
    dst_overlap = (WenoTensor * 2)(_t(ptr=0x100000, h=8, w=10), _t(ptr=0x100000 + 64, h=8, w=10))
    assert L.weno_zoom2x_batched_plan(src, dst_overlap, 2, ctypes.byref(p), 0x300000, ws, None,
                                      ctypes.byref(plan)) == _lib.WENO_EOVERLAP
    assert L.weno_zoom2x_batched_run(None, None) == _lib.WENO_EINVAL


def test_cascade_errors():
    L = _lib.lib()
    src = _t()
    dst = _t(ptr=0x100000, h=32, w=40)
    p = _p()
    need = L.weno_zoom2x_cascade_workspace(ctypes.byref(src), 3)
    assert need > 0
    assert L.weno_zoom2x_cascade(ctypes.byref(src), ctypes.byref(dst), 0, ctypes.byref(p), 0x400000, need, None) == _lib.WENO_EINVAL
    assert L.weno_zoom2x_cascade(ctypes.byref(src), ctypes.byref(dst), 2, ctypes.byref(p), 0x400000, need, None) == _lib.WENO_EINVAL
    assert L.weno_zoom2x_cascade(ctypes.byref(src), ctypes.byref(dst), 3, ctypes.byref(p), 0x400000, need - 1, None) == _lib.WENO_ENOSPC


def test_backward_errors():
    L = _lib.lib()
    x = _t()
    gy = _t(ptr=0x100000, h=8, w=10)
    gx = _t(ptr=0x200000)
    p = _p()
    assert L.weno_zoom2x_backward(None, ctypes.byref(gy), ctypes.byref(gx), ctypes.byref(p), None) == _lib.WENO_EINVAL
    assert L.weno_zoom2x_backward(ctypes.byref(_t(dtype=_lib.WENO_U8)), ctypes.byref(gy), ctypes.byref(gx),
                                  ctypes.byref(p), None) == _lib.WENO_EDTYPE
    assert L.weno_zoom2x_backward(ctypes.byref(x), ctypes.byref(_t(ptr=0x100000, h=8, w=11)), ctypes.byref(gx),
                                  ctypes.byref(p), None) == _lib.WENO_EINVAL


def test_launch_config_validation():
    L = _lib.lib()
    r, c = ctypes.c_int32(), ctypes.c_int32()
    L.weno_get_launch_config(ctypes.byref(r), ctypes.byref(c))
    assert L.weno_set_launch_config(3, 2) == _lib.WENO_EINVAL
    assert L.weno_set_launch_config(64, 3) == _lib.WENO_EINVAL
    assert L.weno_set_launch_config(8192, 1) == _lib.WENO_EINVAL
    assert L.weno_set_launch_config(0, 0) == _lib.WENO_OK
    assert L.weno_set_launch_config(r.value, c.value) == _lib.WENO_OK
    # the adjoint's strip height is separate: 0 (automatic) or 4..4096
    b = ctypes.c_int32(-1)
    L.weno_get_backward_launch_config(ctypes.byref(b))
    assert b.value == 0
    for bad in (3, -1, 4097):
        assert L.weno_set_backward_launch_config(bad) == _lib.WENO_EINVAL
    assert L.weno_set_backward_launch_config(96) == _lib.WENO_OK
    L.weno_get_backward_launch_config(ctypes.byref(b))
    assert b.value == 96
    r2, c2 = ctypes.c_int32(), ctypes.c_int32()
    L.weno_get_launch_config(ctypes.byref(r2), ctypes.byref(c2))
    assert (r2.value, c2.value) == (r.value, c.value)               # the forward setting is unaffected
    assert L.weno_set_backward_launch_config(0) == _lib.WENO_OK


def _query(src, dst):
    r, c, t = ctypes.c_int32(-1), ctypes.c_int32(-1), ctypes.c_int32(-1)
    rc = _lib.lib().weno_query_launch_config(ctypes.byref(src) if src is not None else None,
                                             ctypes.byref(dst) if dst is not None else None,
                                             ctypes.byref(r), ctypes.byref(c), ctypes.byref(t))
    return rc, (r.value, c.value, t.value)


def test_query_launch_config():
    L = _lib.lib()
    assert _query(None, None)[0] == _lib.WENO_EINVAL
    assert _query(_t(ptr=0), None)[0] == _lib.WENO_EINVAL
    assert _query(_t(), _t(ptr=0x100000, h=8, w=9))[0] == _lib.WENO_EINVAL          # not 2x
    assert L.weno_query_launch_config(ctypes.byref(_t()), None, None, None, None) == _lib.WENO_OK
    # the caller's configuration, never with tail strips
    assert L.weno_set_launch_config(64, 2) == _lib.WENO_OK
    try:
        assert _query(_t(n=16, c=3, h=512, w=512), None) == (_lib.WENO_OK, (64, 2, 0))
    finally:
        assert L.weno_set_launch_config(0, 0) == _lib.WENO_OK
    # the automatic choice (a 256-CU device, also where no device is visible)
    rc, (r, c, t) = _query(_t(c=3, h=1080, w=1920), None)
    assert rc == _lib.WENO_OK and (r, c, t) == (27, 2, 0)
    # 512 wide: four two-column strips and 40 columns, walked as a tail column
    rc, (r, c, t) = _query(_t(n=16, c=3, h=512, w=512), None)
    assert rc == _lib.WENO_OK and c == 2 and t > r
    # interleaved (HWC) planes never take tail strips
    hwc = WenoTensor(0x1000, _lib.WENO_U8, 16, 3, 512, 512, 3 * 512 * 512, 1, 3 * 512, 3)
    hwc_out = WenoTensor(0x10000000, _lib.WENO_U8, 16, 3, 1024, 1024, 3 * 1024 * 1024, 1, 3 * 1024, 3)
    rc, (r, c, t) = _query(hwc, hwc_out)
    assert rc == _lib.WENO_OK and t == 0


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(_lib.status_string(s), str)
    assert _lib.lib().weno_version().decode().count(".") == 2


def _pb(boundary):
    p = _p()
    p.boundary = boundary
    return p


def test_boundary_mode_validation():
    L = _lib.lib()
    src, dst = _t(ptr=0x100000), _t(ptr=0x200000, h=8, w=10)
    assert call_zoom(src, dst, _pb(2)) == _lib.WENO_EINVAL
    assert call_zoom(src, dst, _pb(-1)) == _lib.WENO_EINVAL
    ext = _pb(_lib.WENO_BOUNDARY_EXTERNAL)
    # the ghost region starts 4 rows and 4 columns before element 0: it must
    # not wrap below address 0 ...
    assert call_zoom(_t(ptr=16), dst, ext) == _lib.WENO_EINVAL
    # ... nor overlap the output where the 4 x 5 plane itself does not: the
    # region (rows and columns -4 .. 8 of 5-float rows) spans floats -24 .. 48
    # of the plane, which itself spans floats 0 .. 19
    assert call_zoom(_t(ptr=0x100000), _t(ptr=0x100000 + 4 * 40, h=8, w=10), ext) == _lib.WENO_EOVERLAP
    assert call_zoom(_t(ptr=0x100000), _t(ptr=0x100000 - 4 * 84, h=8, w=10), ext) == _lib.WENO_EOVERLAP
    # entry points without ghost samples reject the mode before anything else
    c = ctypes.byref
    s3, d3 = _t(ptr=0x100000, h=4, w=5), _t(ptr=0x800000, h=32, w=40)
    assert L.weno_zoom2x_cascade(c(s3), c(d3), 3, c(ext), 0x400000, 1 << 20, None) == _lib.WENO_EINVAL
    r = _t(ptr=0x800000, h=7, w=9)
    assert L.weno_resample(c(src), c(r), c(ext), 0x400000, 1 << 20, None) == _lib.WENO_EINVAL
    assert L.weno_zoom_to(c(src), c(r), c(ext), 0x400000, 1 << 20, None) == _lib.WENO_EINVAL
    g, gx = _t(ptr=0x200000, h=8, w=10), _t(ptr=0x300000)
    assert L.weno_zoom2x_backward(c(src), c(g), c(gx), c(ext), None) == _lib.WENO_EINVAL


def test_workspace_alignment():
    # position tables and float planes in the workspace need 256-byte alignment
    L = _lib.lib()
    c = ctypes.byref
    src, p = _t(ptr=0x100000), _p()
    r = _t(ptr=0x800000, h=7, w=9)
    assert L.weno_resample(c(src), c(r), c(p), 0x400000 + 16, 1 << 20, None) == _lib.WENO_EINVAL
    assert L.weno_zoom_to(c(src), c(r), c(p), 0x400000 + 16, 1 << 20, None) == _lib.WENO_EINVAL
    d3 = _t(ptr=0x800000, h=32, w=40)
    assert L.weno_zoom2x_cascade(c(src), c(d3), 3, c(p), 0x400000 + 16, 1 << 20, None) == _lib.WENO_EINVAL


def test_descriptor_dims_match_unsqueezed_views():
    """The per-call descriptor reads sizes and strides from the tuples; they
    must equal those of the (N, C, H, W) view torch's unsqueeze builds, for
    planar, channels-interleaved, sliced, transposed and empty tensors."""
    import torch

    from paper_2312_00229_amd import _as4d, _dims4

    base = torch.zeros(2, 3, 10, 12)
    cases = [torch.zeros(5, 7), torch.zeros(5, 7)[:, ::2], torch.zeros(7, 5).t(), torch.zeros(0, 7),
             torch.zeros(3, 5, 7), torch.zeros(5, 7, 3).permute(2, 0, 1), torch.zeros(0, 5, 7),
             torch.zeros(3, 5, 7)[1:, 2:, ::3], base, base.permute(0, 2, 3, 1).contiguous().permute(0, 3, 1, 2),
             base[:, :, 1:9, 2:], torch.zeros(1, 1, 1, 1), torch.zeros(4, 9, 9, 3).permute(0, 3, 1, 2)[::2]]
    for t in cases:
        v = _as4d(t)
        assert _dims4(t.shape, t.stride()) == (*v.shape, *v.stride()), (t.shape, t.stride())
    with pytest.raises(ValueError):
        _dims4((2, 2, 2, 2, 2), (16, 8, 4, 2, 1))


def test_parameter_structs_are_cached_and_checked():
    from paper_2312_00229_amd import Params, _params

    a, b = Params(beta=1.5, nbw=0.25).c(), Params(beta=1.5, nbw=0.25).c()
    assert a is b
    assert (a.beta, a.k_eps, a.h, a.nbw, a.boundary) == (1.5, pytest.approx(1e-8), 1.0, 0.25, 0)
    assert Params(boundary="external").c().boundary == _lib.WENO_BOUNDARY_EXTERNAL
    d = _params(None, 2.0, 1e-8, 1.0, -1.0)
    assert (d.beta, d.h, d.nbw, d.boundary) == (2.0, 1.0, -1.0, 0)
    with pytest.raises(ValueError):
        Params(boundary="wrap").c()
    with pytest.raises(ValueError):
        _params(None, 2.0, 1e-8, 1.0, -1.0, "wrap")


def test_outputs_keep_the_input_layout():
    """Outputs allocated by the binding are planar-contiguous for planar
    inputs and channels-interleaved-contiguous (HWC / NHWC memory) for
    inputs whose channel dim has unit stride."""
    import torch

    from paper_2312_00229_amd import _empty_like_layout, _sized_like_layout

    planar = [torch.zeros(5, 7), torch.zeros(3, 5, 7), torch.zeros(2, 3, 5, 7), torch.zeros(5, 7, 1).permute(2, 0, 1)]
    interleaved = [torch.zeros(5, 7, 3).permute(2, 0, 1), torch.zeros(2, 5, 7, 3).permute(0, 3, 1, 2),
                   torch.zeros(0, 5, 7, 4).permute(0, 3, 1, 2), torch.zeros(3, 2, 5, 7, 3).permute(0, 1, 4, 2, 3)]
    for x in planar + interleaved:
        for out in (_empty_like_layout(x, 2, torch.uint8), _sized_like_layout(x, 3, 1, torch.float32)):
            assert out.shape[:-2] == x.shape[:-2]
            if any(x is p for p in planar):
                assert out.is_contiguous()
            else:
                assert out.movedim(-3, -1).is_contiguous()
        assert _empty_like_layout(x, 2, torch.uint8).shape[-2:] == (2 * x.shape[-2], 2 * x.shape[-1])
