"""WD-WENO 2x image zooming on MI355X (gfx950).

Python binding of the HIP library (include/weno_zoom.h).  Every step of the
method runs in the library's kernels; this module only builds tensor
descriptors, allocates outputs with torch and passes torch's current HIP
stream.  Method: Crnkovic, Skific, Bosner, "WENO based adaptive image zooming
algorithm", arXiv 2312.00229, Section 3.

Tensor layouts: a tensor of 2 (H, W), 3 (C, H, W) or 4 (N, C, H, W) dims, of
dtype uint8 or float32, with any strides -- an HWC image is passed as
`img.permute(2, 0, 1)` and gets an HWC-strided result back.
"""
from __future__ import annotations

import ctypes
import functools
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import WenoBatchPlan, WenoError, WenoParams, WenoTensor

__all__ = [
    "Params",
    "zoom2x",
    "zoom2x_",
    "zoom2x_batched",
    "BatchedZoom",
    "zoom2x_cascade",
    "zoom2x_backward",
    "resample",
    "zoom_to",
    "resample_workspace_bytes",
    "zoom_to_workspace_bytes",
    "WenoZoom2x",
    "set_launch_config",
    "get_launch_config",
    "set_backward_launch_config",
    "get_backward_launch_config",
    "WenoError",
]


_BOUNDARY = {"clamp": _lib.WENO_BOUNDARY_CLAMP, "external": _lib.WENO_BOUNDARY_EXTERNAL}


@dataclass(frozen=True)
class Params:
    beta: float = 2.0
    k_eps: float = 1e-8
    h: float = 1.0
    nbw: float = -1.0  # < 0: h^2 / 8
    # "clamp": samples beyond the plane are its edge samples; "external": the
    # input is a view into a larger array whose rows -4 .. H+4 and columns
    # -4 .. W+4 around it are read as they are (zoom2x and batched only)
    boundary: str = "clamp"

    def _build(self) -> WenoParams:
        if self.boundary not in _BOUNDARY:
            raise ValueError("boundary must be 'clamp' or 'external' (got %r)" % (self.boundary,))
        return WenoParams(float(self.beta), float(self.k_eps), float(self.h), float(self.nbw),
                          _BOUNDARY[self.boundary])

    def c(self) -> WenoParams:
        """The C struct; built once per distinct parameter set."""
        try:
            return _c_params(self.beta, self.k_eps, self.h, self.nbw, self.boundary)
        except TypeError:  # unhashable field values
            return self._build()


_DT = {torch.uint8: _lib.WENO_U8, torch.float32: _lib.WENO_F32}


def _as4d(t: torch.Tensor) -> torch.Tensor:
    if t.dim() == 2:
        return t.unsqueeze(0).unsqueeze(0)
    if t.dim() == 3:
        return t.unsqueeze(0)
    if t.dim() == 4:
        return t
    raise ValueError("expected a tensor of 2, 3 or 4 dims (.., H, W), got %d" % t.dim())


def _dims4(shape, stride):
    """(n, c, h, w, sn, sc, sh, sw) of a 2-, 3- or 4-dim tensor viewed as
    (N, C, H, W): missing leading dims get size 1 and the stride torch's
    unsqueeze(0) would give them (size x stride of the dim after), computed
    from the tuples without building views, since this runs on every call."""
    nd = len(shape)
    if nd == 4:
        return (*shape, *stride)
    if nd == 3:
        c, h, w = shape
        sc, sh, sw = stride
        return (1, c, h, w, c * sc, sc, sh, sw)
    if nd == 2:
        h, w = shape
        sh, sw = stride
        return (1, 1, h, w, h * sh, h * sh, sh, sw)
    raise ValueError("expected a tensor of 2, 3 or 4 dims (.., H, W), got %d" % nd)


def _desc(t: torch.Tensor) -> WenoTensor:
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU (got %s)" % t.device)
    dt = _DT.get(t.dtype)
    if dt is None:
        raise ValueError("dtype must be uint8 or float32 (got %s)" % t.dtype)
    n, c, h, w, sn, sc, sh, sw = _dims4(t.shape, t.stride())
    return WenoTensor(t.data_ptr(), dt, n, c, h, w, sn, sc, sh, sw)


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(device) -> int:
    """Handle of torch's current HIP stream on `device` (a cuda device)."""
    if _raw_stream is not None:
        return _raw_stream(device.index)
    return torch.cuda.current_stream(device).cuda_stream


@functools.lru_cache(maxsize=64)
def _c_params(beta, k_eps, h, nbw, boundary) -> WenoParams:
    # read-only once built: the library takes the struct through a const pointer
    return Params(beta=beta, k_eps=k_eps, h=h, nbw=nbw, boundary=boundary)._build()


def _params(params, beta, k_eps, h, nbw, boundary="clamp") -> WenoParams:
    if params is None:
        return _c_params(beta, k_eps, h, nbw, boundary)
    return params.c()


def _empty_like_layout(x: torch.Tensor, scale: int, dtype) -> torch.Tensor:
    """Output of shape (..., scale H, scale W) in x's memory layout (planar or
    channels-interleaved)."""
    return _sized_like_layout(x, x.shape[-2] * scale, x.shape[-1] * scale, dtype)


def zoom2x_(x: torch.Tensor, out: torch.Tensor, params: Params | None = None, *, beta=2.0, k_eps=1e-8,
            h=1.0, nbw=-1.0, boundary="clamp") -> torch.Tensor:
    """One WD-WENO doubling of x into the caller's `out` (..., 2H, 2W)."""
    p = _params(params, beta, k_eps, h, nbw, boundary)
    s, d = _desc(x), _desc(out)
    _lib.check(_lib.lib().weno_zoom2x(ctypes.byref(s), ctypes.byref(d), ctypes.byref(p), _stream(x.device)),
               "weno_zoom2x")
    return out


def zoom2x(x: torch.Tensor, params: Params | None = None, *, out_dtype=None, beta=2.0, k_eps=1e-8, h=1.0,
           nbw=-1.0, boundary="clamp") -> torch.Tensor:
    """One WD-WENO doubling: (..., H, W) -> (..., 2H, 2W) in x's layout.

    uint8 inputs are read on the [0,1] scale (value/255); `out_dtype` (default:
    x's dtype) selects uint8 or float32 output.  boundary="external": x is a
    view into a larger array and its 4 rows/columns before and 5 after are
    the samples beyond the plane (the paper's function tests pass f there)."""
    out = _empty_like_layout(x, 2, out_dtype or x.dtype)
    return zoom2x_(x, out, params, beta=beta, k_eps=k_eps, h=h, nbw=nbw, boundary=boundary)


class BatchedZoom:
    """A planned batched call: the image table lives in a device workspace and
    `run()` only enqueues kernels (capturable into a CUDA/HIP graph)."""

    def __init__(self, xs, outs, params: Params | None = None):
        if len(xs) != len(outs) or not xs:
            raise ValueError("need equally many (>= 1) inputs and outputs")
        self.xs, self.outs = list(xs), list(outs)
        L = _lib.lib()
        count = len(xs)
        self._srcs = (WenoTensor * count)(*[_desc(t) for t in xs])
        self._dsts = (WenoTensor * count)(*[_desc(t) for t in outs])
        ws = L.weno_zoom2x_batched_workspace(count)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=xs[0].device)
        self.plan = WenoBatchPlan()
        p = (params or Params()).c()
        _lib.check(
            L.weno_zoom2x_batched_plan(self._srcs, self._dsts, count, ctypes.byref(p), self.workspace.data_ptr(), ws,
                                       _stream(xs[0].device), ctypes.byref(self.plan)),
            "weno_zoom2x_batched_plan",
        )

    def run(self):
        _lib.check(_lib.lib().weno_zoom2x_batched_run(ctypes.byref(self.plan), _stream(self.xs[0].device)),
                   "weno_zoom2x_batched_run")
        return self.outs


def zoom2x_batched(xs, params: Params | None = None, out_dtype=None):
    """Zoom a list of images of uneven sizes in one persistent launch."""
    outs = [_empty_like_layout(x, 2, out_dtype or x.dtype) for x in xs]
    return BatchedZoom(xs, outs, params).run()


def zoom2x_batched_noalloc(xs, outs=None, params: Params | None = None, out_dtype=None):
    """zoom2x_batched without a workspace: the library keeps the image table in
    its own fixed device array (at most WENO_NOALLOC_MAX_IMAGES images; calls
    that overlap on one GPU race).  `outs` (optional): the caller's outputs."""
    if not xs:
        raise ValueError("need at least one input")
    if outs is None:
        outs = [_empty_like_layout(x, 2, out_dtype or x.dtype) for x in xs]
    if len(outs) != len(xs):
        raise ValueError("need as many outputs as inputs")
    count = len(xs)
    srcs = (WenoTensor * count)(*[_desc(t) for t in xs])
    dsts = (WenoTensor * count)(*[_desc(t) for t in outs])
    p = (params or Params()).c()
    _lib.check(_lib.lib().weno_zoom2x_batched_noalloc(srcs, dsts, count, ctypes.byref(p), _stream(xs[0].device)),
               "weno_zoom2x_batched_noalloc")
    return outs


def zoom2x_cascade(x: torch.Tensor, levels: int, params: Params | None = None, out_dtype=None,
                   workspace: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """`levels` successive doublings (eq. zoomfactor) with FP32 intermediates,
    grid spacing halved per level.  `out` (optional): the caller's output
    tensor, any strides; `workspace` (optional): cascade_workspace_bytes()."""
    p = (params or Params()).c()
    if out is None:
        out = _empty_like_layout(x, 2 ** levels, out_dtype or x.dtype)
    else:
        _check_out(out, x, x.shape[-2] << levels, x.shape[-1] << levels, out_dtype)
    s, d = _desc(x), _desc(out)
    L = _lib.lib()
    ws = L.weno_zoom2x_cascade_workspace(ctypes.byref(s), int(levels))
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=x.device)
    _lib.check(L.weno_zoom2x_cascade(ctypes.byref(s), ctypes.byref(d), int(levels), ctypes.byref(p),
                                     workspace.data_ptr(), workspace.numel(), _stream(x.device)),
               "weno_zoom2x_cascade")
    return out


def cascade_workspace_bytes(x: torch.Tensor, levels: int) -> int:
    s = _desc(x)
    return int(_lib.lib().weno_zoom2x_cascade_workspace(ctypes.byref(s), int(levels)))


def zoom2x_backward(x: torch.Tensor, grad_y: torch.Tensor, params: Params | None = None,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """Adjoint of zoom2x for float32 x: returns dL/dx given dL/dy, written
    into `out` (float32, x's shape, any strides) when given."""
    p = (params or Params()).c()
    if out is None:
        gx = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    else:
        if tuple(out.shape) != tuple(x.shape) or out.dtype != torch.float32:
            raise ValueError("out must be float32 of shape %s (got %s %s)" % (tuple(x.shape), out.dtype,
                                                                               tuple(out.shape)))
        gx = out
    a, g, o = _desc(x), _desc(grad_y), _desc(gx)
    _lib.check(_lib.lib().weno_zoom2x_backward(ctypes.byref(a), ctypes.byref(g), ctypes.byref(o), ctypes.byref(p),
                                               _stream(x.device)), "weno_zoom2x_backward")
    return gx


def _sized_like_layout(x: torch.Tensor, out_h: int, out_w: int, dtype) -> torch.Tensor:
    """Output of shape (..., out_h, out_w) in x's memory layout: planar, or
    channels interleaved (HWC / NHWC viewed as (.., C, H, W)) when x's channel
    dim has unit stride; allocated with its final strides in one call."""
    shape = list(x.shape)
    shape[-2], shape[-1] = int(out_h), int(out_w)
    if len(shape) >= 3 and x.stride(-3) == 1 and shape[-3] > 1:
        c, h, w = shape[-3:]
        strides = [1, w * c, c]
        inner = c * h * w
        for size in reversed(shape[:-3]):
            strides.insert(0, inner)
            inner *= size
        return torch.empty_strided(shape, strides, dtype=dtype, device=x.device)
    return torch.empty(shape, dtype=dtype, device=x.device)


def _ws_call(fn_ws, fn, what, x, out, params, workspace):
    p = (params or Params()).c()
    s, d = _desc(x), _desc(out)
    need = int(fn_ws(ctypes.byref(s), ctypes.byref(d)))
    if need == 0:
        _lib.check(_lib.WENO_EINVAL, what)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    _lib.check(fn(ctypes.byref(s), ctypes.byref(d), ctypes.byref(p), workspace.data_ptr(), workspace.numel(),
                  _stream(x.device)), what)
    return out


def _check_out(out, x, out_h, out_w, out_dtype):
    want = list(x.shape[:-2]) + [int(out_h), int(out_w)]
    if list(out.shape) != want:
        raise ValueError("out has shape %s, expected %s" % (tuple(out.shape), tuple(want)))
    if out_dtype is not None and out.dtype != out_dtype:
        raise ValueError("out has dtype %s, expected %s" % (out.dtype, out_dtype))
    return out


def resample(x: torch.Tensor, out_h: int, out_w: int, params: Params | None = None, out_dtype=None,
             workspace: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Tensor-product WENO resampling of every (H, W) plane to (out_h, out_w)
    (eq. tensor), end points aligned.  `out` (optional): the caller's output
    tensor, any strides; `workspace` (optional): resample_workspace_bytes()."""
    if out is None:
        out = _sized_like_layout(x, out_h, out_w, out_dtype or x.dtype)
    else:
        _check_out(out, x, out_h, out_w, out_dtype)
    L = _lib.lib()
    return _ws_call(L.weno_resample_workspace, L.weno_resample, "weno_resample", x, out, params, workspace)


def _ws_bytes(fn_ws, x, out_h, out_w, out_dtype):
    s = _desc(x)
    d = WenoTensor(1, _DT[out_dtype or x.dtype], *_as4d(x).shape[:2], int(out_h), int(out_w), 0, 0, 0, 0)
    return int(fn_ws(ctypes.byref(s), ctypes.byref(d)))


def resample_workspace_bytes(x: torch.Tensor, out_h: int, out_w: int, out_dtype=None) -> int:
    """Workspace `resample` needs for x -> (out_h, out_w) (0: invalid sizes)."""
    return _ws_bytes(_lib.lib().weno_resample_workspace, x, out_h, out_w, out_dtype)


def zoom_to_workspace_bytes(x: torch.Tensor, out_h: int, out_w: int, out_dtype=None) -> int:
    """Workspace `zoom_to` needs for x -> (out_h, out_w) (0: invalid sizes)."""
    return _ws_bytes(_lib.lib().weno_zoom_to_workspace, x, out_h, out_w, out_dtype)


def zoom_to(x: torch.Tensor, out_h: int, out_w: int, params: Params | None = None, out_dtype=None,
            workspace: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Zoom to any size (Section 3.3): WD-WENO doublings to the first nested
    grid at least as large, then tensor-WENO resampling.  `out` and
    `workspace` (zoom_to_workspace_bytes()) as for resample."""
    if out is None:
        out = _sized_like_layout(x, out_h, out_w, out_dtype or x.dtype)
    else:
        _check_out(out, x, out_h, out_w, out_dtype)
    L = _lib.lib()
    return _ws_call(L.weno_zoom_to_workspace, L.weno_zoom_to, "weno_zoom_to", x, out, params, workspace)


class WenoZoom2x(torch.autograd.Function):
    """Differentiable WD-WENO doubling of float32 (.., H, W) tensors."""

    @staticmethod
    def forward(ctx, x, params: Params | None = None):
        params = params or Params()
        ctx.params = params
        ctx.save_for_backward(x)
        return zoom2x(x, params)

    @staticmethod
    def backward(ctx, grad_y):
        (x,) = ctx.saved_tensors
        return zoom2x_backward(x, grad_y.contiguous(), ctx.params), None


def set_launch_config(rows_per_strip: int, cols_per_lane: int):
    _lib.check(_lib.lib().weno_set_launch_config(int(rows_per_strip), int(cols_per_lane)), "weno_set_launch_config")


def get_launch_config():
    r, c = ctypes.c_int32(), ctypes.c_int32()
    _lib.lib().weno_get_launch_config(ctypes.byref(r), ctypes.byref(c))
    return int(r.value), int(c.value)


def launch_shape(x: torch.Tensor) -> tuple:
    """(rows_per_strip, cols_per_lane, tail_rows) that zoom2x(x) would launch
    with into an output in x's layout (the configuration set by
    set_launch_config, else the automatic one; tail_rows 0: no one-column
    tail strips)."""
    r, c, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    s = _desc(x)
    _lib.check(_lib.lib().weno_query_launch_config(ctypes.byref(s), None, ctypes.byref(r), ctypes.byref(c),
                                                   ctypes.byref(t)), "weno_query_launch_config")
    return int(r.value), int(c.value), int(t.value)


def set_backward_launch_config(rows_per_strip: int):
    """Strip height of the adjoint kernel (0 = automatic)."""
    _lib.check(_lib.lib().weno_set_backward_launch_config(int(rows_per_strip)), "weno_set_backward_launch_config")


def get_backward_launch_config() -> int:
    r = ctypes.c_int32()
    _lib.lib().weno_get_backward_launch_config(ctypes.byref(r))
    return int(r.value)
