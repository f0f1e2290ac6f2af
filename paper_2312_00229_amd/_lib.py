"""ctypes view of the C ABI in include/weno_zoom.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# WENO_ZOOM_LIB: another build of the same library (e.g. a sanitizer build of
# the host code for the ABI checks)
LIB_PATH = os.environ.get("WENO_ZOOM_LIB") or os.path.join(_PKG, "libweno_zoom.so")

WENO_OK = 0
WENO_EINVAL = -1
WENO_EDTYPE = -2
WENO_EOVERLAP = -3
WENO_ENOSPC = -4
WENO_EHIP = -5
WENO_U8 = 0
WENO_F32 = 1
WENO_BOUNDARY_CLAMP = 0
WENO_BOUNDARY_EXTERNAL = 1
WENO_NOALLOC_MAX_IMAGES = 4096


class WenoTensor(ctypes.Structure):
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("c", ctypes.c_int32),
        ("h", ctypes.c_int32),
        ("w", ctypes.c_int32),
        ("sn", ctypes.c_int64),
        ("sc", ctypes.c_int64),
        ("sh", ctypes.c_int64),
        ("sw", ctypes.c_int64),
    ]


class WenoParams(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_float),
        ("k_eps", ctypes.c_float),
        ("h", ctypes.c_float),
        ("nbw", ctypes.c_float),
        ("boundary", ctypes.c_int32),
    ]


class WenoBatchPlan(ctypes.Structure):
    _fields_ = [
        ("d_workspace", ctypes.c_void_p),
        ("ws_bytes", ctypes.c_size_t),
        ("total_items", ctypes.c_int64),
        ("count", ctypes.c_int32),
        ("rows_per_strip", ctypes.c_int32),
        ("cols_per_lane", ctypes.c_int32),
        ("beta_mode", ctypes.c_int32),
        ("reserved", ctypes.c_int64),
    ]


# every symbol include/weno_zoom.h declares, with its ctypes signature
_T = ctypes.POINTER(WenoTensor)
_P = ctypes.POINTER(WenoParams)
_V = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "weno_default_params": (WenoParams, []),
    "weno_zoom2x": (_I, [_T, _T, _P, _V]),
    "weno_zoom2x_batched_workspace": (ctypes.c_size_t, [ctypes.c_int32]),
    "weno_zoom2x_batched_plan": (_I, [_T, _T, ctypes.c_int32, _P, _V, ctypes.c_size_t, _V,
                                      ctypes.POINTER(WenoBatchPlan)]),
    "weno_zoom2x_batched_run": (_I, [ctypes.POINTER(WenoBatchPlan), _V]),
    "weno_zoom2x_batched": (_I, [_T, _T, ctypes.c_int32, _P, _V, ctypes.c_size_t, _V]),
    "weno_zoom2x_batched_noalloc": (_I, [_T, _T, ctypes.c_int32, _P, _V]),
    "weno_zoom2x_cascade_workspace": (ctypes.c_size_t, [_T, ctypes.c_int32]),
    "weno_zoom2x_cascade": (_I, [_T, _T, ctypes.c_int32, _P, _V, ctypes.c_size_t, _V]),
    "weno_zoom2x_backward": (_I, [_T, _T, _T, _P, _V]),
    "weno_resample_workspace": (ctypes.c_size_t, [_T, _T]),
    "weno_resample": (_I, [_T, _T, _P, _V, ctypes.c_size_t, _V]),
    "weno_zoom_to_workspace": (ctypes.c_size_t, [_T, _T]),
    "weno_zoom_to": (_I, [_T, _T, _P, _V, ctypes.c_size_t, _V]),
    "weno_set_launch_config": (_I, [ctypes.c_int32, ctypes.c_int32]),
    "weno_get_launch_config": (None, [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "weno_query_launch_config": (_I, [_T, _T, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "weno_set_backward_launch_config": (_I, [ctypes.c_int32]),
    "weno_get_backward_launch_config": (None, [ctypes.POINTER(ctypes.c_int32)]),
    "weno_status_string": (ctypes.c_char_p, [_I]),
    "weno_version": (ctypes.c_char_p, []),
}

_lib = None


class WenoError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (what, status_string(status), status))


def lib():
    """Load the in-tree HIP library; fail loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "HIP library %s is missing: build it with `python -m paper_2312_00229_amd.build` "
                "(or __graft_entry__.build())" % LIB_PATH
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().weno_status_string(int(status)).decode()


def check(status: int, what: str):
    if status != WENO_OK:
        raise WenoError(status, what)
