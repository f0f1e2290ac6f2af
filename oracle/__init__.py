"""FP64 CPU oracle for WD-WENO 2x zooming (arXiv 2312.00229, Section 3).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing on the product path may
import this package, and this package imports nothing from the product.

Contents
  weno_oracle.c   plain C, FP64: forward (phases 1 and 2, algorithms 1 and 2)
                  and the hand adjoint, loaded here through ctypes
  brute.py        brute-force mini-oracle: Vandermonde solves and Gauss-Legendre
                  quadrature per candidate, pure-Python loops, tiny inputs only
  torch_ref.py    the same steps as vectorised torch FP64 ops, used as the
                  autograd reference for the adjoint

Readings of open points (see the header of weno_oracle.c): clamp-to-edge
padding, one-fine-step direction vectors, interval-length indicator scale
(`si_mode=0`; `si_mode=1` is the literal sqrt(2)h scale of eq. 2Dsmoothness),
neighbour weight h^2/8 (the proof of Theorem 1; the only printed number that
separates it from the definitions' h^2/4, Table 1 row 2, selects it), 2n x 2m
output.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "weno_oracle.c")
_LIB = os.path.join(_HERE, "libweno_oracle.so")


class _Params(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_double),
        ("keps", ctypes.c_double),
        ("h", ctypes.c_double),
        ("nbw", ctypes.c_double),
        ("si_mode", ctypes.c_int),
    ]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        for name, extra in (
            ("weno_oracle_zoom2x", [dp]),
            ("weno_oracle_weights", [dp]),
            ("weno_oracle_backward", [dp, dp]),
        ):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Params)] + extra
        lib.weno_oracle_backward_planes.restype = ctypes.c_int
        lib.weno_oracle_backward_planes.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                    ctypes.POINTER(_Params), dp, dp]
        _lib = lib
    return _lib


def _params(beta, keps, h, si_mode, nbw):
    return _Params(float(beta), float(keps), float(h), -1.0 if nbw is None else float(nbw), int(si_mode))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _planes(V):
    V = np.asarray(V, dtype=np.float64)
    if V.ndim < 2:
        raise ValueError("expected an array of at least 2 dims (.., H, W)")
    lead = V.shape[:-2]
    return np.ascontiguousarray(V.reshape((-1,) + V.shape[-2:])), lead


def zoom2x(V, beta=2.0, keps=1e-8, h=1.0, si_mode=0, nbw=None) -> np.ndarray:
    """One WD-WENO doubling of every (H, W) plane of V, clamp-to-edge padding.

    Returns float64 of shape (..., 2H, 2W): U[2I, 2J] = V[I, J], U[2I+1, 2J+1]
    is the phase-1 point, U[2I+1, 2J] and U[2I, 2J+1] the phase-2 points."""
    planes, lead = _planes(V)
    lib = _load()
    p = _params(beta, keps, h, si_mode, nbw)
    n, m = planes.shape[-2:]
    out = np.empty((planes.shape[0], 2 * n, 2 * m), dtype=np.float64)
    for c in range(planes.shape[0]):
        src = np.ascontiguousarray(planes[c])
        dst = np.empty((2 * n, 2 * m), dtype=np.float64)
        rc = lib.weno_oracle_zoom2x(_dptr(src), n, m, ctypes.byref(p), _dptr(dst))
        if rc != 0:
            raise ValueError("weno_oracle_zoom2x failed with status %d" % rc)
        out[c] = dst
    return out.reshape(lead + (2 * n, 2 * m))


def weights(V, beta=2.0, keps=1e-8, h=1.0, si_mode=0, nbw=None) -> np.ndarray:
    """omega_k (k = 0..3) at every output point of one plane: (2H, 2W, 4)."""
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
    if V.ndim != 2:
        raise ValueError("weights() takes one (H, W) plane")
    n, m = V.shape
    p = _params(beta, keps, h, si_mode, nbw)
    W = np.empty((2 * n, 2 * m, 4), dtype=np.float64)
    rc = _load().weno_oracle_weights(_dptr(V), n, m, ctypes.byref(p), _dptr(W))
    if rc != 0:
        raise ValueError("weno_oracle_weights failed with status %d" % rc)
    return W


def backward(V, G, beta=2.0, keps=1e-8, h=1.0, si_mode=0, nbw=None) -> np.ndarray:
    """Hand adjoint: dL/dV for dL/dU = G, every plane separately (several
    planes run on separate OpenMP threads)."""
    planes, lead = _planes(V)
    gplanes, glead = _planes(G)
    n, m = planes.shape[-2:]
    if gplanes.shape != (planes.shape[0], 2 * n, 2 * m):
        raise ValueError("G must have shape (..., 2H, 2W) matching V")
    lib = _load()
    p = _params(beta, keps, h, si_mode, nbw)
    out = np.empty(planes.shape, dtype=np.float64)
    if planes.shape[0] > 1:   # one plane per OpenMP thread
        g = np.ascontiguousarray(gplanes)
        rc = lib.weno_oracle_backward_planes(_dptr(planes), planes.shape[0], n, m, ctypes.byref(p), _dptr(g),
                                             _dptr(out))
        if rc != 0:
            raise ValueError("weno_oracle_backward_planes failed with status %d" % rc)
        return out.reshape(lead + (n, m))
    g = np.ascontiguousarray(gplanes[0])
    rc = lib.weno_oracle_backward(_dptr(planes[0]), n, m, ctypes.byref(p), _dptr(g), _dptr(out[0]))
    if rc != 0:
        raise ValueError("weno_oracle_backward failed with status %d" % rc)
    return out.reshape(lead + (n, m))


def quantize_u8_255(X) -> np.ndarray:
    """uint8 code of a value on the 0..255 scale: round half to even, then
    clamp to [0, 255] (the project's reading; the paper does not quantise)."""
    return np.clip(np.rint(np.asarray(X, dtype=np.float64)), 0, 255).astype(np.uint8)


def quantize_u8(U) -> np.ndarray:
    """uint8 code of a [0,1]-scale value: quantize_u8_255(255 u)."""
    return quantize_u8_255(255.0 * np.asarray(U, dtype=np.float64))


def cascade(V, levels, beta=2.0, keps=1e-8, h=1.0):
    """`levels` successive doublings (eq. zoomfactor), FP64 intermediates, the
    grid spacing halved at every level."""
    U = np.asarray(V, dtype=np.float64)
    for lvl in range(levels):
        U = zoom2x(U, beta=beta, keps=keps, h=h / (2 ** lvl))
    return U


def window_zoom2x(V, r0, r1, c0, c1, beta=2.0, keps=1e-8, h=1.0):
    """Output quads [r0, r1) x [c0, c1) of one large plane, computed on a
    window of the input.

    A quad (I, J) depends on inputs I-4..I+5, J-4..J+5; the window keeps 6
    rows/columns beyond that on each side where the image has them and
    otherwise ends at the image border, where the clamp is the image's own.
    Returns the (2(r1-r0), 2(c1-c0)) block of the full result."""
    V = np.asarray(V)
    n, m = V.shape[-2:]
    wr0, wr1 = max(0, r0 - 6), min(n, r1 + 6)
    wc0, wc1 = max(0, c0 - 6), min(m, c1 + 6)
    sub = V[..., wr0:wr1, wc0:wc1]
    U = zoom2x(sub, beta=beta, keps=keps, h=h)
    return U[..., 2 * (r0 - wr0): 2 * (r1 - wr0), 2 * (c0 - wc0): 2 * (c1 - wc0)]
