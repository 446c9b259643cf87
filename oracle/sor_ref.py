"""ctypes front end of the FP64 red-black SOR oracle (test infrastructure only).

Only the test suite and the benchmark's CPU-baseline leg may import this module. The
arithmetic lives in ``sor_oracle.c``; this file converts arrays to contiguous float64 and
calls it.
"""

from __future__ import annotations

import contextlib
import ctypes
import threading

import numpy as np

from . import build as _build

_lock = threading.Lock()
_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _bind(path):
    lib = ctypes.CDLL(path)
    lib.sor_oracle_run.restype = ctypes.c_int
    lib.sor_oracle_run.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 4 + [ctypes.c_int, _dp, _dp, _dp]
    lib.sor_oracle_residual.restype = ctypes.c_int
    lib.sor_oracle_residual.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [_dp, _dp, _dp]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            _build.build(force=False)
            _lib = _bind(_build.lib_path("libsor_oracle.so"))
    return _lib


@contextlib.contextmanager
def library(path):
    """Temporarily run every call through another build of the same source (mutation tests)."""
    global _lib
    _load()
    with _lock:
        saved, _lib = _lib, _bind(path)
    try:
        yield
    finally:
        with _lock:
            _lib = saved


def _ptr(a):
    return a.ctypes.data_as(_dp)


def run(p, f, iters, dx=1.0, dy=1.0, dz=1.0, omega=1.0):
    """iters red-black SOR iterations from p (arrays [nz][ny][nx]); returns (p, res) with
    res[n] = (sum r^2, max |r|) after iteration n + 1."""
    lib = _load()
    p = np.array(p, dtype=np.float64, order="C", copy=True)
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert p.shape == f.shape and p.ndim == 3
    nz, ny, nx = p.shape
    res = np.zeros((max(iters, 1), 2), dtype=np.float64)
    rc = lib.sor_oracle_run(nx, ny, nz, dx, dy, dz, omega, iters, _ptr(p), _ptr(f), _ptr(res))
    if rc != 0:
        raise ValueError("sor_oracle_run rejected its arguments")
    return p, res[:iters]


def residual(p, f, dx=1.0, dy=1.0, dz=1.0):
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = p.shape
    out = np.zeros(2, dtype=np.float64)
    if lib.sor_oracle_residual(nx, ny, nz, dx, dy, dz, _ptr(p), _ptr(f), _ptr(out)) != 0:
        raise ValueError("sor_oracle_residual rejected its arguments")
    return float(out[0]), float(out[1])
