"""ctypes front end of the FP64 C oracle for the 2DSW step (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg
may import this module. The arithmetic lives in ``sw2d_oracle.c``; this file
converts arrays to contiguous float64 and calls it.
"""

from __future__ import annotations

import contextlib
import ctypes
import os
import threading

import numpy as np

from . import build as _build

_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _bind(path):
    lib = ctypes.CDLL(path)
    lib.sw2d_oracle_step.restype = ctypes.c_int
    lib.sw2d_oracle_step.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 5 + [
        _dp, _u8p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
        ctypes.c_double, _dp]
    lib.sw2d_oracle_run.restype = ctypes.c_int
    lib.sw2d_oracle_run.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 5 + [
        _dp, _u8p, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
        ctypes.c_double, _dp]
    lib.sw2d_oracle_reduce.restype = None
    lib.sw2d_oracle_reduce.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, _dp, _u8p, _dp, _dp, _dp, _dp, _dp]
    lib.sw2d_oracle_max_threads.restype = ctypes.c_int
    lib.sw2d_oracle_max_threads.argtypes = []
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            _build.build(force=False)
            _lib = _bind(_build.lib_path("libsw2d_oracle.so"))
    return _lib


@contextlib.contextmanager
def library(path):
    """Temporarily run every oracle call through another build of the same source
    (the mutation tests plant a mistake in a copy and check that a pin catches it)."""
    global _lib
    _load()
    with _lock:
        saved, _lib = _lib, _bind(path)
    try:
        yield
    finally:
        with _lock:
            _lib = saved


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


class DryCellError(RuntimeError):
    """A water cell reached non-positive total depth without the wetting/drying variant."""


FRICTION = 1   # quadratic bottom friction on the predictor (coefficient cd)
FILTER_UV = 2  # the Shapiro filter on the predicted velocities as well
ADVECTION = 4  # first-order upwind momentum advection in the predictor
WETDRY = 8     # wetting and drying with a total-depth threshold hmin


def run(nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v, nsteps, nthreads=1, reductions=True, flags=0, cd=0.0,
        hmin=0.0, wd_margins=None):
    """Advance ``nsteps`` steps in FP64. Returns (eta, u, v, red) with red[s] = (V_tot, V_disp,
    max|u|, max|v|) after step s, or None when ``reductions`` is False. ``flags`` selects the
    model variants (FRICTION with coefficient ``cd``, FILTER_UV, ADVECTION, WETDRY with
    threshold ``hmin``). ``wd_margins``, a float64 array of 2, receives the smallest distance
    of any wet/dry decision from its threshold over the run: |H + eta - hmin| over water
    cells, and |eta_a - eta_b| over faces between a wet and a dry cell (inf if none)."""
    lib = _load()
    H, mask = _f64(H), _u8(mask)
    eta, u, v = _f64(eta).copy(), _f64(u).copy(), _f64(v).copy()
    assert H.shape == mask.shape == eta.shape == u.shape == v.shape == (ny, nx)
    red = np.zeros((max(nsteps, 1), 4)) if reductions else None
    if wd_margins is not None:
        assert wd_margins.dtype == np.float64 and wd_margins.shape == (2,) and wd_margins.flags.c_contiguous
        wd_margins[:] = np.inf
    rc = lib.sw2d_oracle_run(nx, ny, dx, dy, g, dt, eps, _p(H), _p(mask, _u8p), _p(eta), _p(u),
                             _p(v), int(nsteps), _p(red) if red is not None else None, int(nthreads),
                             int(flags), float(cd), float(hmin),
                             _p(wd_margins) if wd_margins is not None else None)
    if rc == 1:
        raise DryCellError("a water cell dried out")
    if rc != 0:
        raise MemoryError("oracle run could not allocate its buffers")
    return eta, u, v, (red[:nsteps] if red is not None else None)


def run_case(case, nsteps=None, nthreads=1, reductions=True, flags=0, cd=0.0, hmin=0.0, wd_margins=None):
    """``run`` on a ``Case``-like object with fields nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v."""
    n = case.steps if nsteps is None else nsteps
    return run(case.nx, case.ny, case.dx, case.dy, case.g, case.dt, case.eps, case.H, case.mask,
               case.eta, case.u, case.v, n, nthreads=nthreads, reductions=reductions, flags=flags, cd=cd,
               hmin=hmin, wd_margins=wd_margins)


def reduce(nx, ny, dx, dy, H, mask, eta, u, v):
    """(V_tot, V_disp, max|u|, max|v|) of one state."""
    lib = _load()
    H, mask, eta, u, v = _f64(H), _u8(mask), _f64(eta), _f64(u), _f64(v)
    out = np.zeros(4)
    rowbuf = np.zeros(2 * ny)
    lib.sw2d_oracle_reduce(nx, ny, dx, dy, _p(H), _p(mask, _u8p), _p(eta), _p(u), _p(v), _p(out),
                           _p(rowbuf))
    return out


def max_threads() -> int:
    return int(_load().sw2d_oracle_max_threads())
