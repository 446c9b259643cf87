"""Loads the in-tree ``libsw2d.so`` and declares its C signatures (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsw2d.so")

SW2D_OK = 0
SW2D_EINVAL = -1
SW2D_EHIP = -2
SW2D_EUNSTABLE = -3
SW2D_ESTATE = -4
SW2D_ENOSPC = -5


class sw2d_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("g", ctypes.c_double), ("dt", ctypes.c_double),
                ("eps", ctypes.c_double), ("flags", ctypes.c_uint32), ("cd", ctypes.c_double),
                ("hmin", ctypes.c_double)]


class sw2d_red(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("vol_total", ctypes.c_double),
                ("vol_disp", ctypes.c_double), ("max_abs_u", ctypes.c_float),
                ("max_abs_v", ctypes.c_float)]


assert ctypes.sizeof(sw2d_red) == 32

class sw2d_sor_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("omega", ctypes.c_double), ("fused", ctypes.c_int32)]


class sw2d_sor_res(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("max_abs_r", ctypes.c_float), ("sum_r2", ctypes.c_double)]


_vp = ctypes.c_void_p
_pp = ctypes.POINTER(ctypes.c_void_p)
_fp = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes); every symbol the public header declares
SIGNATURES = {
    "sw2d_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(sw2d_params)]),
    "sw2d_ring_capacity": (ctypes.c_int32, []),
    "sw2d_create": (ctypes.c_int, [ctypes.POINTER(sw2d_params), _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                   _vp, _pp]),
    "sw2d_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "sw2d_step_timed": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "sw2d_reduce": (ctypes.c_int, [_vp, ctypes.POINTER(sw2d_red), ctypes.c_int32]),
    "sw2d_state": (ctypes.c_int, [_vp, _pp, _pp, _pp]),
    "sw2d_steps_done": (ctypes.c_int64, [_vp]),
    "sw2d_set_state": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int64]),
    "sw2d_set_band_rows": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "sw2d_band_rows": (ctypes.c_int32, [_vp]),
    "sw2d_batch_set_time_blocking": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "sw2d_batch_time_blocking": (ctypes.c_int32, [_vp]),
    "sw2d_sor_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(sw2d_sor_params), ctypes.c_int32]),
    "sw2d_sor_run": (ctypes.c_int, [ctypes.POINTER(sw2d_sor_params), _vp, _vp, ctypes.c_int32, _vp, _vp,
                                    ctypes.c_size_t, _vp]),
    "sw2d_unfused_scratch_bytes": (ctypes.c_size_t, [ctypes.POINTER(sw2d_params)]),
    "sw2d_step_unfused": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_size_t]),
    "sw2d_set_time_blocking": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "sw2d_time_blocking": (ctypes.c_int32, [_vp]),
    "sw2d_destroy": (ctypes.c_int, [_vp]),
    "sw2d_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sw2d_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.POINTER(sw2d_params),
                                                     ctypes.POINTER(ctypes.c_int32)]),
    "sw2d_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(sw2d_params), _pp, _pp, _pp,
                                         ctypes.POINTER(ctypes.c_int32), _vp, ctypes.c_size_t, _vp,
                                         _pp]),
    "sw2d_batch_set_launch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "sw2d_batch_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "sw2d_batch_step_timed": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "sw2d_batch_reduce": (ctypes.c_int, [_vp, ctypes.POINTER(sw2d_red)]),
    "sw2d_batch_state": (ctypes.c_int, [_vp, ctypes.c_int32, _pp, _pp, _pp]),
    "sw2d_batch_steps_done": (ctypes.c_int64, [_vp]),
    "sw2d_batch_set_barrier_timeout": (ctypes.c_int, [_vp, ctypes.c_double]),
    "sw2d_batch_grid": (ctypes.c_int32, [_vp]),
    "sw2d_batch_destroy": (ctypes.c_int, [_vp]),
    # surrogate building blocks
    "sw2d_restrict4": (ctypes.c_int, [_vp] * 5 + [ctypes.c_int32] * 2 + [_vp] * 6),
    "sw2d_pack_input": (ctypes.c_int, [_vp] * 5 + [ctypes.c_int32] * 2 +
                        [_fp, _fp, ctypes.c_float, ctypes.c_uint64, _vp, _vp]),
    "sw2d_conv3x3_fwd_raw": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _fp, _fp,
                                            _vp, _vp, _vp, _vp]),
    "sw2d_cnn_forward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _fp, _fp,
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _vp, _vp]),
    "sw2d_surrogate_advance": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _fp, _fp, ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_void_p), _fp, _vp]),
    "sw2d_surrogate_advance_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _fp, _fp,
                                                      ctypes.POINTER(ctypes.c_void_p),
                                                      ctypes.POINTER(ctypes.c_void_p), _fp]),
    "sw2d_conv3x3_correct": (ctypes.c_int, [_vp, _vp, _vp, _fp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                            ctypes.c_int32, _vp]),
    "sw2d_conv3x3_fwd": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, _vp] +
                         [ctypes.c_int32] * 3 + [_vp]),
    "sw2d_conv3x3_dgrad": (ctypes.c_int, [_vp] * 4 + [ctypes.c_int32] * 3 + [_vp]),
    "sw2d_wgrad_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 4),
    "sw2d_conv3x3_wgrad": (ctypes.c_int, [_vp, ctypes.c_int32, _vp] + [ctypes.c_int32] * 3 +
                           [_vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "sw2d_mse_workspace_bytes": (ctypes.c_size_t, []),
    "sw2d_mse_grad": (ctypes.c_int, [_vp, _vp, _fp, _vp] + [ctypes.c_int32] * 3 +
                      [ctypes.c_float, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "sw2d_sub3": (ctypes.c_int, [_vp] * 6 + [ctypes.c_int32, _vp, _vp]),
    "sw2d_moments_workspace_bytes": (ctypes.c_size_t, []),
    "sw2d_moments": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_size_t, _vp]),
    "sw2d_adam": (ctypes.c_int, [_vp] * 4 + [ctypes.c_int32] * 2 + [ctypes.c_float] * 4 + [_vp]),
    "sw2d_cast_weights": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
    "sw2d_apply_correction": (ctypes.c_int, [_vp] * 5 + [ctypes.c_int32] * 2 + [_fp, _vp]),
    "sw2d_rmse_workspace_bytes": (ctypes.c_size_t, []),
    "sw2d_rmse": (ctypes.c_int, [_vp] * 3 + [ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "sw2d_last_hip_error": (ctypes.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


class Sw2dError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load()
        msg = lib.sw2d_strerror(code).decode()
        if code == SW2D_EHIP:
            msg += ": " + lib.sw2d_last_hip_error().decode()
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def load():
    """The loaded library; raises ``OSError`` when ``libsw2d.so`` has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise OSError(f"{LIB_PATH} is missing: build it with paper_1711_04471_amd/build.py "
                              "(there is no CPU fallback)")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(code: int, where: str) -> int:
    if code != SW2D_OK:
        raise Sw2dError(code, where)
    return code
