"""Python binding of the 2DSW C ABI. PyTorch supplies device memory and the stream only;
every step of the model runs in the library's HIP kernels."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, sw2d_params, sw2d_red

RED_DTYPE = np.dtype([("step", np.int64), ("vol_total", np.float64), ("vol_disp", np.float64),
                      ("max_abs_u", np.float32), ("max_abs_v", np.float32)])


def params(nx, ny, dx, dy, g, dt, eps, flags=0) -> sw2d_params:
    return sw2d_params(int(nx), int(ny), float(dx), float(dy), float(g), float(dt), float(eps),
                       int(flags))


def workspace_bytes(p: sw2d_params) -> int:
    return int(_lib.load().sw2d_workspace_bytes(ctypes.byref(p)))


def ring_capacity() -> int:
    return int(_lib.load().sw2d_ring_capacity())


def _dev_tensor(a, dtype, device):
    t = torch.as_tensor(np.ascontiguousarray(a))
    return t.to(device=device, dtype=dtype).contiguous()


class Sw2d:
    """One closed-basin 2DSW problem resident on a GPU.

    Arguments mirror ``sw2d_create``: the grid and constants, the depth field ``H``, the
    land ``mask`` (nonzero = water) and the initial ``eta, u, v`` (numpy or torch arrays of
    shape [ny][nx]). Device buffers are torch tensors owned by this object.
    """

    def __init__(self, nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v, device="cuda"):
        lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Sw2d runs on a GPU device only")
        self.nx, self.ny = int(nx), int(ny)
        self.p = params(nx, ny, dx, dy, g, dt, eps)
        n = self.nx * self.ny
        self.H = _dev_tensor(H, torch.float32, self.device)
        self.mask = _dev_tensor(mask, torch.uint8, self.device)
        self.state_buf = torch.empty(6 * n, dtype=torch.float32, device=self.device)
        for f, a in enumerate((eta, u, v)):
            self.state_buf[f * n:(f + 1) * n].copy_(_dev_tensor(a, torch.float32, self.device).view(-1))
        wb = lib.sw2d_workspace_bytes(ctypes.byref(self.p))
        if wb == 0:
            raise _lib.Sw2dError(_lib.SW2D_EINVAL, "sw2d_workspace_bytes")
        self.work = torch.empty(int(wb), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib.sw2d_create(ctypes.byref(self.p), self.H.data_ptr(), self.mask.data_ptr(),
                              self.state_buf.data_ptr(), self.work.data_ptr(), int(wb),
                              self.stream.cuda_stream, ctypes.byref(h)), "sw2d_create")
        self.h = h

    @classmethod
    def from_case(cls, case, device="cuda"):
        return cls(case.nx, case.ny, case.dx, case.dy, case.g, case.dt, case.eps, case.H,
                   case.mask, case.eta, case.u, case.v, device=device)

    def _handle(self):
        if self.h is None:
            raise _lib.Sw2dError(_lib.SW2D_ESTATE, "use after close")
        return self.h

    def step(self, nsteps: int) -> None:
        check(_lib.load().sw2d_step(self._handle(), int(nsteps)), "sw2d_step")

    def step_timed(self, nsteps: int) -> float:
        """Run ``nsteps`` steps; return the mean step-kernel duration in ms (HIP events)."""
        ms = ctypes.c_double()
        check(_lib.load().sw2d_step_timed(self._handle(), int(nsteps), ctypes.byref(ms)),
              "sw2d_step_timed")
        return float(ms.value)

    @property
    def band_rows(self) -> int:
        return int(_lib.load().sw2d_band_rows(self._handle()))

    @band_rows.setter
    def band_rows(self, rows: int) -> None:
        check(_lib.load().sw2d_set_band_rows(self._handle(), int(rows)), "sw2d_set_band_rows")

    def reduce(self, k: int = 1, allow_unstable: bool = False) -> np.ndarray:
        out = (sw2d_red * int(k))()
        rc = _lib.load().sw2d_reduce(self._handle(), out, int(k))
        if not (allow_unstable and rc == _lib.SW2D_EUNSTABLE):
            check(rc, "sw2d_reduce")
        return np.frombuffer(bytearray(out), dtype=RED_DTYPE).copy()

    @property
    def steps_done(self) -> int:
        return int(_lib.load().sw2d_steps_done(self._handle()))

    def state(self):
        """Torch views (eta, u, v) of the current device buffers, each [ny][nx]."""
        pe, pu, pv = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        check(_lib.load().sw2d_state(self._handle(), ctypes.byref(pe), ctypes.byref(pu),
                                     ctypes.byref(pv)), "sw2d_state")
        base = self.state_buf.data_ptr()
        n = self.nx * self.ny
        views = []
        for p in (pe, pu, pv):
            off = (p.value - base) // 4
            views.append(self.state_buf[off:off + n].view(self.ny, self.nx))
        return tuple(views)

    def state_numpy(self):
        torch.cuda.synchronize(self.device)
        return tuple(t.cpu().numpy().copy() for t in self.state())

    def set_state(self, eta, u, v, step: int = 0) -> None:
        ts = [_dev_tensor(a, torch.float32, self.device) for a in (eta, u, v)]
        check(_lib.load().sw2d_set_state(self._handle(), *(t.data_ptr() for t in ts), int(step)),
              "sw2d_set_state")
        self._keep = ts  # alive until the enqueued copies have run
        self.stream.synchronize()

    def close(self) -> None:
        if self.h is not None:
            self.stream.synchronize()
            _lib.load().sw2d_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
