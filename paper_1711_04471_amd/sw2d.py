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


FRICTION = 1   # quadratic bottom friction on the predictor (coefficient cd)
FILTER_UV = 2  # the Shapiro filter on the predicted velocities as well
ADVECTION = 4  # first-order upwind momentum advection in the predictor
WETDRY = 8     # wetting and drying with a total-depth threshold hmin (alone)


def params(nx, ny, dx, dy, g, dt, eps, flags=0, cd=0.0, hmin=0.0) -> sw2d_params:
    return sw2d_params(int(nx), int(ny), float(dx), float(dy), float(g), float(dt), float(eps),
                       int(flags), float(cd), float(hmin))


def workspace_bytes(p: sw2d_params) -> int:
    return int(_lib.load().sw2d_workspace_bytes(ctypes.byref(p)))


def ring_capacity() -> int:
    return int(_lib.load().sw2d_ring_capacity())


def _dev_tensor(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    t = torch.as_tensor(np.ascontiguousarray(a))
    return t.to(device=device, dtype=dtype).contiguous()


class Sw2d:
    """One closed-basin 2DSW problem resident on a GPU.

    Arguments mirror ``sw2d_create``: the grid and constants, the depth field ``H``, the
    land ``mask`` (nonzero = water) and the initial ``eta, u, v`` (numpy or torch arrays of
    shape [ny][nx]). Device buffers are torch tensors owned by this object.
    """

    def __init__(self, nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v, device="cuda", flags=0, cd=0.0,
                 hmin=0.0):
        lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Sw2d runs on a GPU device only")
        self.nx, self.ny = int(nx), int(ny)
        self.p = params(nx, ny, dx, dy, g, dt, eps, flags, cd, hmin)
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
    def from_case(cls, case, device="cuda", flags=0, cd=0.0, hmin=0.0):
        return cls(case.nx, case.ny, case.dx, case.dy, case.g, case.dt, case.eps, case.H,
                   case.mask, case.eta, case.u, case.v, device=device, flags=flags, cd=cd, hmin=hmin)

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

    def step_unfused(self, nsteps: int) -> None:
        """The paper-shaped three-kernel split (comparison path)."""
        lib = _lib.load()
        if getattr(self, "_scratch", None) is None:
            nb = lib.sw2d_unfused_scratch_bytes(ctypes.byref(self.p))
            self._scratch = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        check(lib.sw2d_step_unfused(self._handle(), int(nsteps), self._scratch.data_ptr(),
                                    self._scratch.numel()), "sw2d_step_unfused")

    def set_time_blocking(self, steps_per_pass: int, rows: int = 32) -> None:
        check(_lib.load().sw2d_set_time_blocking(self._handle(), int(steps_per_pass), int(rows)),
              "sw2d_set_time_blocking")

    @property
    def time_blocking(self) -> int:
        return int(_lib.load().sw2d_time_blocking(self._handle()))

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


class Sw2dBatch:
    """An ensemble of independent basins advanced together (``sw2d_batch_*``).

    ``cases`` is a sequence of ``Case``-like objects (nx, ny, dx, dy, g, dt, eps, H, mask,
    eta, u, v); ``band_rows`` gives each instance's band height (None = library default).
    """

    def __init__(self, cases, band_rows=None, device="cuda"):
        lib = _lib.load()
        self.device = torch.device(device)
        self.n = len(cases)
        self.shapes = [(int(c.ny), int(c.nx)) for c in cases]
        self.params = (sw2d_params * self.n)(*[params(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps)
                                               for c in cases])
        self.rows = None
        if band_rows is not None:
            self.rows = (ctypes.c_int32 * self.n)(*[int(r) for r in band_rows])
        self.H, self.mask, self.state_buf = [], [], []
        for c in cases:
            n = int(c.nx) * int(c.ny)
            self.H.append(_dev_tensor(c.H, torch.float32, self.device))
            self.mask.append(_dev_tensor(c.mask, torch.uint8, self.device))
            st = torch.empty(6 * n, dtype=torch.float32, device=self.device)
            for f, a in enumerate((c.eta, c.u, c.v)):
                st[f * n:(f + 1) * n].copy_(_dev_tensor(a, torch.float32, self.device).view(-1))
            self.state_buf.append(st)
        wb = lib.sw2d_batch_workspace_bytes(self.n, self.params, self.rows)
        if wb == 0:
            raise _lib.Sw2dError(_lib.SW2D_EINVAL, "sw2d_batch_workspace_bytes")
        self.work = torch.empty(int(wb), dtype=torch.uint8, device=self.device)
        ptrs = lambda ts: (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in ts])
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib.sw2d_batch_create(self.n, self.params, ptrs(self.H), ptrs(self.mask),
                                    ptrs(self.state_buf), self.rows, self.work.data_ptr(), int(wb),
                                    self.stream.cuda_stream, ctypes.byref(h)), "sw2d_batch_create")
        self.h = h

    def _handle(self):
        if self.h is None:
            raise _lib.Sw2dError(_lib.SW2D_ESTATE, "use after close")
        return self.h

    def set_launch(self, steps_per_launch=50, use_graph=True, grid=0):
        check(_lib.load().sw2d_batch_set_launch(self._handle(), int(steps_per_launch),
                                                int(bool(use_graph)), int(grid)),
              "sw2d_batch_set_launch")

    def set_barrier_timeout(self, seconds: float):
        check(_lib.load().sw2d_batch_set_barrier_timeout(self._handle(), float(seconds)),
              "sw2d_batch_set_barrier_timeout")

    def set_time_blocking(self, steps_per_pass: int):
        """K = 1..3 steps per pass; sw2d_batch_step then takes multiples of K."""
        check(_lib.load().sw2d_batch_set_time_blocking(self._handle(), int(steps_per_pass)),
              "sw2d_batch_set_time_blocking")

    @property
    def time_blocking(self) -> int:
        return int(_lib.load().sw2d_batch_time_blocking(self._handle()))

    @property
    def grid(self) -> int:
        return int(_lib.load().sw2d_batch_grid(self._handle()))

    @property
    def steps_done(self) -> int:
        return int(_lib.load().sw2d_batch_steps_done(self._handle()))

    def step(self, nsteps: int) -> None:
        check(_lib.load().sw2d_batch_step(self._handle(), int(nsteps)), "sw2d_batch_step")

    def step_timed(self, nsteps: int) -> float:
        ms = ctypes.c_double()
        check(_lib.load().sw2d_batch_step_timed(self._handle(), int(nsteps), ctypes.byref(ms)),
              "sw2d_batch_step_timed")
        return float(ms.value)

    def reduce(self) -> np.ndarray:
        out = (sw2d_red * self.n)()
        check(_lib.load().sw2d_batch_reduce(self._handle(), out), "sw2d_batch_reduce")
        return np.frombuffer(bytearray(out), dtype=RED_DTYPE).copy()

    def state(self, k: int):
        pe, pu, pv = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        check(_lib.load().sw2d_batch_state(self._handle(), int(k), ctypes.byref(pe),
                                           ctypes.byref(pu), ctypes.byref(pv)), "sw2d_batch_state")
        base = self.state_buf[k].data_ptr()
        ny, nx = self.shapes[k]
        n = nx * ny
        out = []
        for p in (pe, pu, pv):
            off = (p.value - base) // 4
            out.append(self.state_buf[k][off:off + n].view(ny, nx))
        return tuple(out)

    def state_numpy(self, k: int):
        torch.cuda.synchronize(self.device)
        return tuple(t.cpu().numpy().copy() for t in self.state(k))

    def close(self) -> None:
        if self.h is not None:
            self.stream.synchronize()
            _lib.load().sw2d_batch_destroy(self.h)
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


SOR_RES_DTYPE = np.dtype([("iter", np.int32), ("max_abs_r", np.float32), ("sum_r2", np.float64)])


class SorSolver:
    """Red-black SOR for the pressure Poisson equation on a [nz][ny][nx] FP32 grid (the
    boundary layer holds fixed values). Owns the workspace and residual buffer for a given
    iteration count; ``run`` updates ``p`` in place on the current torch stream."""

    def __init__(self, nx, ny, nz, dx, dy, dz, omega, iters, device="cuda", fused=False):
        self.lib = _lib.load()
        self.dev = torch.device(device)
        if self.dev.type == "cuda" and self.dev.index is None:
            self.dev = torch.device("cuda", torch.cuda.current_device())
        self.p = _lib.sw2d_sor_params(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz), float(omega),
                                      int(bool(fused)))
        self.iters = int(iters)
        nb = self.lib.sw2d_sor_workspace_bytes(ctypes.byref(self.p), self.iters)
        if nb == 0:
            raise ValueError("invalid SOR parameters")
        self.work = torch.empty(int(nb), dtype=torch.uint8, device=self.dev)
        self.res = torch.empty((self.iters + 1) * SOR_RES_DTYPE.itemsize, dtype=torch.uint8, device=self.dev)

    @classmethod
    def from_case(cls, case, device="cuda", fused=False):
        return cls(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.omega, case.iters, device=device,
                   fused=fused)

    def run(self, p: torch.Tensor, f: torch.Tensor, residuals=True) -> None:
        for t in (p, f):
            if t.device != self.dev or t.dtype != torch.float32 or not t.is_contiguous() or \
                    t.numel() != self.p.nx * self.p.ny * self.p.nz:
                raise ValueError("p and f must be contiguous float32 [nz][ny][nx] tensors on the solver's device")
        s = torch.cuda.current_stream(self.dev).cuda_stream
        check(self.lib.sw2d_sor_run(ctypes.byref(self.p), p.data_ptr(), f.data_ptr(), self.iters,
                                    self.res.data_ptr() if residuals else None, self.work.data_ptr(),
                                    self.work.numel(), s), "sw2d_sor_run")

    def residuals(self) -> np.ndarray:
        """(iter, max_abs_r, sum_r2) after 0..iters iterations of the last run (synchronises)."""
        return self.res.cpu().numpy().view(SOR_RES_DTYPE)
