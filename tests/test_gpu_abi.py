"""Error handling of the C ABI on the GPU: every failure is a status code, never a crash."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1711_04471_amd import _lib, inputs
from paper_1711_04471_amd.sw2d import Sw2d, params

pytestmark = pytest.mark.gpu


def _expect(code, case, **over):
    kw = dict(nx=case.nx, ny=case.ny, dx=case.dx, dy=case.dy, g=case.g, dt=case.dt, eps=case.eps,
              H=case.H, mask=case.mask, eta=case.eta, u=case.u, v=case.v)
    kw.update(over)
    with pytest.raises(_lib.Sw2dError) as ei:
        Sw2d(**kw)
    assert ei.value.code == code


def test_bad_arguments_are_rejected():
    c = inputs.small_basin(64, 48, seed=3)
    E = _lib.SW2D_EINVAL
    _expect(E, c, eps=1.5)
    _expect(E, c, dt=-1.0)
    _expect(E, c, dt=3.0 * c.dt)  # Courant number above 1
    _expect(E, c, nx=2, ny=2, H=c.H[:2, :2], mask=c.mask[:2, :2], eta=c.eta[:2, :2],
            u=c.u[:2, :2], v=c.v[:2, :2])
    m = c.mask.copy()
    m[0, 10] = 1
    _expect(E, c, mask=m)  # wet border
    H = c.H.copy()
    H[10, 10] = -1.0
    m2 = c.mask.copy()
    m2[10, 10] = 1
    _expect(E, c, H=H, mask=m2)  # water cell without depth
    eta = c.eta.copy()
    eta[20, 20] = np.nan
    _expect(E, c, eta=eta)
    u = c.u.copy()
    u[3, 3] = np.inf
    _expect(E, c, u=u)


def test_small_workspace_and_handle_misuse():
    L = _lib.load()
    c = inputs.small_basin(64, 48, seed=3)
    p = params(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps)
    need = L.sw2d_workspace_bytes(ctypes.byref(p))
    dev = torch.device("cuda")
    H = torch.as_tensor(c.H).to(dev)
    mask = torch.as_tensor(c.mask).to(dev)
    state = torch.zeros(6 * c.nx * c.ny, dtype=torch.float32, device=dev)
    state[:c.nx * c.ny] = torch.as_tensor(c.eta).to(dev).view(-1)
    work = torch.empty(need, dtype=torch.uint8, device=dev)
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream().cuda_stream
    assert L.sw2d_create(ctypes.byref(p), H.data_ptr(), mask.data_ptr(), state.data_ptr(),
                         work.data_ptr(), need - 1, stream, ctypes.byref(h)) == _lib.SW2D_ENOSPC
    assert L.sw2d_create(ctypes.byref(p), H.data_ptr(), mask.data_ptr(), state.data_ptr(),
                         work.data_ptr(), need, stream, ctypes.byref(h)) == _lib.SW2D_OK
    out = (_lib.sw2d_red * 4)()
    assert L.sw2d_reduce(h, out, 1) == _lib.SW2D_ESTATE  # no step done yet
    assert L.sw2d_step(h, -1) == _lib.SW2D_ESTATE
    assert L.sw2d_step(h, 3) == _lib.SW2D_OK
    assert L.sw2d_reduce(h, out, 4) == _lib.SW2D_ESTATE
    assert L.sw2d_reduce(h, out, 3) == _lib.SW2D_OK
    assert [out[i].step for i in range(3)] == [1, 2, 3]
    assert L.sw2d_set_band_rows(h, 4) == _lib.SW2D_EINVAL
    assert L.sw2d_set_band_rows(h, 16) == _lib.SW2D_OK and L.sw2d_band_rows(h) == 16
    assert L.sw2d_destroy(h) == _lib.SW2D_OK


def test_blow_up_is_reported():
    """A finite but enormous surface value (3e38 m, accepted by the input checks) overflows the
    first step's fluxes; the fold of that step is non-finite and sw2d_reduce reports
    SW2D_EUNSTABLE. Every kernel runs to its end: overflow is ordinary IEEE arithmetic."""
    c = inputs.small_basin(96, 80, seed=4)
    wet = np.argwhere(c.mask != 0)
    j, i = wet[len(wet) // 2]
    c.eta = c.eta.copy()
    c.eta[j, i] = np.float32(3e38)
    with Sw2d.from_case(c) as sim:
        sim.step(2)
        red = sim.reduce(2, allow_unstable=True)
        assert not np.isfinite(red["vol_disp"]).all()
        with pytest.raises(_lib.Sw2dError) as ei:
            sim.reduce(1)
        assert ei.value.code == _lib.SW2D_EUNSTABLE
