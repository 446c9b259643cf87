"""The library driven from a plain C program (tests/c_client/sw2d_client.c): no PyTorch and no
Python in the process, only the C ABI of include/sw2d.h and the HIP runtime for device memory
and a stream. The final state must equal, bit for bit, what the Python binding gets from the
same calls, and the folds must match the FP64 oracle."""
import os
import subprocess

import numpy as np
import pytest

from oracle import sw2d_ref
from paper_1711_04471_amd import inputs
from tests.c_client import build as c_client
from tests.helpers import gpu_run, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _client(tmp_path, case, nsteps, spp, rows):
    if not os.path.exists(c_client.BIN):
        pytest.fail(f"{c_client.BIN} is not built (tests/c_client/build.py)")
    assert not case.u.any() and not case.v.any(), "the client starts from rest"
    case.H.astype(np.float32).tofile(tmp_path / "H.f32")
    case.mask.astype(np.uint8).tofile(tmp_path / "mask.u8")
    case.eta.astype(np.float32).tofile(tmp_path / "eta.f32")
    args = [c_client.BIN, str(tmp_path), str(case.nx), str(case.ny), repr(case.dx), repr(case.dy),
            repr(case.g), repr(case.dt), repr(case.eps), str(nsteps), str(spp), str(rows)]
    print("c client:", " ".join(args[2:]), flush=True)
    r = subprocess.run(args, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, f"client exit {r.returncode}: {r.stderr}"
    shape = (case.ny, case.nx)
    e, u, v = (np.fromfile(tmp_path / f"out_{n}.f32", dtype=np.float32).reshape(shape) for n in ("eta", "u", "v"))
    folds = np.array([[float(x) for x in line.split()] for line in r.stdout.splitlines()]).reshape(-1, 5)
    return e, u, v, folds


@pytest.mark.parametrize("name,spp,rows", [("gaussian_basin_64", 1, 0), ("gaussian_basin_64", 4, 32),
                                           ("ragged_333x212", 1, 16), ("ragged_333x212", 3, 64)])
def test_c_client_matches_binding_and_oracle(tmp_path, name, spp, rows):
    c = inputs.gaussian_basin_64() if name == "gaussian_basin_64" else inputs.small_basin(333, 212, seed=43, steps=90)
    n = c.steps
    e, u, v, folds = _client(tmp_path, c, n, spp, rows)
    be, bu, bv, bred = gpu_run(c, nsteps=n, steps_per_pass=spp, band_rows=rows or None)
    assert np.array_equal(e, be) and np.array_equal(u, bu) and np.array_equal(v, bv)
    k = len(bred)
    assert folds.shape == (k, 5)
    assert np.array_equal(folds[:, 0], bred["step"])
    oe, ou, ov, ored = sw2d_ref.run_case(c, nsteps=n)
    assert max(rel_l2(e, oe), rel_l2(u, ou), rel_l2(v, ov)) <= TOL
    for j in range(4):
        np.testing.assert_allclose(folds[:, 1 + j], ored[-k:, j], rtol=TOL, atol=1e-6 * c.dx * c.dy if j == 1 else 0)


def test_c_client_reports_library_errors(tmp_path):
    """A library error reaches the C caller as its status: an all-land grid is refused at
    create with SW2D_EINVAL, which the client turns into exit status 10 - status."""
    from paper_1711_04471_amd import _lib
    c = inputs.small_basin(61, 47, seed=21, steps=4)
    c.mask[:] = 0
    c.eta[:] = 0
    args = [c_client.BIN, str(tmp_path), str(c.nx), str(c.ny), repr(c.dx), repr(c.dy), repr(c.g),
            repr(c.dt), repr(c.eps), "4", "1", "0"]
    c.H.astype(np.float32).tofile(tmp_path / "H.f32")
    c.mask.tofile(tmp_path / "mask.u8")
    c.eta.astype(np.float32).tofile(tmp_path / "eta.f32")
    r = subprocess.run(args, capture_output=True, text=True, timeout=60)
    assert r.returncode == 10 - _lib.SW2D_EINVAL, r.stderr
    assert "sw2d_create" in r.stderr
