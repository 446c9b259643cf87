"""The FP64 C oracle against exact rational arithmetic and hand-derived steps.

Pins: brute force on tiny grids (every land pattern of a 3x3 interior), a ragged
4x5 interior, and the hand-derived two-cell steps in ``golden/two_cell.json``.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import exact, sw2d_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_case(rng, nx, ny, mask_interior):
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[1:-1, 1:-1] = mask_interior
    H = rng.uniform(2.0, 12.0, size=(ny, nx)).astype(np.float32)
    eta = (rng.uniform(-0.5, 0.5, size=(ny, nx)) * mask).astype(np.float32)
    u = rng.uniform(-0.3, 0.3, size=(ny, nx)).astype(np.float32)
    v = rng.uniform(-0.3, 0.3, size=(ny, nx)).astype(np.float32)
    return H, mask, eta, u, v


def _close(c_arr, q_arr, rel=5e-14):
    # a few ulps of the largest value per operation over <= 5 steps; a slip is O(1)
    q = np.array([[float(x) for x in row] for row in q_arr])
    scale = max(np.abs(q).max(), 1e-300)
    return np.abs(np.asarray(c_arr) - q).max() <= rel * scale, np.abs(np.asarray(c_arr) - q).max() / scale


def _compare(rng, nx, ny, mask_interior, steps, dx=300.0, dy=200.0, g=9.81, eps=0.05):
    H, mask, eta, u, v = _tiny_case(rng, nx, ny, mask_interior)
    dt = 0.3 * min(dx, dy) / np.sqrt(g * 12.5)
    ce, cu, cv, _ = sw2d_ref.run(nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v, steps)
    qe, qu, qv = exact.run(nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v, steps)
    for name, c, q in (("eta", ce, qe), ("u", cu, qu), ("v", cv, qv)):
        ok, err = _close(c, q)
        assert ok, f"{name}: relative max error {err:.3e}"


def test_every_mask_of_a_3x3_interior(rng):
    """All 512 land patterns of a 3x3 interior, random depth and state, 3 steps."""
    for bits in itertools.product((0, 1), repeat=9):
        m = np.array(bits, dtype=np.uint8).reshape(3, 3)
        _compare(rng, 5, 5, m, steps=3)


def test_random_masks_5_steps(rng):
    for _ in range(20):
        m = (rng.uniform(size=(3, 3)) < 0.75).astype(np.uint8)
        _compare(rng, 5, 5, m, steps=5)


def test_ragged_4x5_interior(rng):
    for _ in range(5):
        m = (rng.uniform(size=(5, 4)) < 0.8).astype(np.uint8)
        _compare(rng, 6, 7, m, steps=5)


def test_open_4x5_interior_isotropic(rng):
    _compare(rng, 6, 7, np.ones((5, 4), dtype=np.uint8), steps=5, dx=250.0, dy=250.0, eps=1.0)


def _golden_arrays(c):
    nx, ny = c["nx"], c["ny"]
    mask = np.zeros((ny, nx), dtype=np.uint8)
    H = np.full((ny, nx), c["H_land"])
    eta, u, v = (np.zeros((ny, nx)) for _ in range(3))
    for j, i in c["wet"]:
        mask[j, i] = 1
    for field, arr in (("H", H), ("eta", eta), ("u", u), ("v", v)):
        for key, val in c[field].items():
            j, i = map(int, key.split(","))
            arr[j, i] = val
    return nx, ny, mask, H, eta, u, v


def _expect(c, key):
    nx, ny = c["nx"], c["ny"]
    out = np.zeros((ny, nx))
    for k, val in c[key].items():
        j, i = map(int, k.split(","))
        out[j, i] = val
    return out


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "two_cell.json")))["cases"],
                         ids=lambda c: c["name"])
def test_hand_derived_two_cell_steps(case):
    nx, ny, mask, H, eta, u, v = _golden_arrays(case)
    e1, u1, v1, red = sw2d_ref.run(nx, ny, case["dx"], case["dy"], case["g"], case["dt"],
                                   case["eps"], H, mask, eta, u, v, 1)
    np.testing.assert_allclose(e1, _expect(case, "expect_eta"), rtol=0, atol=1e-14)
    np.testing.assert_allclose(u1, _expect(case, "expect_u"), rtol=0, atol=1e-14)
    np.testing.assert_allclose(v1, _expect(case, "expect_v"), rtol=0, atol=1e-14)
    np.testing.assert_allclose(red[0], case["expect_red"], rtol=1e-14, atol=1e-14)
    # the exact form agrees with the same hand derivation
    qe, qu, qv = exact.step(nx, ny, case["dx"], case["dy"], case["g"], case["dt"], case["eps"],
                            H, mask, eta, u, v)
    np.testing.assert_allclose(np.array(qe, dtype=float), _expect(case, "expect_eta"), atol=1e-15)
