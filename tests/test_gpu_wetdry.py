"""GPU parity of the wetting/drying variant (SW2D_WETDRY) against the FP64 oracle.

A wet/dry decision (H + eta > hmin; which side of a wet/dry face stands higher) is a
floating-point comparison, and the kernel takes it in FP32 on its own state while the
oracle takes it in FP64. Where a decision sits within rounding of its threshold the two
may go different ways, and the trajectories then part by far more than rounding. So each
case asserts, from the oracle run alone and before the GPU runs, that every decision
whose flip would change the step discontinuously lies at least 1e-5 m from its threshold:
the depth test of every water cell the flow has reached, and the surface comparison on
every wet/dry face with a nonzero old velocity (with zero old velocity the flip changes
the predictor by g dt/dx times the surface difference only). Decisions on cells the flow
has not reached are taken on the unchanged inputs, where the FP32 and FP64 depth tests
are checked to agree. The cases are seeded shore basins chosen to meet that bar while
flooding and drying tens to hundreds of cells.

Bar: eta, u, v within 1e-5 relative L2; land and inactive faces exactly 0; folds within
1e-5; the final wet set equal away from the threshold; bitwise independence of the band
height; a lake at rest over emerging ground bitwise still; with every cell deep, bitwise
the plain step; at K steps per pass, bitwise the single steps.
"""
import numpy as np
import pytest

from oracle import sw2d_ref
from paper_1711_04471_amd import inputs
from paper_1711_04471_amd.sw2d import FILTER_UV, WETDRY, Sw2d
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
HMIN = 0.0625
MARGIN = 1e-5

# (shape, seed, steps): shore basins whose decisions keep the margin (see the module text)
CASES = [((130, 97), 48, 120), ((257, 190), 54, 100), ((301, 97), 70, 100), ((64, 300), 20, 80)]


def _say(msg):
    print(msg, flush=True)


def _faces(mask):
    w = mask != 0
    au = np.zeros_like(w)
    au[:, :-1] = w[:, :-1] & w[:, 1:]
    av = np.zeros_like(w)
    av[:-1] = w[:-1] & w[1:]
    return au, av


def _oracle_with_margins(c, n):
    """The oracle one step at a time, with the folds of every step and the smallest distance
    of a consequential wet/dry decision from its threshold."""
    H = c.H.astype(np.float64)
    w = c.mask != 0
    e0 = c.eta.astype(np.float64)
    e, u, v = e0.copy(), c.u.astype(np.float64), c.v.astype(np.float64)
    reached = np.zeros_like(w)
    mh = me = np.inf
    d_prev = w & (H + e > HMIN)
    changes = 0
    red = np.zeros((n, 4))
    a, b = slice(None, -1), slice(1, None)
    for s in range(n):
        moving = (e != e0) | (u != 0) | (v != 0)
        moving[:, 1:] |= u[:, :-1] != 0
        moving[1:, :] |= v[:-1, :] != 0
        reached |= moving
        h = H + e
        d = w & (h > HMIN)
        changes += int((d != d_prev).sum())
        d_prev = d
        if (w & reached).any():
            mh = min(mh, np.abs(h - HMIN)[w & reached].min())
        fx = w[:, a] & w[:, b] & (d[:, a] != d[:, b]) & (u[:, a] != 0)
        if fx.any():
            me = min(me, np.abs(e[:, a] - e[:, b])[fx].min())
        fy = w[a, :] & w[b, :] & (d[a, :] != d[b, :]) & (v[a, :] != 0)
        if fy.any():
            me = min(me, np.abs(e[a, :] - e[b, :])[fy].min())
        e, u, v, _ = sw2d_ref.run(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps, H, c.mask, e, u, v, 1,
                                  reductions=False, flags=sw2d_ref.WETDRY, hmin=HMIN)
        red[s] = sw2d_ref.reduce(c.nx, c.ny, c.dx, c.dy, H, c.mask, e, u, v)
    return (e, u, v), red, mh, me, changes


def _gpu(c, n, flags=WETDRY, band_rows=None):
    with Sw2d.from_case(c, flags=flags, hmin=HMIN) as sim:
        if band_rows is not None:
            sim.band_rows = band_rows
        sim.step(n)
        red = sim.reduce(n) if n else None
        e, u, v = sim.state_numpy()
    return e, u, v, red


@pytest.mark.parametrize("shape,seed,steps", CASES)
def test_wetdry_matches_oracle(shape, seed, steps):
    nx, ny = shape
    c = inputs.shore_basin(nx, ny, seed, steps)
    (oe, ou, ov), ored, mh, me, changes = _oracle_with_margins(c, steps)
    assert changes >= 20 and mh >= MARGIN and me >= MARGIN, (changes, mh, me)
    w = c.mask != 0
    h32 = (c.H + c.eta)[w]
    h64 = (c.H.astype(np.float64) + c.eta.astype(np.float64))[w]
    assert np.array_equal(h32 > np.float32(HMIN), h64 > HMIN)
    _say(f"wetdry {c.name} steps {steps}: {changes} wet/dry changes, margins {mh:.2e} {me:.2e}")
    e, u, v, red = _gpu(c, steps)
    errs = (rel_l2(e, oe), rel_l2(u, ou), rel_l2(v, ov))
    assert max(errs) <= TOL, errs
    au, av = _faces(c.mask)
    assert not e[~w].any() and not u[~au].any() and not v[~av].any()
    for col, k in (("vol_total", 0), ("vol_disp", 1), ("max_abs_u", 2), ("max_abs_v", 3)):
        np.testing.assert_allclose(red[col], ored[:, k], rtol=TOL, atol=1e-6 * c.dx * c.dy, err_msg=col)
    ho = c.H.astype(np.float64) + oe
    hg = c.H.astype(np.float64) + e
    clear = w & (np.abs(ho - HMIN) > MARGIN)
    assert np.array_equal((hg > HMIN)[clear], (ho > HMIN)[clear])


def test_wetdry_is_band_height_independent():
    c = inputs.shore_basin(200, 173, seed=48, steps=60)
    runs = [_gpu(c, 60, band_rows=r) for r in (8, 16, 40)]
    for other in runs[1:]:
        for x, y in zip(runs[0][:3], other[:3]):
            assert np.array_equal(x, y)


def test_wetdry_lake_at_rest_over_emerging_ground():
    c = inputs.shore_basin(150, 90, seed=3, n_bumps=0)
    w = c.mask != 0
    assert (w & (c.H + c.eta <= HMIN)).sum() > 500  # dry ground at rest
    e, u, v, _ = _gpu(c, 40)
    assert np.array_equal(e, c.eta) and not u.any() and not v.any()


def test_wetdry_is_the_plain_step_while_every_cell_is_deep():
    c = inputs.small_basin(140, 111, seed=12, steps=50)
    a = _gpu(c, 50)
    b = _gpu(c, 50, flags=0)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("spp", [2, 3, 4])
def test_wetdry_k_steps_per_pass_equal_single_steps(spp):
    """Wetting and drying at K steps per pass, on a shore basin that floods and dries cells:
    every state bit equals single steps, the folds agree up to summation order."""
    c = inputs.shore_basin(257, 190, seed=54, steps=100)
    ref = _gpu(c, 100)
    for rows in (8, 32):
        _say(f"wetdry K={spp} rows={rows}")
        with Sw2d.from_case(c, flags=WETDRY, hmin=HMIN) as sim:
            sim.set_time_blocking(spp, rows=rows)
            sim.step(100)
            red = sim.reduce(100)
            e, u, v = sim.state_numpy()
        for x, y in zip((e, u, v), ref[:3]):
            assert np.array_equal(x, y), (spp, rows)
        np.testing.assert_allclose(red["vol_disp"], ref[3]["vol_disp"], rtol=1e-12, atol=1e-9 * c.dx * c.dy)
        assert np.array_equal(red["max_abs_u"], ref[3]["max_abs_u"])


def test_wetdry_takes_no_other_flag():
    from paper_1711_04471_amd._lib import Sw2dError
    c = inputs.shore_basin(64, 64, seed=2, steps=5)
    with pytest.raises(Sw2dError):
        Sw2d.from_case(c, flags=WETDRY | FILTER_UV, hmin=HMIN)
