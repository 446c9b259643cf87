"""Pins of the oracle's wetting/drying variant.

The rule (a reading: the paper names no wetting scheme): a water cell is wet while
H + eta > hmin; a face between two water cells carries flow when both are wet, or when
one is wet and its surface stands above the other's; the Shapiro filter acts on wet
cells across wet neighbours only, and a dry cell keeps its predicted surface.

* one-step values worked out by hand for each branch of the rule (flooding, a dry cell
  standing higher, a dry cell drained by its old velocity, the filter next to a dry cell);
* with every cell staying wet the variant is the plain step, bit for bit;
* a lake at rest over ground that rises above the water line stays bitwise at rest;
* volume is conserved through flooding and drying, and mirror and transpose symmetry hold;
* a dam break onto a dry bed (with momentum advection) follows Ritter's solution.
"""
import math

import numpy as np
import pytest

from oracle import sw2d_ref

WD, ADV = sw2d_ref.WETDRY, sw2d_ref.ADVECTION


def _row(H, eta, u):
    """One row of water cells between land: arrays [3][n + 2]."""
    n = len(H)
    nx, ny = n + 2, 3
    mask = np.zeros((ny, nx), np.uint8)
    mask[1, 1:-1] = 1
    Hf, ef, uf = (np.zeros((ny, nx)) for _ in range(3))
    Hf[1, 1:-1], ef[1, 1:-1] = H, eta
    uf[1, 1:n] = u  # faces between the row's cells
    return nx, ny, Hf, mask, ef, uf, np.zeros((ny, nx))


def _step_row(H, eta, u, hmin, g=10.0, dt=1.0, dx=10.0, eps=0.2):
    nx, ny, Hf, mask, ef, uf, vf = _row(H, eta, u)
    e1, u1, v1, _ = sw2d_ref.run(nx, ny, dx, dx, g, dt, eps, Hf, mask, ef, uf, vf, 1, flags=WD, hmin=hmin)
    assert not v1.any()
    return e1[1, 1:-1], u1[1, 1:-2]


def test_flooding_step_by_hand():
    """A wet cell next to dry ground with a lower surface: the face opens, the predictor
    takes the full pressure gradient, the flux carries the wet cell's depth. The face
    between the two dry cells stays shut; the wet cell has no wet neighbour to filter with.
    cx = g dt/dx = 1, dt/dx = 0.1."""
    e, u = _step_row(H=[1.0, 0.5, 0.5], eta=[0.0, -0.5, -0.5], u=[0.0, 0.0], hmin=0.01)
    # u* = 0 - 1 (-0.5 - 0) = 0.5; flux 0.5 * h_A = 0.5; eta_A = 0 - 0.1 * 0.5; eta_B = -0.5 + 0.1 * 0.5
    np.testing.assert_allclose(u, [0.5, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(e, [-0.05, -0.45, -0.5], rtol=0, atol=1e-15)


def test_dry_cell_standing_higher_shuts_the_face():
    """The wet cell's surface lies below the dry cell's: no flow, whatever the old velocity
    (the plain step would carry 0.7 - 0.35 = 0.35 m/s and a flux out of the wet cell)."""
    e, u = _step_row(H=[1.0, 0.5], eta=[-0.8, -0.45], u=[0.7], hmin=0.1)
    assert u[0] == 0.0
    np.testing.assert_array_equal(e, [-0.8, -0.45])
    e0, u0 = _plain_row(H=[1.0, 0.5], eta=[-0.8, -0.45], u=[0.7])
    assert abs(u0[0] - 0.35) < 1e-15 and e0[0] != -0.8


def _plain_row(H, eta, u):
    nx, ny, Hf, mask, ef, uf, vf = _row(H, eta, u)
    try:
        e1, u1, _, _ = sw2d_ref.run(nx, ny, 10.0, 10.0, 10.0, 1.0, 0.2, Hf, mask, ef, uf, vf, 1)
    except sw2d_ref.DryCellError:
        pytest.fail("the plain step rejects a dry cell")
    return e1[1, 1:-1], u1[1, 1:-2]


def test_dry_cell_drained_by_its_old_velocity():
    """A dry cell (h = 0.01 <= hmin = 0.02) below a wet neighbour: the face opens because the
    wet side stands higher; the old velocity still points out of the dry cell, so the
    upwind depth is the dry cell's 0.01 m.
    u* = 0.6 - 1 (0 - (-0.49)) = 0.11; flux = 0.11 * 0.01 = 0.0011."""
    e, u = _step_row(H=[0.5, 1.0], eta=[-0.49, 0.0], u=[0.6], hmin=0.02)
    np.testing.assert_allclose(u, [0.11], rtol=1e-14)
    np.testing.assert_allclose(e, [-0.49 - 0.1 * 0.0011, 0.0 + 0.1 * 0.0011], rtol=1e-14, atol=1e-17)


def test_filter_next_to_a_dry_cell():
    """g = 0 and no velocity: no flux anywhere, so the step is the filter alone. Cells
    W1 D W2 W3 with D dry: W1's only water neighbour is dry (unchanged), D keeps its
    surface, W2 and W3 exchange with each other only. e4 = eps / 4 = 0.05."""
    eta = [0.3, -0.9, 0.1, -0.2]
    e, u = _step_row(H=[1.0, 0.95, 1.0, 1.0], eta=eta, u=[0.0, 0.0, 0.0], hmin=0.1, g=0.0)
    assert not u.any()
    want = [0.3, -0.9, 0.1 + 0.05 * (-0.2 - 0.1), -0.2 + 0.05 * (0.1 - (-0.2))]
    np.testing.assert_allclose(e, want, rtol=0, atol=1e-15)


def _terrain(nx, ny, seed, level=-1.0, hmin=0.05, rough=True):
    """Basin whose ground rises through the water line: H is the depth below the datum,
    which sits above the still-water level `level`; the eastern third slopes up to 0.2 m
    below the datum, so a band of cells there is dry ground at rest (eta = -H)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (np.arange(nx) + 0.5) / nx
    H = np.tile(np.clip(6.0 - 9.0 * x, 0.2, None), (ny, 1))
    if rough:
        H += 0.3 * rng.uniform(size=(ny, nx))
    mask = np.zeros((ny, nx), np.uint8)
    mask[1:-1, 1:-1] = 1
    mask[rng.uniform(size=(ny, nx)) < 0.05] = 0
    mask[0], mask[-1], mask[:, 0], mask[:, -1] = 0, 0, 0, 0
    H = H * mask
    eta = np.where(mask != 0, np.maximum(level, -H), 0.0)
    return H, mask, eta


def test_lake_at_rest_over_rising_ground_is_bitwise_still():
    nx, ny = 40, 23
    H, mask, eta = _terrain(nx, ny, 5)
    dry = (mask != 0) & (H + eta <= 0.05)
    assert 20 < dry.sum() < mask.sum() - 100
    z = np.zeros((ny, nx))
    for hmin in (0.0, 0.05):
        e1, u1, v1, _ = sw2d_ref.run(nx, ny, 50.0, 40.0, 9.81, 2.0, 0.1, H, mask, eta, z, z, 60, flags=WD, hmin=hmin)
        assert np.array_equal(e1, eta) and not u1.any() and not v1.any()


def test_equals_the_plain_step_while_every_cell_stays_wet():
    rng = np.random.Generator(np.random.PCG64(9))
    nx, ny = 37, 29
    mask = (rng.uniform(size=(ny, nx)) < 0.85).astype(np.uint8)
    mask[0], mask[-1], mask[:, 0], mask[:, -1] = 0, 0, 0, 0
    H = (4.0 + 6.0 * rng.uniform(size=(ny, nx))) * mask
    eta = 0.5 * rng.standard_normal((ny, nx)) * mask
    u, v = (0.2 * rng.standard_normal((ny, nx)) for _ in range(2))
    au = np.zeros_like(mask, bool)
    au[:, :-1] = (mask[:, :-1] & mask[:, 1:]) != 0
    av = np.zeros_like(mask, bool)
    av[:-1] = (mask[:-1] & mask[1:]) != 0
    u, v = u * au, v * av
    args = (nx, ny, 60.0, 45.0, 9.81, 2.0, 0.1, H, mask, eta, u, v, 40)
    m = np.zeros(2)
    a = sw2d_ref.run(*args, flags=WD, hmin=0.5, wd_margins=m)
    b = sw2d_ref.run(*args)
    assert m[0] > 1.0 and m[1] == np.inf  # every cell wet at every step, no wet/dry face
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def _wave_on_terrain(nx, ny, seed, steps, flags=WD, hmin=0.05):
    H, mask, eta = _terrain(nx, ny, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    jj, ii = np.mgrid[0:ny, 0:nx]
    bump = 0.8 * np.exp(-((ii - 0.45 * nx) ** 2 + (jj - 0.5 * ny) ** 2) / (2 * (0.12 * nx) ** 2))
    wet = (mask != 0) & (H + eta > hmin)
    eta = np.where(wet, eta + bump, eta)
    z = np.zeros((ny, nx))
    return sw2d_ref.run(nx, ny, 50.0, 50.0, 9.81, 1.5, 0.1, H, mask, eta, z, z, steps, flags=flags,
                        hmin=hmin) + (H, mask, eta)


def test_volume_is_conserved_through_flooding_and_drying():
    nx, ny = 48, 30
    e, u, v, red, H, mask, eta0 = _wave_on_terrain(nx, ny, 11, 300)
    w = mask != 0
    dry0 = w & (H + eta0 <= 0.05)
    dry1 = w & (H + e <= 0.05)
    assert (dry0 & ~dry1).sum() > 5, "the wave floods dry ground"
    v0 = math.fsum(eta0[w])
    assert abs(math.fsum(e[w]) - v0) <= 1e-12 * abs(v0)
    assert np.abs(red[:, 1] - red[0, 1]).max() <= 1e-12 * abs(red[0, 1])


def test_mirror_and_transpose_symmetry():
    """Deep in the middle, ground rising through the water line towards the east and west
    walls, a bump in the centre: the state stays mirror symmetric in x, and transposing the
    input transposes the output (u and v swapping roles)."""
    n = 34
    x = np.abs((np.arange(n) + 0.5) / n - 0.5)
    H = np.tile(np.clip(6.0 - 14.0 * x, 0.2, None), (n, 1))
    mask = np.zeros((n, n), np.uint8)
    mask[1:-1, 1:-1] = 1
    mask[9:12, 5:8] = 0
    mask[9:12, n - 8:n - 5] = 0
    assert np.array_equal(mask, mask[:, ::-1])
    H = H * mask
    eta = np.where(mask != 0, np.maximum(-1.0, -H), 0.0)
    jj, ii = np.mgrid[0:n, 0:n]
    c = (n - 1) / 2
    bump = 0.6 * np.exp(-((ii - c) ** 2 + (jj - c) ** 2) / (2 * 4.0 ** 2))
    eta = np.where((mask != 0) & (H + eta > 0.05), eta + bump, eta)
    assert ((mask != 0) & (H + eta <= 0.05)).sum() > 50
    z = np.zeros((n, n))
    e1, u1, v1, _ = sw2d_ref.run(n, n, 50.0, 50.0, 9.81, 1.5, 0.1, H, mask, eta, z, z, 80, flags=WD, hmin=0.05)
    e2, u2, v2, _ = sw2d_ref.run(n, n, 50.0, 50.0, 9.81, 1.5, 0.1, H.T.copy(), mask.T.copy(), eta.T.copy(),
                                 z, z, 80, flags=WD, hmin=0.05)
    np.testing.assert_allclose(e2, e1.T, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v2, u1.T, rtol=0, atol=1e-12)
    np.testing.assert_allclose(u2, v1.T, rtol=0, atol=1e-12)
    # mirror in x: eta symmetric, u antisymmetric about the centre
    np.testing.assert_allclose(e1[:, ::-1], e1, rtol=0, atol=1e-12)
    np.testing.assert_allclose(u1[:, -2::-1], -u1[:, :-1], rtol=0, atol=1e-12)
    assert np.abs(u1).max() > 1e-3
    assert ((mask != 0) & (H + e1 <= 0.05)).sum() != ((mask != 0) & (H + eta <= 0.05)).sum()


def test_dam_break_onto_a_dry_bed_follows_ritter():
    """Flat bed 1 m below the datum; the western half holds 1 m of water at rest, the eastern
    half is dry. With momentum advection the scheme approximates the nonlinear shallow-water
    equations, whose solution is Ritter's rarefaction: h = (2 c0 - x/t)^2 / (9 g) for
    -c0 t <= x <= 2 c0 t (c0 = sqrt(g h0)), h0 behind it, dry ahead of it, and 4/9 h0 at the
    dam. The advective (non-conservative) momentum form cannot carry momentum into a face
    that has just opened, so the tip runs as a bore at about 0.7 c0 instead of thinning out
    to 2 c0; the pin covers the rarefaction behind it, the dam depth, the still water
    upstream, a front that does advance into the dry bed, and the volume."""
    n, dx, g, h0 = 800, 1.0, 9.81, 1.0
    c0 = math.sqrt(g * h0)
    dt = 0.1 * dx / c0
    steps = 1500
    x_dam = 400
    nx, ny = n + 2, 3
    mask = np.zeros((ny, nx), np.uint8)
    mask[1, 1:-1] = 1
    H = np.where(mask != 0, 1.0, 0.0)
    eta = np.zeros((ny, nx))
    eta[1, 1:-1] = np.where(np.arange(n) < x_dam, 0.0, -1.0)
    z = np.zeros((ny, nx))
    e1, u1, _, red = sw2d_ref.run(nx, ny, dx, dx, g, dt, 0.0, H, mask, eta, z, z, steps, flags=WD | ADV,
                                  hmin=1e-4)
    t = steps * dt
    x = (np.arange(n) + 0.5 - x_dam) * dx  # cell centres from the dam
    h = (H + e1)[1, 1:-1]
    xi = x / t
    ritter = (2 * c0 - np.clip(xi, -c0, 2 * c0)) ** 2 / (9 * g)
    fan = (xi > -0.9 * c0) & (xi < -0.1 * c0)
    err = np.abs(h - ritter)[fan].max()
    assert err < 0.01 * h0, err
    assert abs(h[x_dam] - 4 / 9 * h0) < 0.02 * h0
    assert np.all(np.abs(h[xi < -1.1 * c0] - h0) < 1e-3)
    wet = np.nonzero(h > 1e-3)[0]
    assert 0.5 * c0 * t < x[wet.max()] < 2 * c0 * t
    assert np.all(h[xi > 2 * c0] == 0.0)
    assert abs(red[-1, 1] - red[0, 1]) <= 1e-12 * abs(red[0, 1])
