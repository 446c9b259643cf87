"""Pins of the oracle's model variants (friction on the predictor, Shapiro filter on the
velocities) against closed forms and invariants.

* friction: with a level surface the predictor is u / (1 + dt cd |u| / h_face) face by face;
* velocity filter: with g = 0 the velocities evolve by the masked filter alone, whose
  eigenvectors on an Mx x My block of active faces are the Neumann cosines
  cos(pi k (m + 1/2) / M) with factor 1 - eps (sin^2(pi k / 2Mx) + sin^2(pi l / 2My)) per step;
  the filter conserves the sum over active faces; the surface update of a step uses the
  unfiltered velocities;
* both: a lake at rest stays bitwise at rest and the volume is conserved.
"""
import math

import numpy as np
import pytest

from oracle import sw2d_ref

FR, UV = sw2d_ref.FRICTION, sw2d_ref.FILTER_UV


def _basin(n, H=10.0):
    nx = ny = n + 2
    mask = np.zeros((ny, nx), np.uint8)
    mask[1:-1, 1:-1] = 1
    return nx, ny, np.full((ny, nx), H) * mask, mask


def _faces(mask):
    w = mask != 0
    au = np.zeros_like(w)
    au[:, :-1] = w[:, :-1] & w[:, 1:]
    av = np.zeros_like(w)
    av[:-1] = w[:-1] & w[1:]
    return au, av


def test_friction_divides_the_predictor_by_the_old_speed():
    """A tilted surface: us = (u - g dt/dx (eta_E - eta)) / (1 + dt cd |u_old| / h_face)."""
    rng = np.random.default_rng(2)
    n = 10
    nx, ny, _, mask = _basin(n)
    H = (8.0 + 10.0 * rng.uniform(size=(ny, nx))) * mask
    au, av = _faces(mask)
    eta = 0.2 * rng.standard_normal((ny, nx)) * mask
    u = rng.uniform(-0.5, 0.5, (ny, nx)) * au
    v = rng.uniform(-0.5, 0.5, (ny, nx)) * av
    g, dt, dx, dy, cd = 9.81, 3.0, 100.0, 80.0, 0.004
    _, u1, v1, _ = sw2d_ref.run(nx, ny, dx, dy, g, dt, 0.0, H, mask, eta, u, v, 1, flags=FR, cd=cd)
    h = H + eta
    nu = np.zeros_like(u)
    nu[:, :-1] = u[:, :-1] - g * dt / dx * (eta[:, 1:] - eta[:, :-1])
    hu = np.ones_like(h)
    hu[:, :-1] = 0.5 * (h[:, :-1] + h[:, 1:])
    nv = np.zeros_like(v)
    nv[:-1] = v[:-1] - g * dt / dy * (eta[1:] - eta[:-1])
    hv = np.ones_like(h)
    hv[:-1] = 0.5 * (h[:-1] + h[1:])
    np.testing.assert_allclose(u1, np.where(au, nu / (1 + dt * cd * np.abs(u) / hu), 0), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(v1, np.where(av, nv / (1 + dt * cd * np.abs(v) / hv), 0), rtol=1e-13, atol=1e-15)


def test_friction_is_the_closed_form_on_a_level_surface():
    rng = np.random.default_rng(1)
    n = 12
    nx, ny, _, mask = _basin(n)
    H = (5.0 + 20.0 * rng.uniform(size=(ny, nx))) * mask
    au, av = _faces(mask)
    level = 0.3
    eta = level * mask.astype(float)
    u = rng.uniform(-0.5, 0.5, (ny, nx)) * au
    v = rng.uniform(-0.5, 0.5, (ny, nx)) * av
    dt, cd = 2.0, 0.0025
    _, u1, v1, _ = sw2d_ref.run(nx, ny, 100.0, 100.0, 9.81, dt, 0.05, H, mask, eta, u, v, 1, flags=FR, cd=cd)
    h = H + eta
    hu = np.zeros_like(h)
    hu[:, :-1] = 0.5 * (h[:, :-1] + h[:, 1:])
    hv = np.zeros_like(h)
    hv[:-1] = 0.5 * (h[:-1] + h[1:])
    with np.errstate(invalid="ignore", divide="ignore"):
        want_u = np.where(au, u / (1 + dt * cd * np.abs(u) / np.where(au, hu, 1)), 0)
        want_v = np.where(av, v / (1 + dt * cd * np.abs(v) / np.where(av, hv, 1)), 0)
    np.testing.assert_allclose(u1, want_u, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(v1, want_v, rtol=1e-14, atol=1e-16)
    assert np.abs(u1).max() < np.abs(u).max()


@pytest.mark.parametrize("k,l", [(1, 0), (2, 3), (5, 1)])
def test_velocity_filter_modes_decay_by_the_closed_form(k, l):
    n, eps, steps = 16, 0.3, 25
    nx, ny, H, mask = _basin(n)
    au, av = _faces(mask)
    u = np.zeros((ny, nx))
    v = np.zeros((ny, nx))
    mxu, myu = n - 1, n  # active u faces: columns 1..n-1, rows 1..n
    for j in range(1, n + 1):
        for i in range(1, n):
            u[j, i] = math.cos(math.pi * k * (i - 1 + 0.5) / mxu) * math.cos(math.pi * l * (j - 1 + 0.5) / myu)
    mxv, myv = n, n - 1
    for j in range(1, n):
        for i in range(1, n + 1):
            v[j, i] = math.cos(math.pi * l * (i - 1 + 0.5) / mxv) * math.cos(math.pi * k * (j - 1 + 0.5) / myv)
    eta = np.zeros((ny, nx))
    _, ue, ve, _ = sw2d_ref.run(nx, ny, 100.0, 100.0, 0.0, 1.0, eps, H, mask, eta, u, v, steps, flags=UV)
    fu = 1 - eps * (math.sin(math.pi * k / (2 * mxu)) ** 2 + math.sin(math.pi * l / (2 * myu)) ** 2)
    fv = 1 - eps * (math.sin(math.pi * l / (2 * mxv)) ** 2 + math.sin(math.pi * k / (2 * myv)) ** 2)
    np.testing.assert_allclose(ue, fu ** steps * u, rtol=0, atol=1e-13)
    np.testing.assert_allclose(ve, fv ** steps * v, rtol=0, atol=1e-13)


def test_velocity_filter_conserves_the_face_sum_and_follows_the_surface_update():
    rng = np.random.default_rng(4)
    n = 14
    nx, ny, H, mask = _basin(n)
    mask[5:8, 6:9] = 0  # an island
    H = H * mask
    au, av = _faces(mask)
    u = rng.standard_normal((ny, nx)) * au
    v = rng.standard_normal((ny, nx)) * av
    eta = 0.1 * rng.standard_normal((ny, nx)) * mask
    _, ue, ve, _ = sw2d_ref.run(nx, ny, 100.0, 100.0, 0.0, 1.0, 0.4, H, mask, eta, u, v, 7, flags=UV)
    assert math.isclose(math.fsum(ue[au]), math.fsum(u[au]), rel_tol=0, abs_tol=1e-12)
    assert math.isclose(math.fsum(ve[av]), math.fsum(v[av]), rel_tol=0, abs_tol=1e-12)
    assert not ue[~au].any() and not ve[~av].any()
    # one step: the surface comes from the unfiltered predictor
    e1, _, _, _ = sw2d_ref.run(nx, ny, 100.0, 100.0, 9.81, 1.0, 0.4, H, mask, eta, u, v, 1, flags=UV)
    e0, _, _, _ = sw2d_ref.run(nx, ny, 100.0, 100.0, 9.81, 1.0, 0.4, H, mask, eta, u, v, 1)
    assert np.array_equal(e1, e0)


@pytest.mark.parametrize("flags", [FR, UV, FR | UV])
def test_variants_keep_lake_at_rest_and_volume(flags):
    rng = np.random.default_rng(9)
    n = 20
    nx, ny, _, mask = _basin(n)
    mask[8:12, 3:7] = 0
    H = (5 + 30 * rng.uniform(size=(ny, nx))) * mask
    eta = 0.2 * mask.astype(float)
    z = np.zeros((ny, nx))
    e, u, v, _ = sw2d_ref.run(nx, ny, 100.0, 100.0, 9.81, 1.5, 0.1, H, mask, eta, z, z, 30, flags=flags, cd=0.003)
    assert np.array_equal(e, eta) and not u.any() and not v.any()
    bump = eta + 0.3 * np.exp(-((np.arange(nx)[None] - 14) ** 2 + (np.arange(ny)[:, None] - 6) ** 2) / 8.0) * mask
    e, u, v, red = sw2d_ref.run(nx, ny, 100.0, 100.0, 9.81, 1.5, 0.1, H, mask, bump, z, z, 60, flags=flags, cd=0.003)
    assert abs(red[-1, 1] - red[0, 1]) <= 1e-12 * abs(red[0, 1])


AD = sw2d_ref.ADVECTION


def _channel(nx, ny):
    mask = np.zeros((ny, nx), np.uint8)
    mask[1:-1, 1:-1] = 1
    return np.full((ny, nx), 10.0) * mask, mask


@pytest.mark.parametrize("a", [0.03, -0.05])
def test_advection_of_linear_profiles_is_exact(a):
    """Away from the walls a one-sided difference of a linear profile is its slope, on
    either side: u = a i + b (v = 0) gives us = u - dt u a / dx; u = a j with v = V gives
    us = u - dt V a / dy; v = a j gives vs = v - dt v a / dy; v = a i with u = U gives
    vs = v - dt U a / dx. A level surface, so no pressure gradient."""
    nx, ny, dx, dy, dt = 24, 20, 100.0, 70.0, 3.0
    H, mask = _channel(nx, ny)
    au, av = _faces(mask)
    eta = np.zeros((ny, nx))
    jj, ii = np.mgrid[0:ny, 0:nx].astype(float)
    # interior faces: all neighbouring faces (and the four around) active
    inner = np.zeros((ny, nx), bool)
    inner[3:-3, 3:-3] = True
    run = lambda u, v: sw2d_ref.run(nx, ny, dx, dy, 9.81, dt, 0.0, H, mask, eta, u, v, 1, flags=AD)
    # u linear in i, v = 0
    u = (a * ii + 0.1) * au
    _, u1, _, _ = run(u, np.zeros_like(u))
    np.testing.assert_allclose(u1[inner & au], (u - dt * u * a / dx)[inner & au], rtol=1e-13, atol=1e-16)
    # u linear in j advected by a uniform v (either sign)
    for V in (0.2, -0.25):
        u = (a * jj + 0.05) * au
        v = V * av
        _, u1, v1, _ = run(u, v)
        np.testing.assert_allclose(u1[inner & au], (u - dt * V * a / dy)[inner & au], rtol=1e-13, atol=1e-16)
    # v linear in j, u = 0
    v = (a * jj - 0.1) * av
    _, _, v1, _ = run(np.zeros_like(v), v)
    np.testing.assert_allclose(v1[inner & av], (v - dt * v * a / dy)[inner & av], rtol=1e-13, atol=1e-16)
    # v linear in i advected by a uniform u (either sign)
    for U in (-0.15, 0.3):
        v = (a * ii + 0.02) * av
        u = U * au
        _, u1, v1, _ = run(u, v)
        np.testing.assert_allclose(v1[inner & av], (v - dt * U * a / dx)[inner & av], rtol=1e-13, atol=1e-16)


def test_advection_keeps_mirror_and_transpose_symmetry():
    from paper_1711_04471_amd import inputs
    c = inputs.small_basin(41, 36, seed=17, steps=20)
    c.dy, c.dt = 0.7 * c.dx, 0.7 * c.dt  # anisotropic, so the transpose tells dx from dy
    rng = np.random.Generator(np.random.PCG64(71))
    au, av = _faces(c.mask)
    c.u = (rng.uniform(-0.3, 0.3, c.u.shape) * au).astype(np.float32)
    c.v = (rng.uniform(-0.3, 0.3, c.v.shape) * av).astype(np.float32)
    e, u, v, _ = sw2d_ref.run_case(c, flags=AD)
    # mirror in x: eta(i) -> eta(nx-1-i), u on east faces (i) -> -u(nx-2-i), v(i) -> v(nx-1-i)
    mu0 = np.zeros_like(c.u)
    mu0[:, :-1] = -c.u[:, -2::-1]
    me, mu, mv, _ = sw2d_ref.run(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps, c.H[:, ::-1], c.mask[:, ::-1],
                                 c.eta[:, ::-1], mu0, c.v[:, ::-1], c.steps, flags=AD)
    np.testing.assert_allclose(me[:, ::-1], e, rtol=0, atol=1e-13 * np.abs(e).max())
    np.testing.assert_allclose(-mu[:, -2::-1], u[:, :-1], rtol=0, atol=1e-13 * np.abs(u).max())
    np.testing.assert_allclose(mv[:, ::-1], v, rtol=0, atol=1e-13 * np.abs(v).max())
    # transpose: swap axes, u <-> v, dx <-> dy
    te, tu, tv, _ = sw2d_ref.run(c.ny, c.nx, c.dy, c.dx, c.g, c.dt, c.eps, c.H.T, c.mask.T, c.eta.T,
                                 c.v.T, c.u.T, c.steps, flags=AD)
    np.testing.assert_allclose(te.T, e, rtol=0, atol=1e-13 * np.abs(e).max())
    np.testing.assert_allclose(tv.T, u, rtol=0, atol=1e-13 * np.abs(u).max())
    np.testing.assert_allclose(tu.T, v, rtol=0, atol=1e-13 * np.abs(v).max())


@pytest.mark.parametrize("flags", [AD, AD | FR | UV])
def test_advection_keeps_lake_at_rest_and_volume(flags):
    test_variants_keep_lake_at_rest_and_volume(flags)
