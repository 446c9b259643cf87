"""The oracle against closed forms of the linearised scheme.

At small amplitude the total depth is H, and with uniform H on an all-water
rectangle each standing mode eta = E cos(k x) cos(l y) (with u ~ sin(k x_e), v ~
sin(l y_n)) is an eigenfunction of every stage:
  * pressure-gradient predictor:  P_u' = P_u + (g dt/dx) 2 s_x E, P_v' likewise in y;
  * flux divergence:              E* = E - (H dt/dx) 2 s_x P_u' - (H dt/dy) 2 s_y P_v';
  * masked five-point Shapiro:    E' = (1 - eps (s_x^2 + s_y^2)) E*
    (the wall rows see a mirror image of themselves, so dropping land neighbours is exact);
with s_x = sin(k dx / 2), s_y = sin(l dy / 2). A wrong sign, a dropped term, a
transposed dx/dy or an eta update from the old velocities all change these numbers.
The continuum checks: a pulse travels at sqrt(g H) and the gravest seiche of a
basin of length L has period 2 L / sqrt(g H) (Merian's formula).
"""
import math

import numpy as np

from oracle import sw2d_ref


def _basin(nxi, nyi, H=10.0):
    nx, ny = nxi + 2, nyi + 2
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[1:-1, 1:-1] = 1
    return nx, ny, mask, np.full((ny, nx), H)


def _mode_fields(nxi, nyi, dx, dy, m, mp, E, Pu, Pv):
    nx, ny = nxi + 2, nyi + 2
    k, l = m * math.pi / (nxi * dx), mp * math.pi / (nyi * dy)
    xc = (np.arange(nx) - 0.5) * dx  # cell centres from the west wall
    yc = (np.arange(ny) - 0.5) * dy
    xe = np.arange(nx) * dx  # east faces
    yn = np.arange(ny) * dy  # north faces
    eta = E * np.outer(np.cos(l * yc), np.cos(k * xc))
    u = Pu * np.outer(np.cos(l * yc), np.sin(k * xe))
    v = Pv * np.outer(np.sin(l * yn), np.cos(k * xc))
    inner = np.zeros((ny, nx), dtype=bool)
    inner[1:-1, 1:-1] = True
    eta[~inner] = 0.0
    u[:, 0] = 0.0
    u[:, nx - 2:] = 0.0
    u[[0, ny - 1], :] = 0.0
    v[0, :] = 0.0
    v[ny - 2:, :] = 0.0
    v[:, [0, nx - 1]] = 0.0
    return eta, u, v


def _amplify(nxi, nyi, dx, dy, g, dt, eps, H, m, mp, E0, nsteps):
    k, l = m * math.pi / (nxi * dx), mp * math.pi / (nyi * dy)
    sx, sy = math.sin(k * dx / 2), math.sin(l * dy / 2)
    f = 1.0 - eps * (sx * sx + sy * sy)
    E, Pu, Pv = E0, 0.0, 0.0
    for _ in range(nsteps):
        Pu = Pu + g * dt / dx * 2 * sx * E
        Pv = Pv + g * dt / dy * 2 * sy * E
        E = f * (E - H * dt / dx * 2 * sx * Pu - H * dt / dy * 2 * sy * Pv)
    return E, Pu, Pv


def test_mode_amplification_matches_closed_form():
    nxi, nyi, dx, dy, g, H, eps = 32, 24, 100.0, 150.0, 9.81, 10.0, 0.05
    dt = 0.5 * min(dx, dy) / math.sqrt(g * H)
    nx, ny, mask, Hf = _basin(nxi, nyi, H)
    E0, n = 1e-7, 200
    for (m, mp) in ((1, 0), (0, 1), (2, 1), (3, 2)):
        eta, u, v = _mode_fields(nxi, nyi, dx, dy, m, mp, E0, 0.0, 0.0)
        e, uu, vv, _ = sw2d_ref.run(nx, ny, dx, dy, g, dt, eps, Hf, mask, eta, u, v, n)
        E, Pu, Pv = _amplify(nxi, nyi, dx, dy, g, dt, eps, H, m, mp, E0, n)
        te, tu, tv = _mode_fields(nxi, nyi, dx, dy, m, mp, E, Pu, Pv)
        # residue: the nonlinear total depth H + eta, relative size eta/H ~ 1e-8
        assert np.abs(e - te).max() <= 1e-6 * E0, (m, mp, np.abs(e - te).max())
        scale_u = max(abs(Pu), abs(Pv), 1e-30)
        assert np.abs(uu - tu).max() <= 1e-6 * scale_u, (m, mp)
        assert np.abs(vv - tv).max() <= 1e-6 * scale_u, (m, mp)


def test_filter_alone_multiplies_each_mode():
    nxi, nyi, dx, dy, H, eps = 20, 28, 100.0, 80.0, 10.0, 0.3
    nx, ny, mask, Hf = _basin(nxi, nyi, H)
    for (m, mp) in ((1, 1), (5, 3), (19, 27)):
        eta, u, v = _mode_fields(nxi, nyi, dx, dy, m, mp, 0.5, 0.0, 0.0)
        e, uu, vv, _ = sw2d_ref.run(nx, ny, dx, dy, 0.0, 1.0, eps, Hf, mask, eta, u, v, 10)
        k, l = m * math.pi / (nxi * dx), mp * math.pi / (nyi * dy)
        f = 1.0 - eps * (math.sin(k * dx / 2) ** 2 + math.sin(l * dy / 2) ** 2)
        np.testing.assert_allclose(e, f ** 10 * eta, rtol=0, atol=1e-13 * 0.5)
        assert not np.any(uu) and not np.any(vv)


def test_wave_front_moves_at_sqrt_gH():
    nxi, dx, g, H = 400, 100.0, 9.81, 10.0
    nx, ny, mask, Hf = _basin(nxi, 1, H)
    c = math.sqrt(g * H)
    dt = 0.5 * dx / c
    x0 = 100.0 * dx
    xc = (np.arange(nx) - 0.5) * dx
    eta = np.zeros((ny, nx))
    eta[1, 1:-1] = 1e-3 * np.exp(-((xc[1:-1] - x0) ** 2) / (2 * (5 * dx) ** 2))
    z = np.zeros((ny, nx))
    n = 300
    e, _, _, _ = sw2d_ref.run(nx, ny, dx, dx, g, dt, 0.05, Hf, mask, eta, z, z, n)
    row = e[1]
    lo = int((x0 + 0.5 * c * n * dt) / dx)  # the right-going half only
    k = lo + int(np.argmax(row[lo:-1]))
    a, b, cc = row[k - 1], row[k], row[k + 1]
    peak = xc[k] + 0.5 * dx * (a - cc) / (a - 2 * b + cc)
    expect = x0 + c * n * dt
    assert abs(peak - expect) <= dx + 0.01 * c * n * dt, (peak, expect)


def test_gravest_seiche_period():
    nxi, dx, g, H = 256, 100.0, 9.81, 10.0
    nx, ny, mask, Hf = _basin(nxi, 1, H)
    c = math.sqrt(g * H)
    dt = 0.5 * dx / c
    L = nxi * dx
    eta, u, v = _mode_fields(nxi, 1, dx, dx, 1, 0, 1e-6, 0.0, 0.0)
    k = math.pi / L
    proj = np.cos(k * (np.arange(nx) - 0.5) * dx)[1:-1]
    series = [eta[1, 1:-1] @ proj]
    for _ in range(1400):
        eta, u, v, _ = sw2d_ref.run(nx, ny, dx, dx, g, dt, 0.0, Hf, mask, eta, u, v, 1,
                                    reductions=False)
        series.append(eta[1, 1:-1] @ proj)
    s = np.array(series)
    cross = [t + s[t] / (s[t] - s[t + 1]) for t in range(len(s) - 1) if s[t] > 0 >= s[t + 1]
             or s[t] < 0 <= s[t + 1]]
    T = 2.0 * (cross[1] - cross[0]) * dt
    # discrete forward-backward dispersion: sin(w dt / 2) = c dt sin(k dx / 2) / dx
    w = 2.0 / dt * math.asin(c * dt * math.sin(k * dx / 2) / dx)
    assert abs(T - 2 * math.pi / w) <= 1e-6 * T
    # the continuum limit (Merian): T1 = 2 L / sqrt(g H), to O((k dx)^2)
    assert abs(T - 2 * L / c) <= 1e-3 * T
