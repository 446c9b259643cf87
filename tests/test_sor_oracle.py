"""Pins of the FP64 red-black SOR oracle against what the mathematics fixes.

* one iteration equals the matrix form of SOR, x' = (D + w E)^-1 (w b - (w F + (w - 1) D) x),
  with A = D + E + F the negative Laplacian of the interior unknowns taken in red-black
  order (reds first) and solved densely by numpy;
* the iteration converges to a manufactured discrete solution (f = L p* by array slicing);
* asymptotic rates from Young's theory for the consistently ordered 7-point matrix: at
  w = 1 the residual shrinks by rho_J^2 per iteration, rho_J = sum_d c_d cos(pi / (N_d + 1))
  / sum_d c_d; for w above w_opt = 2 / (1 + sqrt(1 - rho_J^2)) every eigenvalue has modulus
  w - 1;
* the residual fold equals a compensated (fsum) recomputation; boundary values are never
  written; the zero problem stays exactly zero.
"""
import math

import numpy as np
import pytest

from oracle import sor_ref

SPACING = (1.0, 1.3, 0.7)


def lap(p, dx, dy, dz):
    """L p on the interior (numpy slicing, the definition written out once more)."""
    cx, cy, cz = 1 / dx ** 2, 1 / dy ** 2, 1 / dz ** 2
    c = p[1:-1, 1:-1, 1:-1]
    return (cx * (p[1:-1, 1:-1, 2:] + p[1:-1, 1:-1, :-2] - 2 * c)
            + cy * (p[1:-1, 2:, 1:-1] + p[1:-1, :-2, 1:-1] - 2 * c)
            + cz * (p[2:, 1:-1, 1:-1] + p[:-2, 1:-1, 1:-1] - 2 * c))


def sor_matrix_iteration(p, f, dx, dy, dz, omega):
    """One SOR iteration in matrix-splitting form over the interior unknowns."""
    nz, ny, nx = p.shape
    cx, cy, cz = 1 / dx ** 2, 1 / dy ** 2, 1 / dz ** 2
    cells = [(k, j, i) for k in range(1, nz - 1) for j in range(1, ny - 1) for i in range(1, nx - 1)]
    order = [c for c in cells if sum(c) % 2 == 0] + [c for c in cells if sum(c) % 2 == 1]
    idx = {c: q for q, c in enumerate(order)}
    n = len(order)
    A = np.zeros((n, n))
    b = np.zeros(n)
    for q, (k, j, i) in enumerate(order):
        A[q, q] = 2 * (cx + cy + cz)
        b[q] = -f[k, j, i]
        for (dk, dj, di), c in (((0, 0, 1), cx), ((0, 0, -1), cx), ((0, 1, 0), cy), ((0, -1, 0), cy),
                                ((1, 0, 0), cz), ((-1, 0, 0), cz)):
            nb = (k + dk, j + dj, i + di)
            if nb in idx:
                A[q, idx[nb]] = -c
            else:
                b[q] += c * p[nb]
    D = np.diag(np.diag(A))
    E = np.tril(A, -1)
    F = np.triu(A, 1)
    x = np.array([p[c] for c in order])
    x_new = np.linalg.solve(D + omega * E, omega * b - (omega * F + (omega - 1) * D) @ x)
    out = p.copy()
    for q, c in enumerate(order):
        out[c] = x_new[q]
    return out


def rho_jacobi(shape, dx, dy, dz):
    nz, ny, nx = shape
    c = (1 / dx ** 2, 1 / dy ** 2, 1 / dz ** 2)
    cos = (math.cos(math.pi / (nx - 1)), math.cos(math.pi / (ny - 1)), math.cos(math.pi / (nz - 1)))
    return sum(a * b for a, b in zip(c, cos)) / sum(c)


@pytest.mark.parametrize("omega", [1.0, 1.45, 1.9])
@pytest.mark.parametrize("shape", [(4, 5, 6), (5, 4, 7)])
def test_one_iteration_equals_matrix_splitting(shape, omega):
    rng = np.random.default_rng(sum(shape) + int(omega * 100))
    p = rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    got, _ = sor_ref.run(p, f, 1, *SPACING, omega=omega)
    want = sor_matrix_iteration(p, f, *SPACING, omega)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_converges_to_manufactured_solution():
    rng = np.random.default_rng(7)
    shape = (8, 9, 10)
    ps = rng.standard_normal(shape)
    f = np.zeros(shape)
    f[1:-1, 1:-1, 1:-1] = lap(ps, *SPACING)
    p0 = ps.copy()
    p0[1:-1, 1:-1, 1:-1] = 0.0
    p, res = sor_ref.run(p0, f, 400, *SPACING, omega=1.7)
    assert np.max(np.abs(p - ps)) < 1e-10
    assert res[-1, 0] < 1e-18
    assert np.all(np.diff(np.log(res[:200, 0])) < 0.5)  # no blow-up on the way


def test_gauss_seidel_rate_is_rho_jacobi_squared():
    shape = (11, 13, 16)  # interior 9 x 11 x 14
    rng = np.random.default_rng(3)
    p0 = np.zeros(shape)
    p0[1:-1, 1:-1, 1:-1] = rng.standard_normal((9, 11, 14))
    _, res = sor_ref.run(p0, np.zeros(shape), 300, *SPACING, omega=1.0)
    rate = math.sqrt(res[-1, 0] / res[-2, 0])
    assert abs(rate - rho_jacobi(shape, *SPACING) ** 2) < 1e-4


def test_overrelaxed_rate_is_omega_minus_one():
    shape = (9, 10, 12)
    rj = rho_jacobi(shape, *SPACING)
    w_opt = 2 / (1 + math.sqrt(1 - rj * rj))
    omega = 0.5 * (w_opt + 2.0)
    rng = np.random.default_rng(5)
    p0 = np.zeros(shape)
    p0[1:-1, 1:-1, 1:-1] = rng.standard_normal((7, 8, 10))
    _, res = sor_ref.run(p0, np.zeros(shape), 400, *SPACING, omega=omega)
    m = 200
    rate = (math.sqrt(res[-1, 0] / res[-1 - m, 0])) ** (1.0 / m)
    assert abs(rate - (omega - 1)) < 0.01 * (omega - 1)


def test_residual_fold_matches_fsum():
    rng = np.random.default_rng(11)
    shape = (6, 7, 9)
    p0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    p, res = sor_ref.run(p0, f, 3, *SPACING, omega=1.3)
    r = f[1:-1, 1:-1, 1:-1] - lap(p, *SPACING)
    assert math.isclose(res[-1, 0], math.fsum((r * r).ravel()), rel_tol=1e-12)
    assert math.isclose(res[-1, 1], float(np.max(np.abs(r))), rel_tol=1e-12)
    s2, mx = sor_ref.residual(p, f, *SPACING)
    assert (s2, mx) == (res[-1, 0], res[-1, 1])


def test_boundary_untouched_and_zero_problem():
    rng = np.random.default_rng(13)
    shape = (5, 6, 7)
    p0 = rng.standard_normal(shape)
    p, _ = sor_ref.run(p0, rng.standard_normal(shape), 4, *SPACING, omega=1.6)
    inner = np.zeros(shape, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    assert np.array_equal(p[~inner], p0[~inner])
    z, res = sor_ref.run(np.zeros(shape), np.zeros(shape), 5, *SPACING, omega=1.6)
    assert not z.any() and not res.any()
