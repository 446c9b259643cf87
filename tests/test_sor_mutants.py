"""Plant plausible mistakes in a copy of the SOR oracle and check that the pins catch each.

Every mutant is compiled from the oracle source with one textual change and must fail at
least one of: the matrix-splitting form of one iteration, convergence to a manufactured
solution, the Gauss-Seidel and over-relaxed asymptotic rates, or the fsum residual check.
"""
import os
import subprocess

import numpy as np
import pytest

from oracle import build as obuild
from oracle import sor_ref

HERE = os.path.dirname(__file__)
SRC = os.path.join(os.path.dirname(HERE), "oracle", "sor_oracle.c")

MUTANTS = {
    "black_before_red": ("sweep(nx, ny, nz, cx, cy, cz, omega, 0, p, f);\n        sweep(nx, ny, nz, cx, cy, cz, omega, 1, p, f);",
                         "sweep(nx, ny, nz, cx, cy, cz, omega, 1, p, f);\n        sweep(nx, ny, nz, cx, cy, cz, omega, 0, p, f);"),
    "relaxation_reversed": ("p[IX(i, j, k)] = old + omega * (g - old);", "p[IX(i, j, k)] = g + omega * (old - g);"),
    "dz_spacing_uses_dy": ("cz = 1.0 / (dz * dz);", "cz = 1.0 / (dy * dy);"),
    "diagonal_without_2": ("const double diag = 2.0 * (cx + cy + cz);", "const double diag = (cx + cy + cz);"),
    "colour_ignores_k": ("if (((i + j + k) & 1) != color) continue;", "if (((i + j) & 1) != color) continue;"),
    "source_sign": ("const double g = (nb - f[IX(i, j, k)]) / diag;", "const double g = (nb + f[IX(i, j, k)]) / diag;"),
    "west_neighbour_twice": ("cx * (p[IX(i + 1, j, k)] + p[IX(i - 1, j, k)]) +\n", "cx * (p[IX(i - 1, j, k)] + p[IX(i - 1, j, k)]) +\n"),
    "residual_drops_z": ("cz * (p[IX(i, j, k + 1)] + p[IX(i, j, k - 1)] - 2.0 * c);", "0.0;"),
}


def _build_mutant(tmp_path, name, find, repl):
    src = open(SRC).read()
    assert src.count(find) == 1, f"{name}: pattern must occur exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(find, repl))
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", *obuild.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    return str(lib)


def _pin_matrix():
    from tests.test_sor_oracle import test_one_iteration_equals_matrix_splitting
    for shape in ((4, 5, 6), (5, 4, 7)):
        for omega in (1.0, 1.45):
            test_one_iteration_equals_matrix_splitting(shape, omega)


def _pin_manufactured():
    from tests.test_sor_oracle import test_converges_to_manufactured_solution
    test_converges_to_manufactured_solution()


def _pin_rates():
    from tests.test_sor_oracle import (test_gauss_seidel_rate_is_rho_jacobi_squared,
                                       test_overrelaxed_rate_is_omega_minus_one)
    test_gauss_seidel_rate_is_rho_jacobi_squared()
    test_overrelaxed_rate_is_omega_minus_one()


def _pin_residual():
    from tests.test_sor_oracle import test_residual_fold_matches_fsum
    test_residual_fold_matches_fsum()


PINS = (_pin_matrix, _pin_manufactured, _pin_rates, _pin_residual)


def test_unmutated_oracle_passes_every_pin():
    for pin in PINS:
        pin()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_is_caught(tmp_path, name):
    lib = _build_mutant(tmp_path, name, *MUTANTS[name])
    caught = []
    with sor_ref.library(lib):
        for pin in PINS:
            try:
                with np.errstate(all="ignore"):
                    pin()
            except (AssertionError, ValueError, np.linalg.LinAlgError):
                caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
