"""Plant plausible mistakes in a copy of the C oracle and check that the pins catch each.

Every mutant is compiled from the oracle source with one textual change and must
fail at least one of: the hand-derived two-cell steps, the closed-form mode
amplification, exact rational arithmetic on tiny grids, or volume conservation.
"""
import json
import os
import subprocess

import numpy as np
import pytest

from oracle import build as obuild
from oracle import exact, sw2d_ref
from paper_1711_04471_amd import inputs

HERE = os.path.dirname(__file__)
SRC = os.path.join(os.path.dirname(HERE), "oracle", "sw2d_oracle.c")

MUTANTS = {
    "upwind_flipped": ("us > 0.0 ? AT(H, j, i) + AT(eta, j, i)", "us < 0.0 ? AT(H, j, i) + AT(eta, j, i)"),
    "eta_from_old_velocity": ("fx = us * h_up;", "fx = AT(u, j, i) * h_up;"),
    "pressure_gradient_sign": ("us = AT(u, j, i) - cx *", "us = AT(u, j, i) + cx *"),
    "dx_for_dy_in_v_predictor": ("vs = AT(v, j, i) - cy *", "vs = AT(v, j, i) - cx *"),
    "west_flux_index": ("double fw = i > 0 ? AT(Fx, j, i - 1) : 0.0;", "double fw = i > 0 ? AT(Fx, j, i) : 0.0;"),
    "south_flux_dropped": ("- ry * (AT(Fy, j, i) - fs)", "- ry * AT(Fy, j, i)"),
    "shapiro_drops_north": ("if (filter_nb(H, eta, mask, nx, ny, j + 1, i, wd, hmin)) s += AT(es, j + 1, i) - c;", ""),
    "shapiro_over_land": ("if (filter_nb(H, eta, mask, nx, ny, j, i - 1, wd, hmin)) s += AT(es, j, i - 1) - c;",
                          "s += AT(es, j, i - 1) - c;"),
    "shapiro_eps_over_2": ("const double e4 = eps / 4.0;", "const double e4 = eps / 2.0;"),
    "depth_from_new_side": ("AT(H, j + 1, i) + AT(eta, j + 1, i);", "AT(H, j, i) + AT(eta, j + 1, i);"),
    "volume_counts_land": ("if (AT(mask, j, i)) {", "{"),
    # model variants
    "friction_uses_new_velocity": ("us = us / (1.0 + kf * fabs(AT(u, j, i)) / hf);", "us = us / (1.0 + kf * fabs(us) / hf);"),
    "friction_one_sided_depth": ("double hf = 0.5 * ((AT(H, j, i) + AT(eta, j, i)) + (AT(H, j, i + 1) + AT(eta, j, i + 1)));",
                                 "double hf = AT(H, j, i) + AT(eta, j, i);"),
    "uv_filter_over_inactive_faces": ("if (act(mask, nx, ny, j + 1, i)) s += AT(a, j + 1, i) - c;", "s += AT(a, j + 1, i) - c;"),
    "advection_downwind_x": ("const double ax = c > 0.0 ? c * (c - face_at(u, nx, ny, j, i - 1)) / dx",
                             "const double ax = c < 0.0 ? c * (c - face_at(u, nx, ny, j, i - 1)) / dx"),
    "advection_vbar_drops_a_face": ("(face_at(v, nx, ny, j - 1, i) + face_at(v, nx, ny, j - 1, i + 1)));",
                                    "(face_at(v, nx, ny, j - 1, i) + 0.0));"),
    "advection_dy_by_dx": ("                                 : vbar * (face_at(u, nx, ny, j + 1, i) - c) / dy;",
                           "                                 : vbar * (face_at(u, nx, ny, j + 1, i) - c) / dx;"),
    "advection_v_wrong_neighbour": ("const double by = c > 0.0 ? c * (c - face_at(v, nx, ny, j - 1, i)) / dy",
                                    "const double by = c > 0.0 ? c * (c - face_at(v, nx, ny, j, i - 1)) / dy"),
    "uv_filter_v_on_u_faces": ("filter_faces(nx, ny, e4, mask, v_out, Fy, v_face);", "filter_faces(nx, ny, e4, mask, v_out, Fy, u_face);"),
    "wetdry_opens_toward_a_higher_dry_cell": ("return (wa && wb) || (wa && ea > eb) || (wb && eb > ea);",
                                              "return (wa && wb) || (wa && ea < eb) || (wb && eb < ea);"),
    "wetdry_any_wet_side_opens": ("return (wa && wb) || (wa && ea > eb) || (wb && eb > ea);", "return wa || wb;"),
    "wetdry_two_dry_cells_open": ("return (wa && wb) || (wa && ea > eb) || (wb && eb > ea);",
                                  "return (wa == wb) || (wa && ea > eb) || (wb && eb > ea);"),
    "wetdry_threshold_inclusive": ("return is_wet(mask, nx, ny, j, i) && AT(H, j, i) + AT(eta, j, i) > hmin;",
                                   "return is_wet(mask, nx, ny, j, i) && AT(H, j, i) + AT(eta, j, i) >= hmin;"),
    "wetdry_dry_cells_filtered": ("out = (wd && !wet_now(H, eta, mask, nx, ny, j, i, hmin)) ? c : c + e4 * s;",
                                  "out = c + e4 * s;"),
    "wetdry_filter_across_dry_neighbours": ("return wd ? wet_now(H, eta, mask, nx, ny, j, i, hmin) : is_wet(mask, nx, ny, j, i);",
                                            "return is_wet(mask, nx, ny, j, i);"),
}


def _build_mutant(tmp_path, name, find, repl):
    src = open(SRC).read()
    assert src.count(find) == 1, f"{name}: pattern must occur exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(find, repl))
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", *obuild.CFLAGS, str(path), "-o", str(lib), "-lm"], check=True)
    return str(lib)


def _pin_golden():
    cases = json.load(open(os.path.join(HERE, "golden", "two_cell.json")))["cases"]
    from tests.test_oracle_exact import test_hand_derived_two_cell_steps
    for c in cases:
        test_hand_derived_two_cell_steps(c)


def _pin_modes():
    from tests.test_oracle_modes import test_mode_amplification_matches_closed_form
    test_mode_amplification_matches_closed_form()


def _pin_exact():
    rng = np.random.Generator(np.random.PCG64(77))
    from tests.test_oracle_exact import _compare
    for _ in range(6):
        m = (rng.uniform(size=(3, 4)) < 0.8).astype(np.uint8)
        _compare(rng, 6, 5, m, steps=3)


def _pin_volume():
    from tests.test_oracle_invariants import test_volume_is_conserved_in_a_closed_basin
    test_volume_is_conserved_in_a_closed_basin()


def _pin_variants():
    from tests import test_oracle_variants as tv
    tv.test_friction_is_the_closed_form_on_a_level_surface()
    tv.test_friction_divides_the_predictor_by_the_old_speed()
    for k, l in ((1, 0), (2, 3)):
        tv.test_velocity_filter_modes_decay_by_the_closed_form(k, l)
    tv.test_velocity_filter_conserves_the_face_sum_and_follows_the_surface_update()
    for a in (0.03, -0.05):
        tv.test_advection_of_linear_profiles_is_exact(a)
    tv.test_advection_keeps_mirror_and_transpose_symmetry()


def _pin_wetdry():
    from tests import test_oracle_wetdry as tw
    tw.test_flooding_step_by_hand()
    tw.test_dry_cell_standing_higher_shuts_the_face()
    tw.test_dry_cell_drained_by_its_old_velocity()
    tw.test_filter_next_to_a_dry_cell()
    tw.test_lake_at_rest_over_rising_ground_is_bitwise_still()
    tw.test_equals_the_plain_step_while_every_cell_stays_wet()
    tw.test_volume_is_conserved_through_flooding_and_drying()
    tw.test_mirror_and_transpose_symmetry()
    tw.test_dam_break_onto_a_dry_bed_follows_ritter()


PINS = (_pin_golden, _pin_modes, _pin_exact, _pin_volume, _pin_variants, _pin_wetdry)


def test_unmutated_oracle_passes_every_pin():
    for pin in PINS:
        pin()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_is_caught(tmp_path, name):
    lib = _build_mutant(tmp_path, name, *MUTANTS[name])
    caught = []
    with sw2d_ref.library(lib):
        for pin in PINS:
            try:
                pin()
            except (AssertionError, sw2d_ref.DryCellError):
                caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
