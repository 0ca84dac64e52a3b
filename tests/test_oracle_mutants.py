"""The pins must catch plausible mistakes in the oracle.  Each case copies
the oracle, plants one mistake in its C source (a dropped term, a wrong
sign, factor, index, constant or branch), rebuilds the copy with gcc and
runs the pins aimed at that part of the method: at least one of them must
fail.  Nothing here touches the GPU path; the planted mistakes live only in
the temporary copy."""
import importlib.util
import os
import shutil
import sys

import pytest

import test_oracle_adjoint as TA
import test_oracle_beads as TB
import test_oracle_collision as TC
import test_oracle_dynamics as TD
import test_oracle_kg as TK
import test_oracle_lattice as TL
import test_oracle_rng as TR
import test_oracle_vacf as TV
import test_oracle_walls as TW
from test_oracle_rng import rocrand_ref  # noqa: F401  (fixture)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# name: (text in lb_oracle.c, replacement, pins as (function, keyword arguments))
MUTANTS = {
    "vacf_phase_sign": ("out[1] -= j[0] * sin(fz);", "out[1] += j[0] * sin(fz);",
                        [(TV.test_transverse_modes_match_fft, {}), (TV.test_transverse_modes_shear_wave_and_uniform_flow, {})]),
    "vacf_axis_extent": ("const double fy = two_pi * (double)y / (double)p->ny;",
                         "const double fy = two_pi * (double)y / (double)p->nx;",
                         [(TV.test_transverse_modes_match_fft, {})]),
    "philox_multiplier": ("M0 = 0xD2511F53u", "M0 = 0xD2511F57u", [(TR.test_philox_matches_rocrand, "rocrand")]),
    "philox_key_bump": ("k1 += W1;", "k1 += W0;", [(TR.test_philox_matches_rocrand, "rocrand")]),
    "box_muller_angle": ("*g1 = r * sin(TWO_PI * ub);", "*g1 = r * cos(TWO_PI * ub);",
                         [(TR.test_fluid_normals_distribution, {})]),
    "equilibrium_u2_term": ("- usq / (2.0 * CS2));", "- usq / (3.0 * CS2));",
                            [(TL.test_equilibrium_moments, {}), (TL.test_equilibrium_has_no_kinetic_projection, {})]),
    "back_transform_norm": ("s += E[k][i] * m[k] / WK[k];", "s += E[k][i] * m[k];",
                            [(TL.test_forward_back_inverse, {})]),
    "noise_fdt_factor": ("const double phi = sqrt(1.0 - gam[k] * gam[k]);", "const double phi = sqrt(1.0 - gam[k]);",
                         [(TC.test_noise_enters_each_mode_with_fdt_amplitude, {"noise_rho0": False})]),
    "bulk_eigenvalue": ("gam[4] = p->gamma_bulk;", "gam[4] = p->gamma_shear;",
                        [(TC.test_stress_update_rule_with_force, {}), (TC.test_kinetic_modes_relax_with_own_eigenvalue, {}),
                         (TD.test_linear_dynamics_equal_operator_power, {"name": "general"})]),
    "ghost_group": ("for (int k = 13; k <= 15; ++k) gam[k] = p->gamma_3b;",
                    "for (int k = 13; k <= 15; ++k) gam[k] = p->gamma_3a;",
                    [(TC.test_kinetic_modes_relax_with_own_eigenvalue, {}),
                     (TD.test_linear_dynamics_equal_operator_power, {"name": "general"})]),
    "force_stress_factor": ("sig[a][b] = 0.5 * (1.0 + p->gamma_shear)", "sig[a][b] = 0.5 * (1.0 - p->gamma_shear)",
                            [(TC.test_stress_update_rule_with_force, {})]),
    "half_force_velocity": ("u[a] = (m[1 + a] + 0.5 * F[a]) / rho;", "u[a] = (m[1 + a] + F[a]) / rho;",
                            [(TC.test_stress_update_rule_with_force, {}), (TD.test_kolmogorov_steady_amplitude, {})]),
    "stream_direction": ("wrap(x + CV[i][0], p->nx)", "wrap(x - CV[i][0], p->nx)",
                         [(TD.test_uniform_flow_advects_a_transverse_wave, {"axis": 0})]),
    "wall_crossing": ("return p->walls && (zz < 0 || zz >= p->nz);", "return p->walls && (zz < 0 || zz > p->nz);",
                      [(TW.test_walls_conserve_mass_with_noise, {}), (TW.test_poiseuille_closed_form, {"name": "gamma0"})]),
    "wall_reflection": ("n[opposite(i) * N + s] = work[i * N + s];", "n[i * N + s] = work[i * N + s];",
                        [(TW.test_poiseuille_closed_form, {"name": "gamma0"}), (TW.test_wall_momentum_exchange, {})]),
    "phi3_constant": ("if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;",
                      "if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.1;",
                      [(TB.test_kernel_moment_conditions, {"W": 3})]),
    "dphi4_slope": ("if (a <= 1.0) return sg * (-2.0 + (4.0 - 8.0 * a)", "if (a <= 1.0) return sg * (-1.9 + (4.0 - 8.0 * a)",
                    [(TB.test_kernel_moment_conditions, {"W": 4})]),
    "phi3_first_node": ("if (W == 3) return floor(R + 0.5) - 1.0;", "if (W == 3) return floor(R) - 1.0;",
                        [(TB.test_w_point_stencil, {"W": 3}), (TB.test_wide_stencil_linear_field_interpolated_exactly,
                                                               {"W": 3})]),
    "ou_noise_amplitude": ("*C3 = sqrt(m * kT * (1.0 - exp(-2.0 * z * h / m)));",
                           "*C3 = sqrt(m * kT * (1.0 - exp(-z * h / m)));",
                           [(TB.test_ou_variance_frozen_fluid, {"three_point": False})]),
    "ou_decay": ("*C1 = exp(-z * h / m);", "*C1 = exp(-0.5 * z * h / m);", [(TB.test_ou_mean_decay_frozen_fluid, {})]),
    "three_point_upper_sixth": ("(k == 5) ? sqrt(3.0)", "(k == 4) ? sqrt(3.0)",
                                [(TR.test_bead_three_point_follows_exact_thresholds, {})]),
    "three_point_selected": ("if (bs->three_point)", "if (0)",
                             [(TB.test_ou_variance_frozen_fluid, {"three_point": True})]),
    "impulse_sign": ("I[a] = -(Pn[a] - mom[3 * b + a] - h * fc[3 * b + a]);",
                     "I[a] = (Pn[a] - mom[3 * b + a] - h * fc[3 * b + a]);",
                     [(TB.test_spread_sums_to_impulse_and_total_momentum, {})]),
    "bead_velocity_half_force": ("for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * p->g[a]) / r;",
                                 "for (int a = 0; a < 3; ++a) u[a] = j[a] / r;",
                                 [(TB.test_bead_in_forced_fluid_at_rest_sees_half_the_force, {"W": 2})]),
    "wca_force_sign": ("fc[3 * j + a] += f * d[a];", "fc[3 * j + a] -= f * d[a];",
                       [(TK.test_forces_are_minus_gradients, {})]),
    "bond_force_sign": ("mag = -bs->kbond * (r - bs->r0) / r;", "mag = bs->kbond * (r - bs->r0) / r;",
                        [(TB.test_bond_force_is_gradient, {})]),
    "wca_cutoff": ("pow(2.0, 1.0 / 3.0) * sigma * sigma", "pow(2.0, 1.0 / 6.0) * sigma * sigma",
                   [(TK.test_wca_vanishes_smoothly_at_cutoff, {}), (TK.test_forces_are_minus_gradients, {})]),
    "fene_form": ("-bs->kbond / (1.0 - r2 / R02)", "-bs->kbond / (1.0 - 0.5 * r2 / R02)",
                  [(TK.test_forces_are_minus_gradients, {})]),
    "adjoint_collision_stress": ("const double As = 0.5 * (1.0 + p->gamma_shear);",
                                 "const double As = 0.5 * (1.0 - p->gamma_shear);",
                                 [(TA.test_collision_adjoint_is_transpose_of_jacobian, {})]),
    "adjoint_weight_gradient": ("for (int a = 0; a < 3; ++a) half_bar[3 * b + a] += wgt_bar[q] * dw[3 * q + a];", ";",
                                [(TA.test_couple_adjoint_matches_finite_differences, {})]),
    "adjoint_bond_jacobian": ("mag2p = -bs->kbond * bs->r0 / (r * r * r);", "mag2p = 0.0;",
                              [(TA.test_couple_adjoint_matches_finite_differences, {})]),
    "adjoint_fene_jacobian": ("mag2p = -2.0 * bs->kbond / (bs->r0 * bs->r0 * (1.0 - x) * (1.0 - x));",
                              "mag2p = -bs->kbond / (bs->r0 * bs->r0 * (1.0 - x) * (1.0 - x));",
                              [(TA.test_kg_couple_adjoint_matches_finite_differences, {})]),
    "adjoint_wca_jacobian": ("(-28.0 * s6 * s6 + 8.0 * s6)", "(-28.0 * s6 * s6 + 4.0 * s6)",
                             [(TA.test_kg_couple_adjoint_matches_finite_differences, {})]),
    "adjoint_body_force_half": ("gbar[a] += 0.5 * uq_bar[a] / rn[q];", "gbar[a] += 0.0;",
                                [(TA.test_coupled_backward_matches_finite_differences, {})]),
}


def mutant_oracle(tmp_path, name, old, new):
    d = tmp_path / name
    shutil.copytree(os.path.join(ROOT, "oracle"), d, ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.tmp*"))
    src = (d / "lb_oracle.c").read_text()
    assert src.count(old) >= 1, f"{name}: target text not found"
    (d / "lb_oracle.c").write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", str(d / "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod  # its dataclasses look their module up there
    spec.loader.exec_module(mod)
    mod.build(force=True)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name, rocrand_ref):  # noqa: F811
    old, new, pins = MUTANTS[name]
    orc = mutant_oracle(tmp_path, name, old, new)
    caught = []
    for fn, kw in pins:
        try:
            if kw == "rocrand":
                fn(orc, rocrand_ref)
            else:
                fn(orc, **kw)
        except Exception as e:  # a failed assertion, or a mistake that breaks the run outright
            caught.append(f"{fn.__name__}: {type(e).__name__}")
    print(name, "caught by", caught)
    assert caught, f"no pin caught the planted mistake {name}"
