"""Plant a plausible mistake in a copy of the oracle source (on the CPU) and check that the
pins of ``oracle_pins.py`` catch it.  Shows that the pins constrain every stage of the
step: equilibrium, forcing, velocity, viscosity, colour gradient, stress, segregation law,
recolouring, streaming and the lattice tables."""
import os

import pytest

import oracle
import oracle_pins as P

MUTANTS = {
    "equilibrium_coefficient": ("eu * eu * INV_2CS4", "eu * eu * INV_CS2"),
    "no_half_force_velocity": ("double ux = (mx + 0.5 * Fx) / rho;", "double ux = mx / rho;"),
    "guo_prefactor": ("(1.0 - 1.0 / (2.0 * tau))", "(1.0 - 1.0 / tau)"),
    "viscosity_arithmetic_mean": ("s += rho[k] / nu_k;", "s += rho[k] * nu_k / (r * r);"),
    "collision_fixed_tau": ("double omega = -(f[i] - feq[i]) / tau;",
                            "double omega = -(f[i] - feq[i]) / p->tau[0];"),
    "colour_gradient_sign_x": ("G[0] = c[l] * gx[k] - c[k] * gx[l];",
                               "G[0] = c[k] * gx[l] - c[l] * gx[k];"),
    "stress_double_counted": ("double a = 0.5 * sigma_of(p, k, l)", "double a = sigma_of(p, k, l)"),
    "stress_normal_projector": ("S[3] += a * (1.0 - n[1] * n[1]);", "S[3] += a * (n[1] * n[1]);"),
    "concentration_factor_scale": ("double v = 1e6 * rho_k[k]", "double v = 1e-6 * rho_k[k]"),
    "concentration_factor_scale_1e4": ("double v = 1e6 * rho_k[k]", "double v = 1e4 * rho_k[k]"),
    "segregation_ct_coefficient_27": (
        "double ct = 35.0 * rho[0] * rho[1] * rho[2] / (r * r * r);\n    if (ct > 1.0) ct = 1.0;\n"
        "    return p->beta0 + p->beta0 * ct * oracle_g",
        "double ct = 27.0 * rho[0] * rho[1] * rho[2] / (r * r * r);\n    if (ct > 1.0) ct = 1.0;\n"
        "    return p->beta0 + p->beta0 * ct * oracle_g"),
    "segregation_ct_not_capped": (
        "    if (ct > 1.0) ct = 1.0;\n    return p->beta0 + p->beta0 * ct * oracle_g",
        "    return p->beta0 + p->beta0 * ct * oracle_g"),
    "leclaire_ct_coefficient_27": (
        "double ct = 35.0 * rho[0] * rho[1] * rho[2] / (r * r * r);\n    if (ct > 1.0) ct = 1.0;\n"
        "    return p->beta0 + p->beta0 * ct * (sin(",
        "double ct = 27.0 * rho[0] * rho[1] * rho[2] / (r * r * r);\n    if (ct > 1.0) ct = 1.0;\n"
        "    return p->beta0 + p->beta0 * ct * (sin("),
    "perturbation_A_coefficient": ("double A = 9.0 * sigma_of(p, k, l) / (2.0 * tau);",
                                   "double A = 9.0 * sigma_of(p, k, l) / tau;"),
    "perturbation_B_rest": ("{-4.0 / 27.0, 2.0 / 27.0", "{-2.0 / 27.0, 2.0 / 27.0"),
    "spencer_factor_35": ("double s = 27.0 * rho[0]", "double s = 35.0 * rho[0]"),
    "segregation_branch_sign": ("if (X < 0.0) return 1.0 - sin(acos(X));",
                                "if (X < 0.0) return sin(acos(X)) - 1.0;"),
    "neumann_opposite_side": ("return (smk * smk + sml * sml - skl * skl) / (2.0 * smk * sml);",
                              "return (smk * smk + skl * skl - sml * sml) / (2.0 * smk * skl);"),
    "recolour_transposed_direction": ("(n[0] * EX[i] + n[1] * EY[i])", "(n[0] * EY[i] + n[1] * EX[i])"),
    "recolour_wrong_colour_share": ("out[k * 9 + i] = c[k] * fdag[i];",
                                    "out[k * 9 + i] = c[(k + 1) % 3] * fdag[i];"),
    "gradient_transposed": ("sy += W[i] * EY[i] * (fwd - bwd);", "sy += W[i] * EX[i] * (fwd - bwd);"),
    "gradient_one_sided": ("sx += W[i] * EX[i] * (fwd - bwd);", "sx += W[i] * EX[i] * fwd;"),
    "streaming_backwards": ("size_t d = (size_t)wrap(y + EY[i], ny) * nx + wrap(x + EX[i], nx);",
                            "size_t d = (size_t)wrap(y - EY[i], ny) * nx + wrap(x - EX[i], nx);"),
    "lattice_diagonal_swap": ("static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};",
                              "static const int EY[9] = {0, 0, 1, 0, -1, 1, -1, -1, 1};"),
    "force_divergence_component": ("oracle_gradient(nx, ny, w->S + 2 * N, dx, dy); /* S_yx */",
                                   "oracle_gradient(nx, ny, w->S + 3 * N, dx, dy); /* S_yx */"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"pattern for {name} must occur exactly once"
    so = oracle.compile_source(src.replace(old, new), os.path.join(tmp_path, f"mut_{name}.so"))
    caught = None
    with oracle.use_library(so):
        for pin in P.FAST_PINS:
            try:
                pin()
            except (AssertionError, FloatingPointError, ValueError, RuntimeError) as e:
                caught = (pin.__name__, e)
                break
    assert caught is not None, f"no pin catches the planted mistake {name}"
