"""The oracle pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU),
builds it, routes the oracle through it and checks that at least one pin
fails.  A pin set that passes a broken oracle proves nothing.
"""
import subprocess

import pytest

import oracle
import test_oracle_cg as cg_pins
import test_oracle_heat as heat_pins

HEAT_PINS = [
    lambda: heat_pins.test_single_sine_mode_decays_by_exact_factor((13, 9, 7), (2, 3, 1), 0.16, 15),
    lambda: heat_pins.test_random_field_matches_dst_exact_solution((13, 10, 8), 0.12, 30, 11),
    heat_pins.test_dense_matrix_power_brute_force,
    heat_pins.test_dirichlet_layer_never_written_and_steps_compose_exactly,
]
CG_PINS = [
    cg_pins.test_operator_matches_sparse_kronecker_sum,
    cg_pins.test_cg_matches_dense_direct_solve,
    lambda: cg_pins.test_finite_termination_in_m_iterations(3),
    cg_pins.test_errors_decrease_monotonically_in_a_norm_and_2_norm,
]

MUTATIONS = {
    "dropped_neighbour_weight": ("const double lap = nsum - 6.0 * c;", "const double lap = nsum - 4.0 * c;", HEAT_PINS),
    "sign_of_update": ("un[p] = c + r * lap;", "un[p] = c - r * lap;", HEAT_PINS),
    "x_stride_for_y": ("((u[p - sx] + u[p + sx]) +", "((u[p - sy] + u[p + sx]) +", HEAT_PINS),
    "skipped_last_row": ("for (long j = 1; j < ny - 1; ++j)\n            for (long i = 1; i < nx - 1; ++i) {\n                const long p = IDX(i, j, k, nx, ny);\n                const double c = u[p];",
                         "for (long j = 1; j < ny - 2; ++j)\n            for (long i = 1; i < nx - 1; ++i) {\n                const long p = IDX(i, j, k, nx, ny);\n                const double c = u[p];", HEAT_PINS),
    "operator_sign": ("y[p] = 6.0 * x[p] - nsum;", "y[p] = 6.0 * x[p] + nsum;", CG_PINS),
    "operator_z_neighbour": ("const double zp = (k < nz - 1) ? x[p + sz] : 0.0;", "const double zp = (k < nz - 1) ? x[p + sy] : 0.0;", CG_PINS),
    "alpha_inverted": ("const double alpha = rho / pq;", "const double alpha = pq / rho;", CG_PINS),
    "beta_inverted": ("const double beta = rho_new / rho;", "const double beta = rho / rho_new;", CG_PINS),
    "residual_sign": ("r[t] = r[t] - alpha * q[t];", "r[t] = r[t] + alpha * q[t];", CG_PINS),
    "direction_drops_beta": ("p[t] = r[t] + beta * p[t];", "p[t] = r[t] + beta * r[t];", CG_PINS),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new, pins = MUTATIONS[name]
    src = open(oracle.source_path()).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                    str(mutated), "-o", str(lib), "-lm"], check=True)
    caught = 0
    with oracle.using_library(str(lib)):
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught += 1
    assert caught >= 1, "no pin caught the planted mistake " + name
