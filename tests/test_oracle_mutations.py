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
import test_oracle_ir as ir_pins
import test_oracle_precision as prec_pins
import test_oracle_sr as sr_pins
import test_oracle_vk as vk_pins

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

PREC_PINS = [
    prec_pins.test_bf16_rounding_matches_exact_ties_to_even,
    prec_pins.test_bf16_step_is_exact_when_the_result_is_representable,
    lambda: prec_pins.test_f32_step_error_against_f64_oracle_within_bound(7),
    prec_pins.test_f32_sine_mode_decays_within_single_precision,
    prec_pins.test_bf16_error_against_f64_within_bound_and_stagnation,
]

OFFSET_PINS = [
    prec_pins.test_bf16_offset_with_zero_base_is_the_bf16_step,
    prec_pins.test_bf16_offset_keeps_the_increments_nearest_rounding_drops,
]

SR_PINS = [
    sr_pins.test_philox_known_answer_vectors,
    sr_pins.test_rounding_is_exactly_unbiased_over_all_random_bits,
    sr_pins.test_step_brackets_the_binary32_step_and_rounds_up_at_the_right_rate,
    sr_pins.test_steps_compose_and_depend_on_the_seed,
    sr_pins.test_stochastic_rounding_removes_the_stagnation,
    sr_pins.test_slab_with_node_offset_equals_the_whole_array,
]

IR_PINS = [
    ir_pins.test_f32_operator_exact_on_small_integers_and_bounded_otherwise,
    ir_pins.test_f32_dot_is_nearly_exact,
    ir_pins.test_refined_solution_meets_the_condition_number_bound,
    ir_pins.test_first_inner_solve_terminates_in_m_iterations,
    ir_pins.test_refinement_converges_in_few_steps_near_the_f64_iteration_count,
]

VK_PINS = [
    lambda: vk_pins.test_step_matches_sparse_divergence_operator((9, 7, 6), 1),
    lambda: vk_pins.test_exact_closed_form_on_linear_fields((2, -3, 5)),
    vk_pins.test_operator_converges_to_the_continuous_divergence_at_second_order,
    vk_pins.test_constant_coefficient_is_the_seven_point_step,
    vk_pins.test_source_only_cases_are_exact,
    vk_pins.test_operator_is_symmetric_on_fields_vanishing_on_the_boundary,
    vk_pins.test_steps_compose_and_dirichlet_layer_is_never_written,
    vk_pins.test_f32_step_against_f64_within_rounding_and_exact_on_integers,
]

MUTATIONS = {
    "vk_face_single_node": ("const double dx = (kc + kap[p + sx]) * (u[p + sx] - c) -",
                            "const double dx = (kc + kc) * (u[p + sx] - c) -", VK_PINS),
    "vk_source_dropped": ("const double lop = (dx + dy) + dz;\n                un[p] = (c + rhs[p]) + beta * lop;",
                          "const double lop = (dx + dy) + dz;\n                un[p] = c + beta * lop;", VK_PINS),
    "vk_z_face_uses_y_stride": ("(kap[p - sz] + kc) * (c - u[p - sz]);\n                const double lop",
                                "(kap[p - sy] + kc) * (c - u[p - sz]);\n                const double lop", VK_PINS),
    "vk_dy_sign": ("const double lop = (dx + dy) + dz;", "const double lop = (dx - dy) + dz;", VK_PINS),
    "vk_kappa_rhs_swapped": ("oracle_heat_vk_sweep_f64(a, kap, rhs, b, nx, ny, nz, beta);",
                             "oracle_heat_vk_sweep_f64(a, rhs, kap, b, nx, ny, nz, beta);", VK_PINS),
    "vk_f32_beta_sign": ("const float lop = (dx + dy) + dz;\n                un[p] = (c + rhs[p]) + beta * lop;",
                         "const float lop = (dx + dy) + dz;\n                un[p] = (c + rhs[p]) - beta * lop;", VK_PINS),
    "vk_f32_x_face_index": ("const float dx = (kc + kap[p + sx])", "const float dx = (kc + kap[p - sx])", VK_PINS),
    "ir_update_sign": ("x[t] = x[t] + (double)d[t];", "x[t] = x[t] - (double)d[t];", IR_PINS),
    "ir_alpha_inverted": ("const float alpha = (float)(rho / pq);", "const float alpha = (float)(pq / rho);", IR_PINS),
    "ir_f32_operator_y_for_z": ("const float zp = (k < nz - 1) ? x[p + sz] : 0.0f;",
                                "const float zp = (k < nz - 1) ? x[p + sy] : 0.0f;", IR_PINS),
    "ir_f32_dot_squares_a": ("neumaier_add(&s, &c, (double)pa[q] * (double)pb[q]);",
                             "neumaier_add(&s, &c, (double)pa[q] * (double)pa[q]);", IR_PINS),
    "ir_inner_direction_drops_beta": ("p[t] = s[t] + beta * p[t];", "p[t] = s[t] + beta * s[t];", IR_PINS),
    "philox_multiplier": ("(uint64_t)0xD2511F53u * c[0]", "(uint64_t)0xD2511F55u * c[0]", SR_PINS),
    "philox_key_schedule": ("k[1] += 0xBB67AE85u;", "k[1] += 0x9E3779B9u;", SR_PINS),
    "philox_word_swap": ("const uint32_t n2 = hi0 ^ c[3] ^ k[1];", "const uint32_t n2 = hi0 ^ c[1] ^ k[1];", SR_PINS),
    "sr_off_by_one": ("lower + rho >= 0x10000u", "lower + rho > 0x10000u", SR_PINS),
    "sr_counter_frozen": ("step0 + (uint64_t)s, node0);", "step0, node0);", SR_PINS),
    "sr_node_offset_dropped": ("oracle_sr_bits(node0 + (uint64_t)p, t, seed)", "oracle_sr_bits((uint64_t)p, t, seed)", SR_PINS),
    "sr_uses_nearest": ("un[p] = oracle_bf16_sr_from_f32(c + r * lap,\n                                                oracle_sr_bits(node0 + (uint64_t)p, t, seed));",
                        "un[p] = oracle_bf16_from_f32(c + r * lap);", SR_PINS),
    "bf16_ties_away": ("if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u)))", "if (lower >= 0x8000u)", PREC_PINS),
    "bf16_truncates": ("out = upper + 1u;", "out = upper;", PREC_PINS),
    "f32_dropped_weight": ("const float lap = nsum - 6.0f * c;\n                un[p] = c + r * lap;",
                           "const float lap = nsum - 5.0f * c;\n                un[p] = c + r * lap;", PREC_PINS),
    "offset_base_not_subtracted": ("dn[p] = oracle_bf16_from_f32(un - oracle_f32_from_bf16(base[p]));",
                                   "dn[p] = oracle_bf16_from_f32(un);", OFFSET_PINS),
    "offset_value_without_base": ("return oracle_f32_from_bf16(base[p]) + oracle_f32_from_bf16(delta[p]);",
                                  "return oracle_f32_from_bf16(delta[p]);", OFFSET_PINS),
    "bf16_step_sign": ("un[p] = oracle_bf16_from_f32(c + r * lap);", "un[p] = oracle_bf16_from_f32(c - r * lap);", PREC_PINS),
    "dropped_neighbour_weight": ("const double lap = nsum - 6.0 * c;", "const double lap = nsum - 4.0 * c;", HEAT_PINS),
    "sign_of_update": ("const double lap = nsum - 6.0 * c;\n                un[p] = c + r * lap;",
                       "const double lap = nsum - 6.0 * c;\n                un[p] = c - r * lap;", HEAT_PINS),
    "x_stride_for_y": ("const double nsum = ((u[p - sx] + u[p + sx]) +",
                       "const double nsum = ((u[p - sy] + u[p + sx]) +", HEAT_PINS),
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
