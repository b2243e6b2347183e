"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch each one.  The mutated source is compiled to a temporary library and
swapped in for the duration of one pin; the committed oracle is untouched.
"""
import contextlib

import pytest

import oracle
from tests import test_oracle_amg as ta
from tests import test_oracle_cpr_conv as tc
from tests import test_oracle_krylov as tk
from tests import test_oracle_linalg as tl
from tests import test_oracle_precision as tp
from tests import test_oracle_ras as tr

# (name, exact text in oracle.c, replacement, pins expected to fail)
MUTANTS = [
    ("spmv_transposed_block",
     "for (int c = 0; c < bs; c++) t += blk[r * bs + c] * xj[c];\n            }\n            y[(size_t)i * bs + r] = t;",
     "for (int c = 0; c < bs; c++) t += blk[c * bs + r] * xj[c];\n            }\n            y[(size_t)i * bs + r] = t;",
     [lambda: tl.test_spmv_matches_dense(1)]),
    ("spmv_dropped_last_term",
     "for (int p = rp[i]; p < rp[i + 1]; p++) {\n                const double *blk = a + (size_t)p * bs * bs;\n                const double *xj = x + (size_t)ci[p] * bs;\n                for (int c = 0; c < bs; c++) t += blk[r * bs + c] * xj[c];\n            }\n            y[(size_t)i * bs + r] = t;",
     "for (int p = rp[i]; p < rp[i + 1] - 1; p++) {\n                const double *blk = a + (size_t)p * bs * bs;\n                const double *xj = x + (size_t)ci[p] * bs;\n                for (int c = 0; c < bs; c++) t += blk[r * bs + c] * xj[c];\n            }\n            y[(size_t)i * bs + r] = t;",
     [lambda: tl.test_spmv_matches_dense(0)]),
    ("ilu_update_sign",
     "for (int e = 0; e < b2; e++) lu[(size_t)s * b2 + e] -= tmp[e];",
     "for (int e = 0; e < b2; e++) lu[(size_t)s * b2 + e] += tmp[e];",
     [lambda: tl.test_ilu_product_equals_a_on_pattern(0),
      lambda: tl.test_ilu_exact_on_tridiagonal(1)]),
    ("ilu_multiplier_order",
     "blk_mm(bs, lu + (size_t)p * b2, inv, tmp);",
     "blk_mm(bs, inv, lu + (size_t)p * b2, tmp);",
     [lambda: tl.test_ilu_product_equals_a_on_pattern(1)]),
    ("lower_solve_skips_dependencies",
     "for (int p = rp[i]; p < rp[i + 1] && ci[p] < i; p++)\n            blk_sub_mv(",
     "for (int p = rp[i]; p < rp[i + 1] && ci[p] < i - 1; p++)\n            blk_sub_mv(",
     [lambda: tl.test_triangular_solves_match_dense(1)]),
    ("givens_sign",
     "g[j + 1] = -sn[j] * g[j];",
     "g[j + 1] = sn[j] * g[j];",
     [lambda: tk.test_gmres_estimate_equals_true_residual_right_preconditioned()]),
    ("mgs_sign",
     "for (size_t i = 0; i < n; i++) w[i] -= h * V[n * k + i];",
     "for (size_t i = 0; i < n; i++) w[i] += h * V[n * k + i];",
     [lambda: tk.test_solution_matches_dense_solve("gmres")]),
    ("bicgstab_omega_sign",
     "omega = tt != 0.0 ? ts / tt : 0.0;",
     "omega = tt != 0.0 ? -ts / tt : 0.0;",
     [lambda: tk.test_solution_matches_dense_solve("bicgstab")]),
    ("bicgstab_beta_inverted",
     "double beta = (rho / rho0) * (alpha / omega);",
     "double beta = (rho0 / rho) * (alpha / omega);",
     [lambda: tk.test_solution_matches_dense_solve("bicgstab")]),
    ("fgmres_updates_with_v",
     "for (size_t i = 0; i < n; i++) x[i] += y[k] * Z[n * k + i];",
     "for (size_t i = 0; i < n; i++) x[i] += y[k] * V[n * k + i];",
     [lambda: tk.test_fgmres_equals_right_gmres_with_fixed_preconditioner()]),
    ("qimpes_weight_sign",
     "w[3 * i + 1] = -y[0];",
     "w[3 * i + 1] = y[0];",
     [lambda: tc.test_quasi_impes_weights_zero_secondary_columns()]),
    ("cpr_pressure_uses_wrong_column",
     "app[p] = w[3 * i] * B[0] + w[3 * i + 1] * B[3] + w[3 * i + 2] * B[6];",
     "app[p] = w[3 * i] * B[0] + w[3 * i + 1] * B[1] + w[3 * i + 2] * B[2];",
     [lambda: tc.test_pressure_matrix_is_decoupled_operator_on_pressure_vectors()]),
    ("cpr_pf_second_stage_on_v",
     "or_bsr_amxpby(nb, 3, pc->rp, pc->ci, pc->a, -1.0, z, 1.0, r);\n            full_solve_f64(pc, r, t);",
     "full_solve_f64(pc, r, t);",
     [lambda: tc.test_cpr_exact_when_stages_are_exact("cpr_pf")]),
    ("cpr_ffpf_skips_second_full_stage",
     "if (pc->kind == OR_PC_CPR_FFPF) {\n        cpr_resid_f64(pc, f, x, r);",
     "if (0) {\n        cpr_resid_f64(pc, f, x, r);",
     [lambda: tc.test_cpr_error_propagator_is_product_of_stage_propagators("cpr_ffpf", 1)]),
    ("cpr_fpf_last_stage_on_f",
     "    cpr_resid_f64(pc, f, x, r);                   /* r = f - A x       */\n    cpr_full_f64(pc, r, x);                       /* x = x + R^-1 r    */\n    free(r);",
     "    cpr_full_f64(pc, f, x);\n    free(r);",
     [lambda: tc.test_cpr_exact_when_stages_are_exact("cpr_fpf"),
      lambda: tc.test_cpr_error_propagator_is_product_of_stage_propagators("cpr_fpf", 1)]),
    ("cpr_multistage_pressure_ignores_weights",
     "        rpv[i] = pc->w[3 * i] * r[3 * i] + pc->w[3 * i + 1] * r[3 * i + 1]\n               + pc->w[3 * i + 2] * r[3 * i + 2];\n    pstage_f64(pc, rpv, p);\n    for (int i = 0; i < nb; i++) x[3 * i] += p[i];",
     "        rpv[i] = r[3 * i];\n    pstage_f64(pc, rpv, p);\n    for (int i = 0; i < nb; i++) x[3 * i] += p[i];",
     [lambda: tc.test_cpr_error_propagator_is_product_of_stage_propagators("cpr_fpf", 3)]),
    ("pcg_beta_inverted",
     "const double beta = rho / rho_prev;",
     "const double beta = rho_prev / rho;",
     [lambda: tk.test_pcg_iterates_minimize_energy_error_over_krylov_space()]),
    ("pcg_alpha_on_rr",
     "const double alpha = rho / pq;",
     "const double alpha = dot((int)n, r, r) / pq;",
     [lambda: tk.test_pcg_iterates_minimize_energy_error_over_krylov_space()]),
    ("lgmres_skips_stored_corrections",
     "const int steps = m + nstored;",
     "const int steps = m + 0 * nstored;",
     [lambda: tk.test_lgmres_cycles_minimize_over_augmented_space(1)]),
    ("lgmres_stores_iterate_not_correction",
     "for (size_t i = 0; i < n; i++) Zs[i] = dx[i] / dn;",
     "for (size_t i = 0; i < n; i++) Zs[i] = x[i] / dn;",
     [lambda: tk.test_lgmres_cycles_minimize_over_augmented_space(2)]),
    ("ras_prolongs_overlap_rows",
     "if (pc->part[g] == S->s)",
     "if (g >= 0)",
     [lambda: tr.test_ras_matches_dense_restricted_schwarz([0, 12, 24, 36], 1)]),
    ("ras_overlap_not_grown",
     "for (int d = 0; d < overlap; d++) {",
     "for (int d = 0; d < 0 * overlap; d++) {",
     [lambda: tr.test_ras_matches_dense_restricted_schwarz([0, 5, 23, 36], 2)]),
    ("gelu_grad_missing_density_term",
     "return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * pi);",
     "return 0.5 * (1.0 + erf(x / sqrt(2.0)));",
     [lambda: tc.test_conv_finite_differences()]),
    ("conv_input_grad_tap_flip",
     "int kk = k - dzz, jj = j - dy, ii = i - dx;",
     "int kk = k + dzz, jj = j + dy, ii = i + dx;",
     [lambda: tc.test_conv_finite_differences()]),
    ("conv_cross_correlation_as_convolution",
     "int kk = k + dz, jj = j + dy, ii = i + dx;\n                                    if (kk < 0",
     "int kk = k - dz, jj = j - dy, ii = i - dx;\n                                    if (kk < 0",
     [lambda: tc.test_conv_finite_differences()]),
    ("adam_no_bias_correction",
     "double mh = m[i] / c1, vh = v[i] / c2;",
     "double mh = m[i], vh = v[i];",
     [lambda: tc.test_adam_first_step_closed_form()]),
    ("bf16_truncation",
     "u += 0x7fffu + ((u >> 16) & 1u);",
     "u += 0u;",
     [lambda: tl.test_bf16_rounding_closed_forms()]),
    ("learned_accepts_ties",
     "if (n2 < n1) accept = 1;",
     "if (n2 <= n1) accept = 1;",
     [lambda: tc.test_learned_stage_zero_net_falls_back_bit_exactly()]),
    ("amg_row_sum_rule_ignored",
     "const int dependent = !(max_row_sum < 1.0 && fabs(rsum) > max_row_sum * fabs(diag));",
     "const int dependent = 1;",
     [lambda: ta.test_strength_hand_example()]),
    ("amg_strength_sign",
     "if (ci[q] != i && -s * a[q] >= theta * mx) sci[m++] = ci[q];",
     "if (ci[q] != i && -a[q] >= theta * mx) sci[m++] = ci[q];",
     [lambda: ta.test_strength_hand_example()]),
    ("amg_no_second_pass",
     "        if (cf[i] != FPT) continue;\n        for (int q = srp[i]; q < srp[i + 1]; q++)\n            if (cf[sci[q]] == CPT) mark[sci[q]] = i;",
     "        continue;\n        for (int q = srp[i]; q < srp[i + 1]; q++)\n            if (cf[sci[q]] == CPT) mark[sci[q]] = i;",
     [lambda: ta.test_splitting_invariants((8, 7, 6), 2),
      lambda: ta.test_splitting_invariants((10, 9, 5), 3)]),
    ("amg_weak_not_lumped",
     "diag += a[q];                    /* weak: lumped */",
     "(void)0;                         /* weak: lumped */",
     [lambda: ta.test_interpolation_keeps_constants_on_zero_row_sums()]),
    ("amg_distribution_sign",
     "num[pos[mm]] += a[q] * a[p] / den;",
     "num[pos[mm]] -= a[q] * a[p] / den;",
     [lambda: ta.test_interpolation_keeps_constants_on_zero_row_sums()]),
    ("amg_truncation_not_rescaled",
     "const double scale = sum_kept != 0.0 ? sum_all / sum_kept : 1.0;",
     "const double scale = 1.0;",
     [lambda: ta.test_truncation_drops_small_weights_and_keeps_row_sums()]),
    ("amg_weight_sign",
     "num[t] = -num[t] / diag;",
     "num[t] = num[t] / diag;",
     [lambda: ta.test_chain_splitting_interpolation_and_galerkin(),
      lambda: ta.test_vcycle_converges_on_poisson(0)]),
    ("amg_transpose_values",
     "if (v) tv[p] = v[q];",
     "if (v) tv[p] = v[p];",
     [lambda: ta.test_galerkin_coarse_matrices()]),
    ("amg_gs_reads_old_inside_chunk",
     "else if (j >= c0 && j < i) s -= L->a[q] * xn[j];",
     "else if (j >= c0 && j < i) s -= L->a[q] * xo[j];",
     [lambda: ta.test_vcycle_matches_dense_algorithm4(4, 2)]),
    ("amg_no_post_smoothing",
     "    amg_smooth(M, L);                                     /* x = T(x, A, b) */",
     "    (void)0;                                              /* x = T(x, A, b) */",
     [lambda: ta.test_vcycle_matches_dense_algorithm4(0, 2)]),
    ("cpr_full_stage_ignored",
     "    if (pc->full) or_pc_apply(pc->full, r, t);",
     "    if (0) or_pc_apply(pc->full, r, t);",
     [lambda: tr.test_cpr_with_ras_full_stage_converges()]),
    ("amg_coarse_correction_sign",
     "        L->x[i] += s;",
     "        L->x[i] -= s;",
     [lambda: ta.test_vcycle_matches_dense_algorithm4(0, 2),
      lambda: ta.test_vcycle_converges_on_poisson(0)]),
    # reduced-precision emulation (mixed-precision extension)
    ("lowp_forward_double_accumulator",
     "                float s = 0.0f;\n                for (int c = 0; c < bs; c++) s += blk[r * bs + c] * yk[c];\n                t[r] -= s;",
     "                double s = 0.0;\n                for (int c = 0; c < bs; c++) s += (double)blk[r * bs + c] * yk[c];\n                t[r] = (float)((double)t[r] - s);",
     [lambda: tp.test_forward_sweep_accumulates_in_float()]),
    ("lowp_backward_double_accumulator",
     "                float s = 0.0f;\n                for (int c = 0; c < bs; c++) s += blk[r * bs + c] * xj[c];\n                t[r] -= s;",
     "                double s = 0.0;\n                for (int c = 0; c < bs; c++) s += (double)blk[r * bs + c] * xj[c];\n                t[r] = (float)((double)t[r] - s);",
     [lambda: tp.test_backward_sweep_accumulates_in_float()]),
    ("pstage_f32_double_residual",
     "            float t = 0.0f;\n            for (int q = pc->rp[i]; q < pc->rp[i + 1]; q++) t += pc->appf[q] * p[pc->ci[q]];\n            res[i] = rpv[i] - t;",
     "            double t = 0.0;\n            for (int q = pc->rp[i]; q < pc->rp[i + 1]; q++) t += (double)pc->appf[q] * p[pc->ci[q]];\n            res[i] = (float)((double)rpv[i] - t);",
     [lambda: tp.test_cpr_pf_pressure_stage_in_float()]),
    ("bf16_variant_rounds_diagonal_inverse",
     "for (int e = 0; e < b2; e++) L->f[(size_t)p * b2 + e] = (float)inv[e];",
     "for (int e = 0; e < b2; e++) L->f[(size_t)p * b2 + e] = (prec == OR_PREC_BF16) ? or_bf16_round((float)inv[e]) : (float)inv[e];",
     [lambda: tp.test_diagonal_inverse_kept_in_float_for_bf16_factors()]),
    ("bf16_variant_keeps_float_off_diagonals",
     "L->f[(size_t)p * b2 + e] = (prec == OR_PREC_BF16) ? or_bf16_round(v) : v;",
     "L->f[(size_t)p * b2 + e] = v;",
     [lambda: tp.test_forward_sweep_accumulates_in_float(),
      lambda: tp.test_bf16_rounds_off_diagonal_blocks_of_3x3_factors()]),
    ("conv_bf16_activations_not_rounded",
     "round_copy(cells * cout, act, h[l + 1], bf16);",
     "round_copy(cells * cout, act, h[l + 1], 0);",
     [lambda: tp.test_conv_bf16_emulation_rounds_input_and_activations()]),
    ("conv_bf16_input_not_rounded",
     "round_copy(cells * CONV_C[0], in, h[0], bf16);",
     "round_copy(cells * CONV_C[0], in, h[0], 0);",
     [lambda: tp.test_conv_bf16_emulation_rounds_input_and_activations()]),
    ("conv_bf16_weights_not_rounded",
     "round_copy(nw, pp, W, bf16);",
     "round_copy(nw, pp, W, 0);",
     [lambda: tp.test_conv_bf16_emulation_rounds_weights()]),

]


@contextlib.contextmanager
def _swapped(lib):
    saved = oracle._lib
    oracle._lib = lib
    try:
        yield
    finally:
        oracle._lib = saved


def test_mutant_texts_present():
    src = oracle.source()
    for name, old, new, _ in MUTANTS:
        assert src.count(old) >= 1, name


@pytest.mark.parametrize("mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(mut, tmp_path):
    name, old, new, pins = mut
    src = oracle.source()
    assert old in src
    so = oracle.compile_variant(src.replace(old, new, 1), str(tmp_path / f"lib_{name}.so"))
    lib = oracle.load(so)
    caught = 0
    with _swapped(lib):
        for pin in pins:
            try:
                pin()
            except (AssertionError, RuntimeError):
                caught += 1
    assert caught >= 1, f"no pin caught mutant {name}"
