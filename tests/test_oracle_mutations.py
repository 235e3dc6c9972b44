"""Strength of the oracle pins: plausible mistakes planted in copies of
oracle.c (on the CPU) must each make at least one pin fail."""

import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_shading as shading
import test_oracle_preint as preint
import test_oracle_filters as filters

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "bspline_w1_w2_swapped": (
        "w[1] = (3.0 * f * f * f - 6.0 * f * f + 4.0) / 6.0;\n    w[2] = (-3.0 * f * f * f + 3.0 * f * f + 3.0 * f + 1.0) / 6.0;",
        "w[2] = (3.0 * f * f * f - 6.0 * f * f + 4.0) / 6.0;\n    w[1] = (-3.0 * f * f * f + 3.0 * f * f + 3.0 * f + 1.0) / 6.0;",
    ),
    "bspline_w2_sign": ("w[2] = (-3.0 * f * f * f + 3.0 * f * f", "w[2] = (3.0 * f * f * f + 3.0 * f * f"),
    "bspline_w0_w3_swapped": ("w[0] = g * g * g / 6.0;", "w[0] = f * f * f / 6.0;"),
    "tf_weights_swapped": (
        "out[c] = (1.0 - w) * (double)tf[4 * j + c] + w * (double)tf[4 * (j + 1) + c];",
        "out[c] = w * (double)tf[4 * j + c] + (1.0 - w) * (double)tf[4 * (j + 1) + c];",
    ),
    "opacity_without_step": ("double alpha = -expm1(-val[3] * cx->step);", "double alpha = -expm1(-val[3]);"),
    "sample_at_segment_start": ("double t = ((double)k + 0.5) * cx->step;", "double t = ((double)k) * cx->step;"),
    "camera_axes_transposed": ("d[k] = f[k] + a * r[k] + b * u[k];", "d[k] = f[k] + a * u[k] + b * r[k];"),
    "ert_late": ("if (1.0 - T >= cx->ert) break;", "if (1.0 - T >= cx->ert + 0.05) break;"),
    "adjoint_drops_suffix": ("ds += g[c] * (Tnext * r->val[c] - S[c]);", "ds += g[c] * (Tnext * r->val[c]);"),
    "adjoint_alpha_sign": ("dval[c] = g[c] * r->Tk * r->alpha;", "dval[c] = -g[c] * r->Tk * r->alpha;"),
    "footprint_low_apron_dropped": ("long x0 = or_clampl(bx * edge - 1, 0, nx - 1)", "long x0 = or_clampl(bx * edge, 0, nx - 1)"),
    "occupancy_margin_dropped": ("long jlo = (long)floorf(ulo) - 1, jhi = (long)ceilf(uhi) + 1;",
                                 "long jlo = (long)floorf(ulo), jhi = (long)ceilf(uhi);"),
    "dweight_d1_wrong": ("d[1] = (9.0 * f * f - 12.0 * f) / 6.0;", "d[1] = (9.0 * f * f - 6.0 * f) / 6.0;"),
    "gradient_y_takes_x_derivative": ("g[1] += w[0][a] * dw[1][b] * w[2][c] * V;",
                                      "g[1] += dw[0][a] * w[1][b] * w[2][c] * V;"),
    "light_one_sided": ("double nl = fabs(n[0] * L[0] + n[1] * L[1] + n[2] * L[2]);",
                        "double nl = fmax(n[0] * L[0] + n[1] * L[1] + n[2] * L[2], 0.0);"),
    "specular_dropped": ("c[a] = c[a] * (sh[0] + sh[1] * nl) + sh[2] * spec;", "c[a] = c[a] * (sh[0] + sh[1] * nl);"),
    "normal_not_shrunk": ("double m = gm > sh[8] ? gm : sh[8];", "double m = gm;"),
    "half_vector_not_normalised": ("double nh = fabs(n[0] * Hs[0] + n[1] * Hs[1] + n[2] * Hs[2]) / hn;",
                                   "double nh = fabs(n[0] * Hs[0] + n[1] * Hs[1] + n[2] * Hs[2]);"),
    "preint_tau_quadratic_dropped": ("double t = tau + ea[3] * xs[r] + 0.5 * (eb[3] - ea[3]) * xs[r] * xs[r] / piece;",
                                     "double t = tau + ea[3] * xs[r];"),
    "preint_lookup_front_back_swapped": ("or_preint_lookup(tab, K, (sf.v - v0) * scale, (sb.v - v0) * scale, seg);",
                                         "or_preint_lookup(tab, K, (sb.v - v0) * scale, (sf.v - v0) * scale, seg);"),
    "preint_back_value_at_midpoint": ("double tf_ = (double)k * step, tb = (double)(k + 1) * step;",
                                      "double tf_ = (double)k * step, tb = ((double)k + 0.5) * step;"),
    "preint_skip_front_block_only": (
        "double lo = fmin(minmax[2 * bf], minmax[2 * bb]), hi = fmax(minmax[2 * bf + 1], minmax[2 * bb + 1]);",
        "double lo = minmax[2 * bf], hi = minmax[2 * bf + 1];"),
    "preint_bilinear_corners_swapped": ("w[0] * (1.0 - w[1]) * p10 + (1.0 - w[0]) * w[1] * p01",
                                        "w[0] * (1.0 - w[1]) * p01 + (1.0 - w[0]) * w[1] * p10"),
    "prefilter_end_rows_unclamped": ("diag[i] = (i == 0 || i == n - 1) ? 5.0 : 4.0;", "diag[i] = 4.0;"),
    "prefilter_without_z_pass": ("for (long x = 0; x < nx; ++x) or_tridiag_line(out + x + nx * y, nz, nx * ny, sub, diag, sup, rhs);",
                                 "for (long x = 0; x < nx; ++x) (void)0;"),
    "catmull_rom_w1_wrong": ("w[1] = (3.0 * f * f * f - 5.0 * f * f + 2.0) / 2.0;",
                             "w[1] = (3.0 * f * f * f - 4.0 * f * f + 2.0) / 2.0;"),
    "catmull_rom_range_not_widened": ("if (widen > 0.0f) {", "if (widen > 1e30f) {"),
    "catmull_rom_widened_low_end_wrong_way": ("float wlo = fmaf(-widen, d, lo)", "float wlo = fmaf(widen, d, lo)"),
    "preclass_colour_not_opacity_weighted": ("for (int q = 0; q < 3; ++q) acc[q] += wt * t[3] * t[q];",
                                             "for (int q = 0; q < 3; ++q) acc[q] += wt * t[q];"),
    "preclass_colour_not_normalised": ("for (int q = 0; q < 3; ++q) out[q] = acc[3] > 0.0 ? acc[q] / acc[3] : 0.0;",
                                       "for (int q = 0; q < 3; ++q) out[q] = acc[q];"),
    "trilinear_weights_swapped": ("    w[1] = 1.0 - f;\n    w[2] = f;", "    w[1] = f;\n    w[2] = 1.0 - f;"),
}


def _lit_single_sample_half_slope(lib):
    shading.test_lit_single_sample_closed_form(lib, 0.5)

PINS = [
    pins.test_bspline_weights_worked_values,
    pins.test_bspline_weights_match_kernel_everywhere,
    pins.test_clamp_edge_worked_examples,
    pins.test_reconstruction_matches_rational_brute_force,
    pins.test_beer_lambert_axis_aligned_slab,
    pins.test_beer_lambert_oblique_rays,
    pins.test_oracle_matches_brute_force_tiny_volume,
    pins.test_oracle_matches_brute_force_table_tf_and_ert,
    pins.test_blocks_match_numpy_footprint,
    pins.test_occupancy_perturbation,
    pins.test_grad_closed_form_homogeneous_medium,
    pins.test_grad_volume_matches_central_differences,
    pins.test_grad_tf_matches_central_differences,
    shading.test_derivative_weights_match_the_kernel_derivative,
    shading.test_gradient_of_quadratic_field_is_exact,
    shading.test_gradient_matches_rational_brute_force,
    _lit_single_sample_half_slope,
    shading.test_lit_render_matches_brute_force,
    preint.test_table_linear_extinction_closed_form,
    preint.test_table_matches_adaptive_quadrature,
    lambda lib: preint.test_preint_skip_is_lossless(lib, 0.5, 8),
    lambda lib: preint.test_preint_skip_is_lossless(lib, 2.5, 4),
    preint.test_preint_skip_joins_both_blocks,
    preint.test_preint_render_matches_brute_force,
    lambda lib: filters.test_prefiltered_spline_interpolates_every_voxel(lib, (5, 6, 7), np.float64),
    filters.test_prefilter_line_matches_a_banded_solver,
    filters.test_catmull_rom_weights_match_the_kernel,
    filters.test_catmull_rom_interpolates_and_reproduces_quadratics,
    filters.test_catmull_rom_skip_is_lossless_with_widened_ranges,
    filters.test_preclassification_equals_post_for_linear_tfs,
    filters.test_preclassification_matches_brute_force,
    filters.test_trilinear_is_the_eight_tap_formula,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found exactly once"
    mutant_c = tmp_path / "oracle_mutant.c"
    mutant_c.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so),
                    str(mutant_c), "-lm"], check=True)
    prev = oracle.use(oracle.load(str(so)))
    caught = []
    try:
        for pin in PINS:
            try:
                pin(None)
            except AssertionError:
                caught.append(pin.__name__)
                break
    finally:
        oracle.use(prev)
    assert caught, f"no pin caught the planted mistake {name}"
