"""Planted mistakes in the FP64 oracle (CPU): each must fail at least one of its pins.

Every case copies ``oracle/nic_oracle.c``, plants one plausible slip (a dropped term, a wrong sign,
a transposed index or operand, a wrong constant), builds the copy with the oracle's own gcc flags
into a fresh library, loads the oracle's Python wrapper against it, and runs the pins named for the
case from ``test_oracle_pins.py``.  The case passes when one of those pins fails on the mutant;
a control runs the same pins on an unmodified copy and requires all of them to pass.  The HIP
library is not involved.
"""
import importlib.util
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_INIT = os.path.join(ROOT, "oracle", "__init__.py")
ORACLE_C = os.path.join(ROOT, "oracle", "nic_oracle.c")


def _pins():
    spec = importlib.util.spec_from_file_location("_pins_for_mutants", os.path.join(HERE, "test_oracle_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


def _oracle_copy(tmp_path, name, old=None, new=None):
    src = open(ORACLE_C).read()
    if old is not None:
        assert src.count(old) == 1, f"mutation site not unique: {old!r}"
        src = src.replace(old, new)
    c_path = tmp_path / f"{name}.c"
    c_path.write_text(src)
    spec = importlib.util.spec_from_file_location(f"_oracle_{name}", ORACLE_INIT)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod      # dataclasses look their module up by name
    spec.loader.exec_module(mod)
    mod._SRC = str(c_path)
    mod._LIB = str(tmp_path / f"lib{name}.so")
    mod.build(force=True)
    return mod


# (id, site in nic_oracle.c, planted replacement, pins expected to catch it [(name, kwargs)])
MUTANTS = [
    ("hash_prime", "(v1 * 2654435761u)", "(v1 * 2654435769u)",
     [("test_vertex_index_bruteforce", {}), ("test_encode_indices_bruteforce", {})]),
    ("dense_index_transposed", "(uint64_t)v0 + s * ((uint64_t)v1 + s * (uint64_t)v2)",
     "(uint64_t)v2 + s * ((uint64_t)v1 + s * (uint64_t)v0)",
     [("test_vertex_index_bruteforce", {}), ("test_affine_reproduction_on_dense_level", {})]),
    ("trilinear_weight_swapped", "w[k] = (c0 ? f[0] : 1.0 - f[0])", "w[k] = (c0 ? 1.0 - f[0] : f[0])",
     [("test_affine_reproduction_on_dense_level", {}), ("test_grid_vertices_return_exact_entries", {"N": 16, "log2T": 14})]),
    ("level_resolution_off_by_one", "float pos = x[d] * (float)o->res[l];",
     "float pos = x[d] * (float)(o->res[l] - 1);",
     [("test_grid_vertices_return_exact_entries", {"N": 16, "log2T": 14}), ("test_affine_reproduction_on_dense_level", {})]),
    ("layernorm_unbiased_variance", "    v /= (double)o->C;\n", "    v /= (double)(o->C - 1);\n",
     [("test_layernorm_invariants", {}), ("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("layernorm_eps_outside_sqrt", "double s = 1.0 / sqrt(v + c->ln_eps);", "double s = 1.0 / (sqrt(v) + c->ln_eps);",
     [("test_layernorm_invariants", {}), ("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("relu_dropped", "st->h[k][u] = s > 0.0 ? s : 0.0;", "st->h[k][u] = s;",
     [("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("sigmoid_sign", "return c->mu_max / (1.0 + exp(-y));", "return c->mu_max / (1.0 + exp(y));",
     [("test_field_and_gradient_match_torch", {"layernorm": 1}), ("test_constant_field_line_integral_closed_form", {})]),
    ("bias_gradient_dropped", "gd[o->o_b[k] + u] += ga[u];", "gd[o->o_b[k] + u] += 0.0 * ga[u];",
     [("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("layernorm_backward_sign", "gx[i] = st->rstd * (g[i] - mg - st->xhat[i] * mgx);",
     "gx[i] = st->rstd * (g[i] - mg + st->xhat[i] * mgx);",
     [("test_layernorm_backward_invariants", {}), ("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("table_gradient_weight_dropped", "+= st->w[l][k] * gx[l * o->F + f];", "+= gx[l * o->F + f];",
     [("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("ray_sum_without_step", "A += st->mu * delta;", "A += st->mu;",
     [("test_constant_field_line_integral_closed_form", {})]),
    ("step_without_length", "*delta = dt * len;", "*delta = dt;",
     [("test_central_ray_passes_through_origin", {}), ("test_constant_field_line_integral_closed_form", {})]),
    ("jitter_ignored", "t0 + ((double)i + (double)jitter[i]) * dt", "t0 + ((double)i + 0.5) * dt",
     [("test_samples_follow_pixel_ray", {})]),
    ("detector_axis_sign", "double P0 = dc0 + u * (-sa);", "double P0 = dc0 + u * sa;",
     [("test_samples_follow_pixel_ray", {})]),
    ("l1_gradient_sign", "((rs > 0.0) - (rs < 0.0)) / (double)R", "((rs < 0.0) - (rs > 0.0)) / (double)R",
     [("test_finite_differences_l1_loss", {})]),
    ("adam_bias_correction_dropped", "double mh = m[i] / bc1;", "double mh = m[i];",
     [("test_adam_first_step_closed_form", {}), ("test_adam_matches_torch", {})]),
    ("adam_eps_inside_sqrt", "(sqrt(vh) + eps)", "sqrt(vh + eps)",
     [("test_adam_first_step_closed_form", {}), ("test_adam_matches_torch", {})]),
    ("philox_multiplier", "(uint64_t)0xD2511F53u * (uint64_t)c[0]", "(uint64_t)0xD2511F57u * (uint64_t)c[0]",
     [("test_philox_known_answers", {})]),
    ("philox_key_schedule", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;",
     [("test_philox_known_answers", {})]),
    ("psnr_amplitude_not_power", "return 10.0 * log10(mx * mx / mse);", "return 10.0 * log10(mx / mse);",
     [("test_psnr_closed_forms", {})]),
    ("ssim_constant", "c2 = (0.03 * L) * (0.03 * L);", "c2 = (0.3 * L) * (0.3 * L);",
     [("test_ssim_pins", {})]),
    ("voxel_trilinear_half_offset", "double u = (double)x[k] * (double)n - 0.5;", "double u = (double)x[k] * (double)n;",
     [("test_trilinear_reproduces_affine_and_voxels", {})]),
    ("voxel_loss_gradient_sign", "((r > 0.0) - (r < 0.0)) / (double)B", "((r < 0.0) - (r > 0.0)) / (double)B",
     [("test_voxel_loss_finite_differences", {})]),
    ("layernorm_gain_gradient", "gd[o->o_lng + i] += gh[i] * st->xhat[i];", "gd[o->o_lng + i] += gh[i];",
     [("test_field_and_gradient_match_torch", {"layernorm": 1})]),
    ("mask_backward_dropped", "for (int i = 0; i < o->C; ++i) gx[i] *= c->mask[i];",
     "for (int i = 0; i < o->C; ++i) gx[i] *= 1.0;",
     [("test_channel_mask_pins", {"layernorm": 1}), ("test_channel_mask_pins", {"layernorm": 0})]),
    ("pixel_cycle_walk_once", "while ((int64_t)y >= n_pix) y = feistel(seed, t, h, y);",
     "if ((int64_t)y >= n_pix) y = feistel(seed, t, h, y);",
     [("test_ray_pixels_distinct_and_in_range", {"n_pix": 1000, "R": 1000}),
      ("test_ray_pixels_distinct_and_in_range", {"n_pix": 65, "R": 64}), ("test_ray_pixels_full_permutation", {})]),
    ("view_epoch_length", "uint32_t e = t / (uint32_t)V, pos = t % (uint32_t)V;",
     "uint32_t e = t / (uint32_t)(V + 1), pos = t % (uint32_t)V;",
     [("test_view_order_visits_every_view_each_epoch", {})]),
    ("table_init_range", "params[e] = (2.0 * u - 1.0) * 1e-4;", "params[e] = (2.0 * u - 1.0) * 1e-3;",
     [("test_init_params_distribution", {})]),
    ("render_voxel_corner_not_centre", "float x[3] = {(float)(((double)ix + 0.5) / (double)nx)",
     "float x[3] = {(float)(((double)ix) / (double)nx)",
     [("test_render_volume_matches_field", {})]),
    ("train_adam_step_index", "(int64_t)t + 1, lr, b1, b2, eps);", "(int64_t)t + 2, lr, b1, b2, eps);",
     [("test_train_is_the_composed_schedule", {})]),
    ("train_view_of_next_step", "int32_t view = ora_view_for_step(seed, t, V);",
     "int32_t view = ora_view_for_step(seed, t + 1, V);",
     [("test_train_is_the_composed_schedule", {})]),
    ("train_gradient_not_reset", "    memset(grad, 0, sizeof(double) * (size_t)np);\n", "\n",
     [("test_train_is_the_composed_schedule", {})]),
    ("softplus_threshold", "(y > 20.0) ? y : log1p(exp(y))", "(y > 2.0) ? y : log1p(exp(y))",
     [("test_output_activations_match_torch", {"out_act": 2})]),
    ("softplus_gradient_sign", "(y > 20.0) ? 1.0 : 1.0 / (1.0 + exp(-y))", "(y > 20.0) ? 1.0 : 1.0 / (1.0 + exp(y))",
     [("test_output_activations_match_torch", {"out_act": 2})]),
    ("identity_head_gradient", "if (c->out_act == 1) return 1.0;", "if (c->out_act == 1) return 0.5;",
     [("test_output_activations_match_torch", {"out_act": 1})]),
    ("thread_buffers_dropped", "      for (int t = 1; t < nth; ++t) grad[i] += bufs[t][i];",
     "      for (int t = 1; t < nth; ++t) grad[i] += 0.0 * bufs[t][i];",
     [("test_ray_batch_thread_count_invariance", {})]),
]


def _run(pins, mod, cases):
    failed = []
    for name, kw in cases:
        try:
            getattr(pins, name)(mod, **kw)
        except Exception as e:   # an assertion (or any error) raised by the pin
            failed.append(f"{name}: {type(e).__name__}")
    return failed


def test_control_copy_passes_every_pin_used(tmp_path):
    pins = _pins()
    mod = _oracle_copy(tmp_path, "control")
    cases = sorted({(n, tuple(sorted(kw.items()))) for *_, cs in MUTANTS for n, kw in cs})
    assert _run(pins, mod, [(n, dict(kw)) for n, kw in cases]) == []


@pytest.mark.parametrize("mid,old,new,cases", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, mid, old, new, cases):
    pins = _pins()
    mod = _oracle_copy(tmp_path, mid, old, new)
    assert _run(pins, mod, cases), f"mutant {mid} survived {[c[0] for c in cases]}"
