"""Planted mistakes in the oracle must be caught by its pins.

Each case swaps one oracle function for a plausible wrong version (a dropped
term, a wrong sign or index, a transposed operand) and checks that at least one
pin test fails.  Everything runs on the CPU; nothing touches the GPU path.
"""
import numpy as np
import pytest

from oracle import nrc_oracle as O
import tests.test_oracle_pins as P


def _freq_no_pi(p, preset=O.PRESET_CONFIG):
    return O.__dict__["_orig_freq"](p / np.pi, preset)


def _one_blob_no_tails(s, k=O.N_BLOBS):
    c = k * np.asarray(s, dtype=np.float64)
    out = np.empty(np.shape(s) + (k,))
    for j in range(k):
        out[..., j] = O.quartic_cdf(j + 1 - c) - O.quartic_cdf(j - c)
    return out


def _forward_transposed(mats, h0):
    return O.__dict__["_orig_forward"]([np.asarray(w).T if w.shape[0] == w.shape[1] else w for w in mats], h0)


def _loss_no_stop_gradient(y_hat, y, eps=O.LOSS_EPS):
    # differentiates through the denominator as well
    y_hat = np.asarray(y_hat, float)
    n = y_hat.shape[0]
    lum = y_hat.mean(axis=1, keepdims=True)
    den = lum * lum + eps
    diff = y_hat - y
    loss = float((diff * diff / den).sum() / (3 * n))
    d_den = -(diff * diff / den ** 2).sum(axis=1, keepdims=True) * 2 * lum / 3
    return loss, (2 * diff / den + d_den) / (3 * n)


def _loss_wrong_sign(y_hat, y, eps=O.LOSS_EPS):
    loss, g = O.__dict__["_orig_relative_l2"](y_hat, y, eps)
    return loss, -g


def _backward_no_mask(mats, hs, delta_out):
    grads = [None] * len(mats)
    delta = np.asarray(delta_out, float)
    for l in range(len(mats) - 1, -1, -1):
        grads[l] = delta.T @ hs[l]
        g_in = delta @ np.asarray(mats[l], float)
        if l == 0:
            return grads, g_in
        delta = g_in


def _adam_swapped_betas(w, m, v, t, g, cfg):
    swapped = O.AdamConfig(lr=cfg.lr, beta1=cfg.beta2, beta2=cfg.beta1, eps=cfg.eps)
    return O.__dict__["_orig_adam"](w, m, v, t, g, swapped)


def _adam_no_bias_correction(w, m, v, t, g, cfg):
    t = t + 1
    m = cfg.beta1 * m + (1 - cfg.beta1) * g
    v = cfg.beta2 * v + (1 - cfg.beta2) * g * g
    return w - cfg.lr * m / (np.sqrt(v) + cfg.eps), m, v, t


def _reflectance_shifted_columns(enc, preset):
    a, b = O.albedo_columns(preset)
    enc = np.asarray(enc, float)
    return enc[:, a - 1:a + 2] + enc[:, b - 1:b + 2]


def _query_gradient_no_albedo_term(state, enc, grad_out):
    f, hs = O.forward(state.mats(), enc)
    grads, g_in = O.backward(state.mats(), hs, np.asarray(grad_out) * O.reflectance(enc, state.preset))
    return np.concatenate([g.reshape(-1) for g in grads]), g_in


def _gradient_factor_dropped(state, enc, y):
    # the loss sees f R but the gradient ignores R on the way back
    f, hs = O.forward(state.mats(), enc)
    r = O.reflectance(enc, state.preset) if state.factorize else 1.0
    loss, d_out = O.relative_l2(f * r, y, state.loss_eps)
    grads, _ = O.backward(state.mats(), hs, d_out)
    return loss, np.concatenate([g.reshape(-1) for g in grads])


def _lcg_even_increment(n, seed):
    m = O.lcg_modulus(n)
    x, out = seed % m, []
    for _ in range(m):
        if x < n:
            out.append(x)
        x = (O.LCG_A * x + O.LCG_C - 1) % m
    return np.array(out, dtype=np.int64)


def _lcg_keeps_n(n, seed):
    m = O.lcg_modulus(n)
    x, out = seed % m, []
    for _ in range(m):
        if x <= n:
            out.append(x)
        x = (O.LCG_A * x + O.LCG_C) % m
    return np.array(out, dtype=np.int64)


def _targets_wrong_tail(radiance, throughput, tail_rgb, tail_index):
    return np.asarray(radiance, float) + np.asarray(throughput, float) * np.asarray(tail_rgb, float)[
        (np.asarray(tail_index) + 1) % len(tail_rgb)]


def _sph_angles_swapped(v):
    return O.__dict__["_orig_sph"](v)[:, ::-1]


def _sph_azimuth_unshifted(v):
    v = np.asarray(v, dtype=np.float64)
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    return np.stack([theta / np.pi, np.arctan2(v[:, 1], v[:, 0]) / (2.0 * np.pi)], axis=1)


def _tri_sine_phase(x):
    # the printed wave shifted by a quarter period (in phase with sin(pi x))
    return 2.0 * np.abs(np.mod(x - 0.5, 2.0) - 1.0) - 1.0


def _tri_unit_period(x):
    # the reduction taken mod 1 instead of mod 2
    return 2.0 * np.abs(np.mod(x, 1.0) - 1.0) - 1.0


def _loss_sum_luminance(y_hat, y, eps=O.LOSS_EPS):
    y_hat = np.asarray(y_hat, float)
    n = y_hat.shape[0]
    lum = y_hat.sum(axis=1, keepdims=True)
    den = lum * lum + eps
    diff = y_hat - np.asarray(y, float)
    return float((diff * diff / den).sum() / (3 * n)), 2 * diff / den / (3 * n)


def _loss_eps_squared(y_hat, y, eps=O.LOSS_EPS):
    y_hat = np.asarray(y_hat, float)
    n = y_hat.shape[0]
    lum = y_hat.mean(axis=1, keepdims=True)
    den = (lum + eps) ** 2
    diff = y_hat - np.asarray(y, float)
    return float((diff * diff / den).sum() / (3 * n)), 2 * diff / den / (3 * n)


def _adam_eps_inside_sqrt(w, m, v, t, g, cfg):
    t = t + 1
    m = cfg.beta1 * m + (1 - cfg.beta1) * g
    v = cfg.beta2 * v + (1 - cfg.beta2) * g * g
    m_hat, v_hat = m / (1 - cfg.beta1 ** t), v / (1 - cfg.beta2 ** t)
    return w - cfg.lr * m_hat / np.sqrt(v_hat + cfg.eps), m, v, t


def _ema_no_bias_correction(w_bar_prev, w, t, alpha):
    return (1.0 - alpha) * w + alpha * w_bar_prev


def _frame_batches_unshuffled(n, steps, batch, seed):
    used = min(n, steps * batch)
    return [np.arange(s * used // steps, (s + 1) * used // steps) for s in range(steps)]


def _frame_batches_fixed_size(n, steps, batch, seed):
    perm = O.lcg_permutation(n, seed)
    return [perm[s * batch:(s + 1) * batch] for s in range(steps)]


def _one_blob_bins_reversed(s, k=O.N_BLOBS):
    return O.__dict__["_orig_one_blob"](s, k)[..., ::-1]


def _gauss_twice_as_wide(u):
    return O.__dict__["_orig_gauss_cdf"](np.asarray(u, dtype=np.float64) / 2.0)


MUTANTS = [
    ("freq", _freq_no_pi, [P.test_freq_matches_libm_closed_form, P.test_freq_dyadic_points_exact]),
    ("one_blob", _one_blob_no_tails, [P.test_one_blob_exact_dyadic_fixture, P.test_one_blob_invariants]),
    ("forward", _forward_transposed, [P.test_forward_brute_force_tiny]),
    ("relative_l2", _loss_no_stop_gradient, [P.test_loss_gradient_is_stop_gradient_derivative]),
    ("relative_l2", _loss_wrong_sign, [P.test_loss_gradient_is_stop_gradient_derivative,
                                       P.test_backward_matches_torch_autograd_fp64]),
    ("backward", _backward_no_mask, [P.test_backward_central_differences_weights_and_inputs]),
    ("adam", _adam_swapped_betas, [P.test_adam_matches_torch_optim_fp64]),
    ("adam", _adam_no_bias_correction, [P.test_adam_constant_gradient_closed_form]),
    ("reflectance", _reflectance_shifted_columns, [P.test_factorised_prediction_scales_by_raw_albedos]),
    ("query_gradient", _query_gradient_no_albedo_term, [P.test_factorised_query_gradient_central_differences]),
    ("gradient", _gradient_factor_dropped, [P.test_factorised_train_gradient_central_differences]),
    ("lcg_permutation", _lcg_even_increment, [P.test_lcg_full_period_and_permutation]),
    ("lcg_permutation", _lcg_keeps_n, [P.test_lcg_orbit_matches_hand_derived_fixture]),
    ("self_training_targets", _targets_wrong_tail, [P.test_self_training_targets]),
    ("sph", _sph_angles_swapped, [P.test_sph_axes, P.test_sph_inverts_spherical_parametrisation]),
    ("sph", _sph_azimuth_unshifted, [P.test_sph_axes, P.test_sph_inverts_spherical_parametrisation]),
    ("tri", _tri_sine_phase, [P.test_triangle_wave_closed_form, P.test_encode_paper_tri_preset_layout]),
    ("tri", _tri_unit_period, [P.test_triangle_wave_closed_form, P.test_encode_paper_tri_preset_layout]),
    ("relative_l2", _loss_sum_luminance, [P.test_loss_single_sample_by_hand]),
    ("relative_l2", _loss_eps_squared, [P.test_loss_single_sample_by_hand]),
    ("adam", _adam_eps_inside_sqrt, [P.test_adam_constant_gradient_closed_form]),
    ("ema_step", _ema_no_bias_correction, [P.test_ema_matches_explicit_weighted_average,
                                           P.test_ema_first_step_and_constant_weights]),
    ("frame_batches", _frame_batches_unshuffled, [P.test_frame_batches_are_disjoint_and_spread_over_the_records]),
    ("frame_batches", _frame_batches_fixed_size, [P.test_frame_batches_are_disjoint_and_spread_over_the_records]),
    ("one_blob", _one_blob_bins_reversed, [P.test_one_blob_exact_dyadic_fixture]),
    ("gauss_cdf", _gauss_twice_as_wide, [P.test_gauss_one_blob_matches_numerical_bin_integrals,
                                         P.test_gauss_one_blob_invariants]),
]


@pytest.mark.parametrize("name,mutant,pins", MUTANTS, ids=[m[1].__name__ for m in MUTANTS])
def test_pins_catch_planted_mistake(monkeypatch, name, mutant, pins):
    monkeypatch.setitem(O.__dict__, "_orig_" + name, getattr(O, name))
    monkeypatch.setattr(O, name, mutant)
    caught = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, f"no pin caught the planted mistake in {name}"
