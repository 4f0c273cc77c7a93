"""The oracle pins must fail on plausible mistakes.  Each case plants one slip in the oracle
(monkeypatched, CPU only, undone after the test) and checks that at least one pin rejects it."""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
import tests.test_oracle_training as tpins
import tests.test_oracle_misalignment as mpins
import tests.test_oracle_input_gap as gpins
import tests.test_oracle_f4 as fpins
from oracle import dpx_oracle as o

TWO_PI = 2 * np.pi


def _h_sign_flipped(M, dx, wl, n_medium, z, shift=(0.0, 0.0), band_limited=False):
    f = o.spatial_frequencies(M, dx)
    q = (n_medium / wl) ** 2 - f[None, :] ** 2 - f[:, None] ** 2
    return np.where(q > 0, np.exp(-1j * TWO_PI * z * np.sqrt(np.maximum(q, 0))), 0)


def _h_no_cut(M, dx, wl, n_medium, z, shift=(0.0, 0.0), band_limited=False):
    f = o.spatial_frequencies(M, dx)
    q = (n_medium / wl) ** 2 - f[None, :] ** 2 - f[:, None] ** 2
    return np.exp(1j * TWO_PI * z * np.sqrt(q.astype(complex)))


def _h_axes_scaled(M, dx, wl, n_medium, z, shift=(0.0, 0.0), band_limited=False):
    f = o.spatial_frequencies(M, dx)
    q = (n_medium / wl) ** 2 - f[None, :] ** 2 - 0.5 * f[:, None] ** 2
    return np.where(q > 0, np.exp(1j * TWO_PI * z * np.sqrt(np.maximum(q, 0))), 0)


_orig_transfer = o.transfer_function


def _ramp_mutant(ramp):
    """A transfer function whose shift ramp is computed by ``ramp(f, sx, sy)``."""
    def H(M, dx, wl, n_medium, z, shift=(0.0, 0.0), band_limited=False):
        f = o.spatial_frequencies(M, dx)
        return _orig_transfer(M, dx, wl, n_medium, z) * ramp(f, M, dx, float(shift[0]), float(shift[1]))
    return H


_h_ramp_sign_flipped = _ramp_mutant(
    lambda f, M, dx, sx, sy: np.exp(+1j * TWO_PI * (f[None, :] * sx + f[:, None] * sy)))
_h_ramp_sign_flipped.__name__ = "_h_ramp_sign_flipped"
_h_ramp_axes_swapped = _ramp_mutant(
    lambda f, M, dx, sx, sy: np.exp(-1j * TWO_PI * (f[:, None] * sx + f[None, :] * sy)))
_h_ramp_axes_swapped.__name__ = "_h_ramp_axes_swapped"
# frequency in cycles per sample (k/M) times a shift left in metres
_h_ramp_index_units = _ramp_mutant(
    lambda f, M, dx, sx, sy: np.exp(-1j * TWO_PI * (f[None, :] * dx * sx + f[:, None] * dx * sy)))
_h_ramp_index_units.__name__ = "_h_ramp_index_units"


def _gap_shifts_reversed(D):
    D = np.asarray(D, float)
    return np.vstack([D[1:], np.zeros((1, 2))]) - D


def _gap_shifts_absolute(D):
    return np.asarray(D, float).copy()


def _gap_jitter_reversed(Dz):
    Dz = np.asarray(Dz, float)
    return Dz - np.append(Dz[1:], 0.0)


_orig_forward = o.forward


def _forward_without_input_gap(design, *args, **kw):
    return _orig_forward(dict(design, z_in=0.0), *args, **kw)


def _quantize_ties_up(h, h_max, bits):
    levels = (1 << bits) - 1
    k = np.floor(np.asarray(h, np.float32) * np.float32(levels / h_max) + np.float32(0.5))
    return (np.clip(k, 0, levels) * np.float32(h_max / levels)).astype(np.float32)


def _quantize_power_of_two_levels(h, h_max, bits):
    levels = 1 << bits
    k = np.rint(np.asarray(h, np.float32) * np.float32(levels / h_max))
    return (np.clip(k, 0, levels) * np.float32(h_max / levels)).astype(np.float32)


def _band_limit_without_factor_two(M, dx, wl, n_medium, z):
    return (n_medium / wl) / np.sqrt((z / (M * dx)) ** 2 + 1.0)


def _h_band_limited_x_only(M, dx, wl, n_medium, z, shift=(0.0, 0.0), band_limited=False):
    H = _orig_transfer(M, dx, wl, n_medium, z, shift)
    if band_limited:
        f = o.spatial_frequencies(M, dx)
        H = np.where((np.abs(f[None, :]) <= o.band_limit(M, dx, wl, n_medium, z)), H, 0.0)
    return H


def _phase_only_sign_flipped(phi, wl, lam_ref):
    return np.exp(-1j * np.asarray(phi, float) * (lam_ref / wl))


def _phase_only_unscaled(design, phi, lam_ref, u_in=None, mode="naive", wavelengths=None):
    """Eq. 3 layers that impose phi at every wavelength (no lambda_ref / lambda scaling)."""
    ws = range(design["n_wl"]) if wavelengths is None else list(wavelengths)
    out = []
    for w in ws:
        d1 = dict(design, wl=np.array([design["wl"][w]]), n_mat=np.array([design["n_mat"][w]]),
                  n_wl=1, kappa=None)
        lay = np.asarray(phi, np.float64) * (float(design["wl"][w]) / (2 * np.pi))
        out.append(_orig_forward(dict(d1, n_mat=np.array([design["n_medium"] + 1.0])), lay, u_in, mode)[0])
    return np.array(out)


def _idft_no_norm(V, mode="naive"):
    return np.fft.ifft2(V, axes=(-2, -1)) * V.shape[-1]


def _crop_shifted(U, N):
    return U[..., 1:1 + N, 1:1 + N]


def _fov_at_corner(design):
    return slice(0, design["fov"])


def _fov_at_far_corner(design):
    N, F = design["n"], design["fov"]
    return slice(N - F, N)


def _fov_one_sample_off(design):
    N, F = design["n"], design["fov"]
    a = (N - F) // 2 + 1
    return slice(a, a + F)


def _t_sign_flipped(h, wl, n_mat, kappa, n_medium):
    c_t, c_a = o.layer_constants(wl, n_mat, kappa, n_medium)
    return np.exp(-c_a * np.asarray(h, float)) * np.exp(-1j * c_t * np.asarray(h, float))


def _t_index_not_relative(h, wl, n_mat, kappa, n_medium):
    h = np.asarray(h, float)
    return np.exp(1j * TWO_PI * n_mat * h / wl)


def _loss_missing_inner(I, tau):
    L, g, per = _orig_loss(I, tau)
    I = np.asarray(I, float)
    S = I.sum(axis=(1, 2))
    W, P = I.shape[0], I.shape[1] * I.shape[2]
    d = I / S[:, None, None] - tau / tau.sum(axis=(1, 2))[:, None, None]
    return L, 2.0 / (W * P) * d / S[:, None, None], per


_orig_loss = o.loss
_orig_adam = o.adam_update


def _adam_no_bias_correction(g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    return -lr * m / (np.sqrt(v) + eps), m, v


def _adam_eps_inside(g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    return -lr * (m / (1 - b1 ** step)) / np.sqrt(v / (1 - b2 ** step) + eps), m, v


def _sigmoid_wrong_slope(x):
    return 1.0 / (1.0 + np.exp(-2.0 * x))


def _psnr_image_peak(I, tau):
    I = np.asarray(I, float)
    tau = np.asarray(tau, float)
    out = []
    for w in range(I.shape[0]):
        a, b = I[w] / I[w].sum(), tau[w] / tau[w].sum()
        mse = np.mean((a - b) ** 2)
        out.append(np.inf if mse == 0 else 10 * np.log10(a.max() ** 2 / mse))
    return np.array(out)


def _swap_shortest_first(ps, wl):
    by_psnr = np.argsort(-np.asarray(ps), kind="stable")
    by_length = np.argsort(np.asarray(wl), kind="stable")
    src = np.empty(len(wl), dtype=np.int64)
    src[by_length] = by_psnr
    return src

CASES = [
    ("quantize_heights", _quantize_ties_up, [fpins.test_quantiser_ties_go_to_even_levels]),
    ("quantize_heights", _quantize_power_of_two_levels, [fpins.test_quantiser_one_bit_and_exact_levels]),
    ("band_limit", _band_limit_without_factor_two, [fpins.test_band_limit_is_where_the_sampled_phase_steps_by_pi, (64, 20e-6)]),
    ("transfer_function", _h_band_limited_x_only, [fpins.test_band_limited_transfer_function_is_a_symmetric_mask]),
    ("forward_phase_only", _phase_only_unscaled, [fpins.test_phase_only_grating_diffraction_orders, (0.47e-6,)]),
    ("phase_only_transmission", _phase_only_sign_flipped, [fpins.test_phase_only_layer_is_the_unit_contrast_thickness_model]),
    ("forward", _forward_without_input_gap, [gpins.test_input_gap_equals_a_leading_transparent_layer]),
    ("transfer_function", _h_ramp_sign_flipped, [mpins.test_integer_shift_on_periodic_grid_is_a_roll, (3, -2)]),
    ("transfer_function", _h_ramp_axes_swapped, [mpins.test_integer_shift_on_periodic_grid_is_a_roll, (3, -2)]),
    ("transfer_function", _h_ramp_index_units, [mpins.test_subpixel_shift_moves_the_gaussian_centroid_by_the_shift]),
    ("gap_shifts_from_layer_offsets", _gap_shifts_reversed, [mpins.test_layer_offsets_match_a_physically_displaced_stack]),
    ("gap_jitter_from_layer_offsets", _gap_jitter_reversed, [mpins.test_axial_layer_offsets_match_moved_plane_positions]),
    ("gap_shifts_from_layer_offsets", _gap_shifts_absolute, [mpins.test_layer_offsets_match_a_physically_displaced_stack]),
    ("transfer_function", _h_sign_flipped, [pins.test_tilted_plane_wave, (3, 0)]),
    ("transfer_function", _h_no_cut, [pins.test_evanescent_wave_is_cut_even_at_short_range]),
    ("transfer_function", _h_axes_scaled, [pins.test_tilted_plane_wave, (0, 5)]),
    ("idft2", _idft_no_norm, [pins.test_normal_plane_wave_picks_up_exp_jkz]),
    ("crop_centered", _crop_shifted, [pins.test_mirror_symmetry_and_linearity]),
    ("fov_slice", _fov_at_corner, [pins.test_field_of_view_is_the_central_window, (16, 8, 1)]),
    ("fov_slice", _fov_at_far_corner, [pins.test_field_of_view_is_the_central_window, (18, 8, 2)]),
    ("fov_slice", _fov_one_sample_off, [pins.test_field_of_view_is_the_central_window, (20, 12, 4)]),
    ("fov_slice", _fov_at_corner, [pins.test_field_of_view_of_a_symmetric_design_is_flip_symmetric]),
    ("fov_slice", _fov_at_far_corner, [pins.test_field_of_view_of_a_symmetric_design_is_flip_symmetric]),
    ("transmission", _t_sign_flipped, [pins.test_prism_deflects_toward_thicker_side]),
    ("transmission", _t_index_not_relative, [pins.test_prism_deflects_toward_thicker_side]),
    ("loss", _loss_missing_inner, [pins.test_loss_gradient_finite_difference_and_euler]),
    ("adam_update", _adam_no_bias_correction, [tpins.test_adam_constant_gradient_closed_form]),
    ("adam_update", _adam_eps_inside, [tpins.test_adam_constant_gradient_closed_form]),
    ("sigmoid", _sigmoid_wrong_slope, [tpins.test_sigmoid_step_follows_the_chain_rule]),
    ("psnr", _psnr_image_peak, [tpins.test_psnr_of_a_known_perturbation]),
    ("channel_swap", _swap_shortest_first, [tpins.test_channel_swap_assigns_best_images_to_longest_wavelengths]),
]


@pytest.mark.parametrize("name,mutant,check", CASES,
                         ids=[f"{c[0]}:{c[1].__name__}" for c in CASES])
def test_pin_rejects_mutant(monkeypatch, name, mutant, check):
    monkeypatch.setattr(o, name, mutant)
    fn, *args = check
    with pytest.raises(AssertionError):
        fn(*(args[0] if args else ()))


def test_gradient_pin_rejects_dropped_absorption_term(monkeypatch):
    """Adjoint that forgets the -c_a Re(conj(g) v) term of dL/dh (only matters with kappa > 0)."""
    orig = o.layer_constants

    def grad_without_ca(design, h, u_in, dl_di, mode="naive", wavelengths=None):
        N, K = design["n"], design["layers"]
        _, vs, os_ = o.forward(design, h, u_in, mode, keep=True)
        out = np.zeros((K, N, N))
        fs = o.fov_slice(design)
        for w in range(design["n_wl"]):
            wl, nm, ka = float(design["wl"][w]), float(design["n_mat"][w]), float(design["kappa"][w])
            c_t, _ = orig(wl, nm, ka, design["n_medium"])
            g = np.zeros((N, N), complex)
            g[fs, fs] = 2.0 * dl_di[w] * os_[w]
            for l in range(K - 1, -1, -1):
                g = o.propagate(g, design["pad"], design["dx"], wl, design["n_medium"],
                                float(design["z"][l]), mode, adjoint=True)
                out[l] += -c_t * (np.conj(g) * vs[w, l]).imag
                g = np.conj(o.transmission(h[l], wl, nm, ka, design["n_medium"])) * g
        return out

    monkeypatch.setattr(o, "grad", grad_without_ca)
    with pytest.raises(AssertionError):
        pins.test_gradient_matches_central_differences(True, 1)
