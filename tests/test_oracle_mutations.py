"""Plant plausible mistakes in the oracle (CPU only) and check that a pin fails.

Each mutation swaps one oracle function for a subtly wrong version: a backward
difference, a missing conjugate, a wrong range-kernel sign, a dropped term, an
NC filter with a wrong box schedule, wrapping windows or wrong increments, a
bilateral grid with a wrong Gaussian, without the periodic extension, with bins
rounded down or halves to even, a cap one bin too high or cells rounded halves
to even, an initial-guide Gaussian with sigma for sigma^2 or a short radius, an
adaptive-manifold filter with a shifted backward coefficient, the unhalved range
sigma in its blur, no column pass or no blend for far pixels.
The pins of ``test_oracle.py`` must reject every one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import blfls_oracle as ob
import tests.test_oracle as pins
import tests.test_oracle_nc as nc_pins
import tests.test_oracle_grid as grid_pins
import tests.test_oracle_amf as amf_pins


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(ob, name, fn)
    if hasattr(oracle, name):  # private helpers live in the module only
        monkeypatch.setattr(oracle, name, fn)


def _bad_blf_sign(p, q, sigma_s, sigma_r, radius):
    q = p if q is None else q
    num = np.zeros_like(p)
    den = np.zeros_like(p)
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2 * sigma_s ** 2))
            if math.isfinite(sigma_r):
                w = w * np.exp(-((np.roll(q, (-dy, -dx), (0, 1)) + q) ** 2) / (2 * sigma_r ** 2))
            num += w * np.roll(p, (-dy, -dx), (0, 1))
            den += w
    return num / den


def _bad_blf_sigma(p, q, sigma_s, sigma_r, radius):
    # spatial kernel with sigma instead of sigma^2
    q = p if q is None else q
    num = np.zeros_like(p)
    den = np.zeros_like(p)
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2 * sigma_s))
            if math.isfinite(sigma_r):
                w = w * np.exp(-((np.roll(q, (-dy, -dx), (0, 1)) - q) ** 2) / (2 * sigma_r ** 2))
            num += w * np.roll(p, (-dy, -dx), (0, 1))
            den += w
    return num / den


def _bad_solve_noconj(f, gx, gy, lam):
    F1, Fx, Fy = ob.difference_otf(*f.shape)
    num = np.fft.fft2(f) + lam * (Fx * np.fft.fft2(gx) + Fy * np.fft.fft2(gy))
    den = F1 + lam * (np.conj(Fx) * Fx + np.conj(Fy) * Fy)
    return np.real(np.fft.ifft2(num / den))


def _bad_solve_dropped_y(f, gx, gy, lam):
    F1, Fx, Fy = ob.difference_otf(*f.shape)
    num = np.fft.fft2(f) + lam * (np.conj(Fx) * np.fft.fft2(gx))
    den = F1 + lam * (np.conj(Fx) * Fx + np.conj(Fy) * Fy)
    return np.real(np.fft.ifft2(num / den))


def _bad_otf_transposed(H, W):
    F1, Fx, Fy = ob.__dict__["_orig_otf"](H, W)
    return F1, Fy, Fx


def _bad_nc_schedule_flat(sigma_s, n_iter=3):
    # every pass with the widest box
    return [math.sqrt(3.0) * sigma_s] * int(n_iter)


def _bad_nc_schedule_sigma(sigma_s, n_iter=3):
    # box half-width sigma_k instead of sqrt(3) sigma_k
    n = int(n_iter)
    return [sigma_s * math.sqrt(3.0) * 2.0 ** (n - k) / math.sqrt(4.0 ** n - 1.0) for k in range(1, n + 1)]


def _bad_nc_box_wrap(F, d, r, axis):
    # windows wrap around the borders
    F = np.asarray(F, dtype=np.float64)
    if axis == 0:
        return _bad_nc_box_wrap(F.T, d.T, r, 1).T
    num, cnt = F.copy(), np.ones_like(F)
    for sgn in (1, -1):
        dist = np.zeros(F.shape)
        live = np.ones(F.shape, dtype=bool)
        for k in range(1, int(r) + 2):
            inc = np.roll(d, -k if sgn > 0 else k - 1, axis=1)
            dist = dist + inc
            live &= dist <= r
            num += np.where(live, np.roll(F, -sgn * k, axis=1), 0.0)
            cnt += live
    return num / cnt


def _bad_nc_increments(q, a, inv_span=None):
    # increments from the guide values instead of their differences
    d = 1.0 + float(a) * np.abs(np.asarray(q, dtype=np.float64))
    return d, d.copy()


def _bad_gauss_sigma(img, sigma):
    # exp(-d^2 / (2 sigma)) instead of exp(-d^2 / (2 sigma^2))
    img = np.asarray(img, dtype=np.float64)
    r = int(math.ceil(3.0 * sigma))
    acc, tot = np.zeros_like(img), 0.0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma))
            acc += w * np.roll(img, (-dy, -dx), axis=(-2, -1))
            tot += w
    return acc / tot


def _bad_gauss_radius(img, sigma):
    # radius ceil(2 sigma) instead of ceil(3 sigma)
    img = np.asarray(img, dtype=np.float64)
    r = int(math.ceil(2.0 * sigma))
    acc, tot = np.zeros_like(img), 0.0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
            acc += w * np.roll(img, (-dy, -dx), axis=(-2, -1))
            tot += w
    return acc / tot


_orig_grid_scale = ob._grid_scale


def _bad_grid_range_floor(q, sigma_r, inv_span=None):
    # bins floor(t) instead of floor(t + 1/2)
    q = np.asarray(q, dtype=np.float64)
    qmin, _span, inv, _c = _orig_grid_scale(q, sigma_r, inv_span)
    z = np.floor((q - qmin) * inv).astype(np.int64)
    return qmin, inv, z, int(z.max()) + 1


def _bad_grid_range_half_even(q, sigma_r, inv_span=None):
    # halves rounded to even instead of up
    q = np.asarray(q, dtype=np.float64)
    qmin, _span, inv, _c = _orig_grid_scale(q, sigma_r, inv_span)
    z = np.round((q - qmin) * inv).astype(np.int64)
    return qmin, inv, z, int(z.max()) + 1


def _bad_grid_scale_cap(q, sigma_r, inv_span=None):
    # the cap lets GRID_ZMAX + 1 bins through
    q = np.asarray(q, dtype=np.float64)
    qmin = float(q.min())
    span = float(q.max()) - qmin
    inv = 0.0 if math.isinf(sigma_r) else 1.0 / float(np.float32(sigma_r))
    if inv_span is not None:
        inv *= float(inv_span)
    capped = span * inv > ob.GRID_ZMAX
    if capped:
        inv = ob.GRID_ZMAX / span
    return qmin, span, inv, capped


def _bad_grid_cell_half_even(sigma_s):
    return max(1, int(round(float(np.float32(sigma_s)))))


def _bad_grid_taps(sigma_cells):
    # Gaussian with sigma instead of sigma^2
    k = np.arange(-ob.GRID_PAD, ob.GRID_PAD + 1, dtype=np.float64)
    if sigma_cells <= 0.0:
        return (k == 0).astype(np.float64)
    return np.exp(-(k * k) / (2.0 * sigma_cells))


_orig_grid_filter = ob.grid_filter


def _bad_grid_zero_border(p, q, sigma_s, sigma_r, inv_span=None):
    # the grid built over the image alone (zero beyond the border) instead of its periodic extension
    p = np.asarray(p, dtype=np.float64)
    H, W = p.shape
    big = np.zeros((3 * H, 3 * W))
    big[H:2 * H, W:2 * W] = p
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    qbig = np.full((3 * H, 3 * W), qq.min())
    qbig[H:2 * H, W:2 * W] = qq
    return _orig_grid_filter(big, qbig, sigma_s, sigma_r, inv_span)[H:2 * H, W:2 * W]


def _bad_amf_rf_backward_index(X, alpha):
    # the right-to-left pass takes the coefficient of its own sample, not of the step
    out = []
    W = alpha.shape[1]
    for x in X:
        y = np.array(x, dtype=np.float64, copy=True)
        for j in range(1, W):
            y[:, j] = (1.0 - alpha[:, j]) * y[:, j] + alpha[:, j] * y[:, j - 1]
        for j in range(W - 2, -1, -1):
            y[:, j] = (1.0 - alpha[:, j]) * y[:, j] + alpha[:, j] * y[:, j + 1]
        out.append(y)
    return out


_orig_amf_alpha = ob._amf_alpha
_orig_amf_blur = ob.amf_blur
_orig_amf_filter = ob.amf_filter


def _bad_amf_alpha_sigma(eta, sigma_s, sigma_r, axis, inv_span):
    # the blur's range term with sigma_r instead of sigma_r / sqrt(2)
    return _orig_amf_alpha(eta, sigma_s, sigma_r * math.sqrt(2.0), axis, inv_span)


def _bad_amf_rows_only(X, eta, sigma_s, sigma_r, inv_span=None):
    ref = np.zeros(X[0].shape) if eta is None else eta
    ah = _orig_amf_alpha(ref, sigma_s, math.inf if eta is None else sigma_r, 1, inv_span)
    return ob.amf_rf_line_rows(X, ah)


def _bad_amf_no_blend(p, q, sigma_s, sigma_r, height=0, inv_span=None, return_manifolds=False):
    # num / den everywhere: pixels far from every manifold are not kept
    g, mans = _orig_amf_filter(p, q, sigma_s, sigma_r, height, inv_span, return_manifolds=True)
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    s = float(np.float32(sigma_s))
    r = float(np.float32(sigma_r))
    k = 0.0 if math.isinf(r) else 1.0 / (r * r)
    scale = 1.0 if inv_span is None else float(inv_span)
    num = np.zeros_like(p)
    den = np.zeros_like(p)
    for eta in mans:
        present = ~np.isnan(eta)
        dq = np.where(present, (eta - qq) * scale, 0.0)
        psi = np.where(present, np.exp(-k * dq * dq), 0.0)
        bn, bd = ob.amf_blur([psi * p, psi], eta, s, r, inv_span)
        num += psi * bn
        den += psi * bd
    g = np.where(den > 0, num / np.where(den > 0, den, 1.0), p)
    return (g, mans) if return_manifolds else g


MUTATIONS = {
    "backward_grad_x": ("grad_x", lambda f: f - np.roll(f, 1, axis=-1)),
    "grad_y_along_x": ("grad_y", lambda f: np.roll(f, -1, axis=-1) - f),
    "range_sign": ("bilateral_filter", _bad_blf_sign),
    "spatial_sigma": ("bilateral_filter", _bad_blf_sigma),
    "solve_no_conj": ("blfls_solve", _bad_solve_noconj),
    "solve_drops_y_term": ("blfls_solve", _bad_solve_dropped_y),
    "nc_flat_schedule": ("nc_schedule", _bad_nc_schedule_flat),
    "nc_box_sigma_not_sqrt3": ("nc_schedule", _bad_nc_schedule_sigma),
    "nc_windows_wrap": ("nc_box_pass", _bad_nc_box_wrap),
    "nc_increments_from_values": ("nc_increments", _bad_nc_increments),
    "grid_sigma_not_squared": ("_grid_taps", _bad_grid_taps),
    "grid_zero_border": ("grid_filter", _bad_grid_zero_border),
    "grid_bin_floor": ("grid_range", _bad_grid_range_floor),
    "grid_bin_half_to_even": ("grid_range", _bad_grid_range_half_even),
    "grid_cap_off_by_one": ("_grid_scale", _bad_grid_scale_cap),
    "grid_cell_half_to_even": ("grid_cell", _bad_grid_cell_half_even),
    "gaussian_guide_sigma_not_squared": ("gaussian_blur", _bad_gauss_sigma),
    "gaussian_guide_radius": ("gaussian_blur", _bad_gauss_radius),
    "amf_backward_coefficient_index": ("amf_rf_line_rows", _bad_amf_rf_backward_index),
    "amf_blur_sigma_not_halved": ("_amf_alpha", _bad_amf_alpha_sigma),
    "amf_blur_rows_only": ("amf_blur", _bad_amf_rows_only),
    "amf_no_far_pixel_blend": ("amf_filter", _bad_amf_no_blend),
}

PIN_SUITE = [
    pins.test_gradients_match_loops,
    lambda: pins.test_P1_fft_solve_equals_dense(5, 7, 20.0),
    pins.test_P2_stencil_residual,
    lambda: pins.test_P3_blf_bruteforce(6, 7, 2, 1.0, 0.3, False),
    lambda: pins.test_hand_derived_1x4(20.0),
    pins.test_P6_identity_filter_keeps_f,
    lambda: pins.test_P7_sigma_r_infinite_closed_form(32, 40, 1.5, 5),
    pins.test_P11_symmetries,
    pins.test_normalisation_is_a_range_rescale,
    lambda: nc_pins.test_nc_matches_pixel_loops(5, 7, 2.0, 0.3, 3),
    lambda: nc_pins.test_nc_schedule_variances_sum_to_sigma_s_squared(3),
    nc_pins.test_nc_without_range_term_is_iterated_box_filtering,
    nc_pins.test_nc_keeps_constants_and_clean_steps,
    lambda: grid_pins.test_grid_with_unit_cells_and_no_range_is_the_exact_gaussian(0.75),
    grid_pins.test_grid_commutes_with_whole_cell_shifts,
    pins.test_grid_range_hand_derived_bins,
    pins.test_grid_bin_margin_hand_derived,
    lambda: pins.test_grid_cell_hand_derived(2.5, 3),
    lambda: pins.test_grid_cell_hand_derived(8.5, 9),
    lambda: pins.test_gaussian_blur_is_the_library_gaussian_on_a_torus(1.7),
    lambda: pins.test_gaussian_blur_impulse_support_and_variance(1.7),
    pins.test_nc_decision_margin_by_loops,
    lambda: amf_pins.test_amf_matches_explicit_operators(6, 6, 3.0, 0.05, 3),
    amf_pins.test_rf_step_that_cannot_be_crossed_splits_the_line,
    amf_pins.test_range_off_is_the_separable_exponential_kernel,
]


def _some_pin_fails():
    for pin in PIN_SUITE:
        try:
            pin()
        except AssertionError:
            return True
    return False


def test_unmutated_suite_passes():
    assert not _some_pin_fails()


@pytest.mark.parametrize("mutation", sorted(MUTATIONS))
def test_mutation_is_caught(monkeypatch, mutation):
    name, fn = MUTATIONS[mutation]
    _patch(monkeypatch, name, fn)
    assert _some_pin_fails(), f"no pin caught the planted mistake {mutation}"


def test_transposed_otf_is_caught(monkeypatch):
    monkeypatch.setitem(ob.__dict__, "_orig_otf", ob.difference_otf)
    _patch(monkeypatch, "difference_otf", _bad_otf_transposed)
    assert _some_pin_fails()
