"""Plant plausible mistakes in the oracle (CPU only) and check that a pin fails.

Each mutation swaps one oracle function for a subtly wrong version: a backward
difference, a missing conjugate, a wrong range-kernel sign, a dropped term.
The pins of ``test_oracle.py`` must reject every one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import blfls_oracle as ob
import tests.test_oracle as pins


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(ob, name, fn)
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


MUTATIONS = {
    "backward_grad_x": ("grad_x", lambda f: f - np.roll(f, 1, axis=-1)),
    "grad_y_along_x": ("grad_y", lambda f: np.roll(f, -1, axis=-1) - f),
    "range_sign": ("bilateral_filter", _bad_blf_sign),
    "spatial_sigma": ("bilateral_filter", _bad_blf_sigma),
    "solve_no_conj": ("blfls_solve", _bad_solve_noconj),
    "solve_drops_y_term": ("blfls_solve", _bad_solve_dropped_y),
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
