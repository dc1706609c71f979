"""Pins of the oracle's adaptive-manifold filter and AMF-LS (CPU only).

AMF-LS (Section III-D) embeds the adaptive-manifold filter in place of the
BLF.  These tests pin the oracle's filter to what its definition and
elementary mathematics fix: the same filter built from explicit linear
operators (the closed forms of the recursive passes) with per-pixel loops, the
closed-form impulse response of the recursive filter, a step too long to cross
splitting a line into independent parts, the separable exponential kernel the
filter reduces to when the range kernel is off, constants, convexity, clean
steps that must pass unchanged, its closeness to the exact filter of Eq. (1)
that it approximates, and the method-level invariants shared with BLF-LS.
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image


def _rand(shape, seed):
    return np.random.default_rng(seed).random(shape)


@pytest.mark.parametrize("H,W,sigma_s,sigma_r,height", [
    (5, 7, 2.0, 0.3, 2),
    (6, 6, 3.0, 0.05, 3),
    (1, 9, 4.0, 0.2, 2),
    (8, 1, 4.0, 0.2, 1),
    (4, 5, 12.0, 0.5, 0),
    (5, 6, 2.5, math.inf, 2),
])
def test_amf_matches_explicit_operators(H, W, sigma_s, sigma_r, height):
    p = _rand((H, W), 1) * 0.4
    q = _rand((H, W), 2) * 0.4
    for guide in (None, q):
        for inv in (None, np.float32(2.5)):
            a = oracle.amf_filter(p, guide, sigma_s, sigma_r, height, inv_span=inv)
            b = oracle.amf_filter_dense(p, guide, sigma_s, sigma_r, height, inv_span=inv)
            assert np.max(np.abs(a - b)) < 1e-13


def test_rf_interior_impulse_response_is_the_symmetric_exponential():
    # left-to-right then right-to-left with a constant coefficient a: away from the
    # ends, an impulse spreads as (1 - a) / (1 + a) a^|k|
    n, c = 401, 200
    sigma_s = 2.0
    a = math.exp(-math.sqrt(2.0) / sigma_s)
    x = np.zeros((1, n))
    x[0, c] = 1.0
    y = oracle.amf_rf_line_rows([x], np.full((1, n), a))[0][0]
    k = np.arange(n) - c
    ref = (1.0 - a) / (1.0 + a) * a ** np.abs(k)
    mid = slice(c - 60, c + 61)
    assert np.max(np.abs(y[mid] - ref[mid])) < 1e-14


def test_rf_step_that_cannot_be_crossed_splits_the_line():
    # a zero coefficient between columns 6 and 7 (an infinite step) must cut the line
    # in both directions: each side is filtered as if alone
    rng = np.random.default_rng(3)
    x = rng.random((3, 15))
    alpha = rng.uniform(0.3, 0.9, (3, 15))
    alpha[:, 7] = 0.0
    y = oracle.amf_rf_line_rows([x], alpha)[0]
    left = oracle.amf_rf_line_rows([x[:, :7]], alpha[:, :7])[0]
    right_alpha = alpha[:, 7:].copy()
    right = oracle.amf_rf_line_rows([x[:, 7:]], right_alpha)[0]
    assert np.array_equal(y[:, :7], left)
    assert np.array_equal(y[:, 7:], right)


def test_manifold_blur_does_not_cross_a_range_cliff():
    # a manifold that jumps by far more than sigma_r' between two columns gives a step
    # coefficient that underflows to zero: the blur on each side ignores the other
    H, W = 6, 12
    eta = np.zeros((H, W))
    eta[:, 5:] = 1e6
    x = _rand((H, W), 4)
    both = oracle.amf_blur([x], eta, 3.0, 0.1)[0]
    left = oracle.amf_blur([x[:, :5]], eta[:, :5], 3.0, 0.1)[0]
    right = oracle.amf_blur([x[:, 5:]], eta[:, 5:], 3.0, 0.1)[0]
    assert np.array_equal(both[:, :5], left)
    assert np.array_equal(both[:, 5:], right)


def test_range_off_is_the_separable_exponential_kernel():
    # sigma_r = inf: psi = 1, no children, every step d = 1; the two 1-D passes make
    # the kernel ((1 - a) / (1 + a))^2 a^(|dx| + |dy|) away from the borders
    H, W, sigma_s = 80, 80, 2.0
    p = _rand((H, W), 5)
    g = oracle.amf_filter(p, None, sigma_s, math.inf)
    a = math.exp(-math.sqrt(2.0) / sigma_s)
    c = ((1.0 - a) / (1.0 + a)) ** 2
    R = 34                       # a^35 ~ 1e-11
    i0, i1 = R + 1, H - R - 1
    ref = np.zeros((i1 - i0, i1 - i0))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            ref += c * a ** (abs(dx) + abs(dy)) * p[i0 + dy:i1 + dy, i0 + dx:i1 + dx]
    assert np.max(np.abs(g[i0:i1, i0:i1] - ref)) < 1e-9


def test_constant_field_passes_unchanged_and_outputs_stay_in_range():
    H, W = 24, 20
    q = _rand((H, W), 6) * 0.3
    c = np.full((H, W), 0.37)
    for guide in (None, q):
        g = oracle.amf_filter(c, guide, 3.0, 0.05)
        assert np.max(np.abs(g - 0.37)) < 1e-15
    p = _rand((H, W), 7) * 0.3
    for guide in (None, q):
        g = oracle.amf_filter(p, guide, 3.0, 0.05, height=3)
        assert g.min() >= p.min() - 1e-15 and g.max() <= p.max() + 1e-15


def test_clean_step_passes_unchanged():
    # two levels far apart in sigma_r: each side's manifold sits on its own level and
    # nothing leaks across (the BLF of Eq. (1) leaves such a field unchanged too)
    H, W = 20, 30
    p = np.zeros((H, W))
    p[:, 13:] = 1.0
    g = oracle.amf_filter(p, None, 4.0, 0.05)
    assert np.max(np.abs(g - p)) < 1e-9
    bl = oracle.bilateral_filter(p, None, 4.0, 0.05, 12)
    assert np.max(np.abs(bl - p)) < 1e-9


def test_tree_height_rule():
    assert oracle.amf_tree_height(12.0, 0.02) == 2     # floor(log2 12) - 1 = 2, ceil(1.96)
    assert oracle.amf_tree_height(16.0, 0.02) == 3
    assert oracle.amf_tree_height(64.0, 0.02) == 5
    assert oracle.amf_tree_height(1.0, 0.1) == 2       # clamped below
    assert oracle.amf_tree_height(12.0, math.inf) == 2
    assert oracle.amf_tree_height(1e5, 1e-4) == oracle.AMF_MAX_HEIGHT


def test_range_off_needs_one_manifold():
    p = _rand((16, 18), 8)
    _, mans = oracle.amf_filter(p, None, 3.0, math.inf, return_manifolds=True)
    assert len(mans) == 3 and np.all(np.isnan(mans[1])) and np.all(np.isnan(mans[2]))
    _, mans = oracle.amf_filter(p, None, 3.0, 0.05, height=3, return_manifolds=True)
    assert len(mans) == 7
    assert not np.all(np.isnan(mans[1]))


def test_normalised_range_equals_scaled_sigma_r():
    # scaling the range differences by 1/span is the filter with sigma_r * span, except for
    # the tree height, which reads sigma_r itself
    p = voronoi_image(24, 28, 9)
    p = oracle.grad_x(p)
    span = 0.8
    a = oracle.amf_filter(p, None, 4.0, 0.05, height=2, inv_span=1.0 / span)
    b = oracle.amf_filter(p, None, 4.0, float(np.float32(0.05)) * span, height=2)
    # sigma_r * span is rounded to FP32 inside amf_filter; compare loosely
    assert np.max(np.abs(a - b)) < 1e-6


@pytest.mark.parametrize("sigma_s,sigma_r", [(4.0, 0.05), (8.0, 0.05), (4.0, 0.2)])
def test_amf_approximates_the_bilateral_filter(sigma_s, sigma_r):
    # the AMF stands in for Eq. (1): on piecewise-smooth gradient fields it must sit far
    # closer to the exact filter than the unfiltered field does
    f = voronoi_image(96, 96, 5)
    p = oracle.grad_x(f)
    exact = oracle.bilateral_filter(p, None, sigma_s, sigma_r, oracle.default_radius(sigma_s))
    amf = oracle.amf_filter(p, None, sigma_s, sigma_r)
    rng2 = (p.max() - p.min()) ** 2
    psnr = lambda x: 10 * math.log10(rng2 / np.mean((x - exact) ** 2))
    assert psnr(amf) > psnr(p) + 7.0
    assert psnr(amf) > 38.0


def test_amf_ls_method_invariants():
    f = voronoi_image(32, 36, 10)
    u = oracle.smooth(f, 0.0, 3.0, 0.05, filter="amf")
    assert np.max(np.abs(u - f)) < 1e-14
    c = np.full((16, 20), 0.25)
    assert np.max(np.abs(oracle.smooth(c, 30.0, 3.0, 0.05, filter="amf") - c)) < 1e-14
    u = oracle.smooth(f, 20.0, 3.0, 0.05, filter="amf")
    assert abs(u.mean() - f.mean()) < 1e-13
    # the gradient fields AMF-LS hands to the solve are the filter's output
    _, gx, gy = oracle.smooth_channel(f, 20.0, 3.0, 0.05, filter="amf", return_fields=True)
    assert np.max(np.abs(gx - oracle.amf_filter(oracle.grad_x(f), None, 3.0, 0.05))) < 1e-15
    assert np.max(np.abs(gy - oracle.amf_filter(oracle.grad_y(f), None, 3.0, 0.05))) < 1e-15
