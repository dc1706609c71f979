"""Pins of the oracle's NC filter and NC-LS (CPU only).

NC-LS (Section III-D) embeds the normalized-convolution filter of the domain
transform in place of the BLF.  These tests pin the oracle's filter to what its
definition and elementary mathematics fix: pixel-by-pixel loops, the variance
identity of the iteration schedule, plain iterated box filters when the range
term is off, constants and clean steps that must pass unchanged, linearity in
the filtered signal, mirror symmetry, and the method-level invariants shared
with BLF-LS (lambda = 0, constant image, mean preservation).
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image


def _rand(shape, seed):
    return np.random.default_rng(seed).random(shape)


@pytest.mark.parametrize("H,W,sigma_s,sigma_r,n_iter", [
    (5, 7, 2.0, 0.3, 3),
    (6, 6, 3.0, 0.05, 3),
    (1, 9, 4.0, 0.2, 2),
    (8, 1, 4.0, 0.2, 1),
    (4, 5, 12.0, 0.5, 3),   # boxes wider than the image
])
def test_nc_matches_pixel_loops(H, W, sigma_s, sigma_r, n_iter):
    p = _rand((H, W), 1)
    q = _rand((H, W), 2)
    for guide in (None, q):
        a = oracle.nc_filter(p, guide, sigma_s, sigma_r, n_iter)
        b = oracle.nc_filter_bruteforce(p, guide, sigma_s, sigma_r, n_iter)
        assert np.max(np.abs(a - b)) < 1e-14


@pytest.mark.parametrize("n_iter", [1, 2, 3, 5])
def test_nc_schedule_variances_sum_to_sigma_s_squared(n_iter):
    sigma_s = 7.5
    radii = oracle.nc_schedule(sigma_s, n_iter)
    assert len(radii) == n_iter
    # a box of half-width r has variance r^2 / 3; the passes' variances add up
    assert abs(sum(r * r / 3.0 for r in radii) - sigma_s ** 2) < 1e-9
    # each box halves the previous one's width
    for r0, r1 in zip(radii, radii[1:]):
        assert abs(r0 / r1 - 2.0) < 1e-12
    if n_iter == 1:
        assert abs(radii[0] - math.sqrt(3.0) * sigma_s) < 1e-12


def _box_clipped(F, rad, axis):
    """Mean over the pixels within `rad` of each pixel along `axis`, clipped at the borders
    (cumulative sums; independent of the oracle's loops)."""
    F = np.moveaxis(np.asarray(F, dtype=np.float64), axis, -1)
    n = F.shape[-1]
    c = np.concatenate([np.zeros(F.shape[:-1] + (1,)), np.cumsum(F, axis=-1)], axis=-1)
    idx = np.arange(n)
    lo = np.maximum(idx - rad, 0)
    hi = np.minimum(idx + rad, n - 1)
    out = (c[..., hi + 1] - c[..., lo]) / (hi - lo + 1)
    return np.moveaxis(out, -1, axis)


def test_nc_without_range_term_is_iterated_box_filtering():
    p = _rand((23, 31), 3)
    sigma_s = 4.0
    out = oracle.nc_filter(p, None, sigma_s, math.inf, 3)
    ref = p
    for r in oracle.nc_schedule(sigma_s, 3):
        rad = int(math.floor(float(np.float32(r))))  # increments are exactly 1
        ref = _box_clipped(ref, rad, 1)
        ref = _box_clipped(ref, rad, 0)
    assert np.max(np.abs(out - ref)) < 1e-13


def test_nc_keeps_constants_and_clean_steps():
    c = np.full((9, 13), 0.375)
    assert np.max(np.abs(oracle.nc_filter(c, None, 3.0, 0.1) - c)) < 1e-15
    # a step whose jump costs more transformed distance than the widest box:
    # no window crosses it, so each side is a constant and passes unchanged
    step = np.zeros((10, 16))
    step[:, 8:] = 0.5
    step[5:, :] += 0.25
    out = oracle.nc_filter(step, None, 3.0, 0.01)
    assert np.max(np.abs(out - step)) < 1e-15


def test_nc_is_linear_in_the_filtered_signal():
    q = _rand((12, 17), 4)
    p1, p2 = _rand((12, 17), 5), _rand((12, 17), 6)
    lhs = oracle.nc_filter(2.0 * p1 - 0.5 * p2, q, 3.0, 0.2)
    rhs = 2.0 * oracle.nc_filter(p1, q, 3.0, 0.2) - 0.5 * oracle.nc_filter(p2, q, 3.0, 0.2)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_nc_mirror_symmetry():
    p = _rand((11, 14), 7)
    q = _rand((11, 14), 8)
    out = oracle.nc_filter(p, q, 2.5, 0.15)
    flipped = oracle.nc_filter(p[::-1, ::-1].copy(), q[::-1, ::-1].copy(), 2.5, 0.15)
    assert np.max(np.abs(flipped[::-1, ::-1] - out)) < 1e-13


def test_nc_normalisation_is_a_range_rescale():
    # a guide field whose span is a power of two: dividing the differences by it
    # is exact in FP32, so the normalised filter equals the raw filter with
    # sigma_r times the span, bit for bit in its decisions
    g = _rand((14, 18), 9)
    g = (g - g.min()) / (g.max() - g.min()) * 4.0
    p = _rand((14, 18), 10)
    inv = np.float32(0.25)
    a = oracle.nc_filter(p, g, 3.0, 0.05, 3, inv)
    b = oracle.nc_filter(p, g, 3.0, 0.05 * 4.0, 3)
    assert np.max(np.abs(a - b)) < 1e-15


def test_ncls_special_cases():
    f = voronoi_image(24, 32, 11)
    # lambda = 0 returns the input; a constant image is unchanged; the mean is kept
    assert np.max(np.abs(oracle.smooth(f, 0.0, 3.0, 0.05, filter="nc") - f)) < 1e-14
    c = np.full((16, 20), 0.3)
    assert np.max(np.abs(oracle.smooth(c, 50.0, 3.0, 0.05, filter="nc") - c)) < 1e-14
    u = oracle.smooth(f, 30.0, 3.0, 0.05, filter="nc")
    assert abs(u.mean() - f.mean()) < 1e-14
    # the solve of Eq. (8) with the NC-filtered fields: same normal-equation residual
    _, gx, gy = oracle.smooth_channel(f, 30.0, 3.0, 0.05, filter="nc", return_fields=True)
    assert np.max(np.abs(oracle.blfls_solve(f, gx, gy, 30.0) - u)) < 1e-12


def test_ncls_joint_with_itself_equals_self_guided():
    f = voronoi_image(20, 28, 12)
    a = oracle.smooth(f, 20.0, 3.0, 0.05, filter="nc")
    b = oracle.smooth(f, 20.0, 3.0, 0.05, guide=f, filter="nc")
    assert np.max(np.abs(a - b)) < 1e-15


def test_ncls_smooths_more_with_larger_sigmas():
    # Section III-C: larger sigma_s and sigma_r smooth the gradients more
    f = voronoi_image(32, 32, 13)

    def tv(u):
        return np.abs(oracle.grad_x(u)).sum() + np.abs(oracle.grad_y(u)).sum()

    t_small = tv(oracle.smooth(f, 20.0, 2.0, 0.02, filter="nc"))
    t_big = tv(oracle.smooth(f, 20.0, 6.0, 0.2, filter="nc"))
    assert t_big < t_small < tv(f)
