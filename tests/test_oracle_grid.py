"""Pins of the oracle's bilateral-grid approximation of Eq. (1) (CPU only).

The grid filter is pinned to its definition written as one sum per output
(pixel loops over the periodic extension), to the exact filter of Eq. (1) in
the case where the two coincide (one pixel per cell, range term off: both are
the normalised periodic Gaussian of radius 2), and to invariants: constants
pass unchanged, the output is linear in the filtered signal for a fixed
guide, and shifting the image by whole cells shifts the output.
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image


def _rand(shape, seed):
    return np.random.default_rng(seed).random(shape)


@pytest.mark.parametrize("H,W,ss,sr", [
    (5, 7, 1.0, 0.3),
    (6, 9, 2.0, 0.2),
    (8, 5, 3.0, 0.5),
    (4, 6, 2.0, math.inf),   # one range bin
    (6, 6, 2.0, 0.01),       # more bins than the cap: the range cell widens
])
def test_grid_matches_pixel_sums(H, W, ss, sr):
    p, q = _rand((H, W), 1), _rand((H, W), 2)
    for guide in (None, q):
        a = oracle.grid_filter(p, guide, ss, sr)
        b = oracle.grid_filter_bruteforce(p, guide, ss, sr)
        assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("ss", [0.75, 1.0, 1.25])
def test_grid_with_unit_cells_and_no_range_is_the_exact_gaussian(ss):
    # s = 1: every pixel is its own cell, the slice reads cells exactly; with one
    # range bin the grid filter is the normalised periodic Gaussian of radius 2,
    # which is the exact filter of Eq. (1) with the range kernel off and r = 2
    p = _rand((12, 15), 3)
    g = oracle.grid_filter(p, None, ss, math.inf)
    ref = oracle.bilateral_filter(p, None, ss, math.inf, 2)
    assert np.max(np.abs(g - ref)) < 1e-13


def test_grid_keeps_constants_and_is_linear():
    c = np.full((10, 12), -0.25)
    assert np.max(np.abs(oracle.grid_filter(c, None, 3.0, 0.1) - c)) < 1e-15
    q = _rand((10, 12), 4)
    p1, p2 = _rand((10, 12), 5), _rand((10, 12), 6)
    lhs = oracle.grid_filter(3.0 * p1 + 0.5 * p2, q, 3.0, 0.1)
    rhs = 3.0 * oracle.grid_filter(p1, q, 3.0, 0.1) + 0.5 * oracle.grid_filter(p2, q, 3.0, 0.1)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_grid_commutes_with_whole_cell_shifts():
    p = _rand((12, 18), 7)
    q = _rand((12, 18), 8)
    s = oracle.grid_cell(3.0)
    g = oracle.grid_filter(p, q, 3.0, 0.2)
    gs = oracle.grid_filter(np.roll(p, (s, 2 * s), (0, 1)), np.roll(q, (s, 2 * s), (0, 1)), 3.0, 0.2)
    assert np.max(np.abs(np.roll(g, (s, 2 * s), (0, 1)) - gs)) < 1e-13


def test_grid_normalisation_is_a_range_rescale():
    g = _rand((12, 14), 9)
    g = (g - g.min()) / (g.max() - g.min()) * 4.0   # span 4: exact FP32 scaling
    p = _rand((12, 14), 10)
    a = oracle.grid_filter(p, g, 3.0, 0.2, np.float32(0.25))
    b = oracle.grid_filter(p, g, 3.0, 0.8)
    assert np.max(np.abs(a - b)) < 1e-15


def test_grid_ls_special_cases():
    f = voronoi_image(24, 32, 21)
    assert np.max(np.abs(oracle.smooth(f, 0.0, 4.0, 0.05, filter="grid") - f)) < 1e-14
    c = np.full((16, 20), 0.3)
    assert np.max(np.abs(oracle.smooth(c, 50.0, 4.0, 0.05, filter="grid") - c)) < 1e-14
    u = oracle.smooth(f, 30.0, 4.0, 0.05, filter="grid")
    assert abs(u.mean() - f.mean()) < 1e-14


def test_grid_approximates_the_exact_filter():
    # the approximation the paper's experiments rely on: on a Voronoi field the
    # grid result stays close to the exact windowed filter (error well below the
    # field's own variation)
    f = voronoi_image(64, 64, 22)
    px = oracle.grad_x(f)
    exact = oracle.bilateral_filter(px, None, 4.0, 0.05, 12)
    approx = oracle.grid_filter(px, None, 4.0, 0.05)
    assert np.sqrt(np.mean((approx - exact) ** 2)) < 0.25 * np.sqrt(np.mean((px - exact) ** 2))
