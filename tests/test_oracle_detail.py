"""Pins of the oracle's detail enhancement (CPU only).

The experiments section enhances detail by boosting the detail layer f - u
(input minus smoothed output) m times over the smoothed base: u + m (f - u).
Pinned by what that definition fixes: m = 0 is the smoothed image, m = 1 the
input, the result is affine in m, the base-plus-detail split holds, and the
boost acts after the last rolling-guidance iteration.
"""
import numpy as np

import oracle
from synth import voronoi_image


def test_detail_gain_endpoints_and_affinity():
    f = voronoi_image(24, 30, 3)
    u = oracle.smooth(f, 20.0, 3.0, 0.1)
    assert np.array_equal(oracle.smooth(f, 20.0, 3.0, 0.1, detail_gain=0.0), u)
    assert np.max(np.abs(oracle.smooth(f, 20.0, 3.0, 0.1, detail_gain=1.0) - f)) < 1e-14
    e5 = oracle.smooth(f, 20.0, 3.0, 0.1, detail_gain=5.0)
    e2 = oracle.smooth(f, 20.0, 3.0, 0.1, detail_gain=2.0)
    # affine in m: e(m) = u + m (f - u), so e5 - e2 = 3 (f - u)
    assert np.max(np.abs((e5 - e2) - 3.0 * (f - u))) < 1e-13
    # the enhanced image keeps the smoothed base: e - m (f - u) = u
    assert np.max(np.abs(e5 - 5.0 * (f - u) - u)) < 1e-13


def test_detail_gain_applies_after_the_last_iteration_only():
    f = voronoi_image(20, 24, 4)
    u3 = oracle.smooth(f, 20.0, 3.0, 0.05, iterations=3)
    e3 = oracle.smooth(f, 20.0, 3.0, 0.05, iterations=3, detail_gain=5.0)
    assert np.max(np.abs(e3 - (u3 + 5.0 * (f - u3)))) < 1e-13


def test_detail_gain_with_normalisation_is_in_input_units():
    f = voronoi_image(20, 24, 5) * 0.5 + 0.2
    u = oracle.smooth(f, 20.0, 3.0, 0.3, normalize=True)
    e = oracle.smooth(f, 20.0, 3.0, 0.3, normalize=True, detail_gain=5.0)
    assert np.max(np.abs(e - (u + 5.0 * (f - u)))) < 1e-13
