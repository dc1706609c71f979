"""Pins of the oracle's log-domain tone mapping (CPU only).

The experiments section tone-maps HDR images by splitting log intensity into
a BLF-LS base and a detail layer, compressing the base and recombining.  Pinned
by what that construction fixes: the compressed base spans exactly the target
contrast with its maximum at 0, the detail layer passes unchanged, colour
ratios are kept, lambda = 0 (base = log intensity) is a global power law of the
intensity, and a uniformly scaled input gives the same output.
"""
import math

import numpy as np

import oracle
from synth import voronoi_rgb


def _hdr(H, W, seed):
    # linear radiance over about four decades: 10^(4 v - 2) per channel
    v = voronoi_rgb(H, W, seed)
    return 10.0 ** (4.0 * v - 2.0)


def _intensity(rgb):
    return np.maximum((20.0 * rgb[0] + 40.0 * rgb[1] + rgb[2]) / 61.0, oracle.TM_FLOOR)


def test_tonemap_compresses_the_base_to_the_target_contrast():
    rgb = _hdr(40, 48, 1)
    lam, ss, sr = 20.0, 3.0, 0.05
    out = oracle.tonemap(rgb, lam, ss, sr, contrast=5.0, normalize=True)
    L = np.log10(_intensity(rgb))
    base = oracle.smooth(L, lam, ss, sr, normalize=True)
    Lout = np.log10(_intensity(out))
    comp = Lout - (L - base)                   # remove the detail layer
    assert abs(comp.max()) < 1e-12
    assert abs((comp.max() - comp.min()) - math.log10(5.0)) < 1e-12
    # the compressed base is an affine image of the base
    cf = math.log10(5.0) / (base.max() - base.min())
    assert np.max(np.abs(comp - (base - base.max()) * cf)) < 1e-12


def test_tonemap_keeps_colour_ratios():
    rgb = _hdr(24, 30, 2)
    out = oracle.tonemap(rgb, 20.0, 3.0, 0.05, normalize=True)
    assert np.max(np.abs(out[0] / out[1] - rgb[0] / rgb[1])) < 1e-9
    assert np.max(np.abs(out[2] / out[1] - rgb[2] / rgb[1])) < 1e-9


def test_tonemap_without_smoothing_is_a_power_law():
    # lambda = 0: base = log intensity, no detail; I_out = (I / I_max)^cf
    rgb = _hdr(20, 24, 3)
    out = oracle.tonemap(rgb, 0.0, 3.0, 0.05, contrast=10.0)
    I = _intensity(rgb)
    cf = 1.0 / (math.log10(I.max()) - math.log10(I.min()))
    assert np.max(np.abs(_intensity(out) - (I / I.max()) ** cf)) < 1e-12


def test_tonemap_ignores_exposure():
    rgb = _hdr(24, 30, 4)
    a = oracle.tonemap(rgb, 20.0, 3.0, 0.05, normalize=True)
    b = oracle.tonemap(rgb * 37.0, 20.0, 3.0, 0.05, normalize=True)
    assert np.max(np.abs(a - b)) < 1e-9
