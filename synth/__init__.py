"""Seeded synthetic images shaped like the paper's smoothing workloads.

The paper evaluates on photographs (detail enhancement, HDR, flash/no-flash,
texture and clip-art images) that are not available here.  These generators
stand in for them: piecewise-constant regions (strong edges the smoothing must
keep), a low-amplitude periodic texture and fine noise (detail it must remove).

This module draws random numbers and lays out arrays only.  It holds none of
the method's arithmetic, so both the FP64 oracle and the GPU path can take
their inputs from it without sharing any part of the computation.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "voronoi_image",
    "voronoi_rgb",
    "joint_pair",
    "config_seed",
    "quantized",
]

N_SITES = 32
TEXTURE_AMP = 0.05
TEXTURE_PERIOD = 8.0
NOISE_SIGMA = 0.02


def config_seed(config: int, channel: int = 0) -> int:
    """Seed of one channel of a workload: 1000*config + channel."""
    return 1000 * int(config) + int(channel)


def voronoi_image(height: int, width: int, seed: int) -> np.ndarray:
    """One grayscale image, float64, shape (height, width), values in [0, 1].

    Recipe (draw order fixed, one ``numpy.random.default_rng(seed)``):
      1. 32 sites uniform on [0, W) x [0, H)  (x then y per site);
      2. one level U[0, 1) per site;
      3. one texture angle theta ~ U[0, pi);
      4. noise N(0, 0.02^2) per pixel, row-major.
    Pixel (i, j) has coordinates x = j, y = i.  Its label is the nearest site
    in Euclidean distance (ties to the lower site index).  Value = level +
    0.05 sin(2 pi (x cos(theta) + y sin(theta)) / 8) + noise, clipped to [0, 1].
    """
    if height < 1 or width < 1:
        raise ValueError("image sides must be positive")
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, size=(N_SITES, 2)) * np.array([width, height], dtype=np.float64)
    levels = rng.uniform(0.0, 1.0, size=N_SITES)
    theta = rng.uniform(0.0, np.pi)
    noise = rng.normal(0.0, NOISE_SIGMA, size=(height, width))

    ys = np.arange(height, dtype=np.float64)
    xs = np.arange(width, dtype=np.float64)
    labels = np.empty((height, width), dtype=np.int64)
    # nearest site, a band of rows at a time to bound memory
    band = max(1, (1 << 22) // (width * N_SITES))
    for i0 in range(0, height, band):
        yy = ys[i0:i0 + band, None, None]
        d2 = (xs[None, :, None] - sites[None, None, :, 0]) ** 2 + (yy - sites[None, None, :, 1]) ** 2
        labels[i0:i0 + band] = np.argmin(d2, axis=2)
    img = levels[labels]
    X, Y = np.meshgrid(xs, ys)
    img = img + TEXTURE_AMP * np.sin(2.0 * np.pi * (X * np.cos(theta) + Y * np.sin(theta)) / TEXTURE_PERIOD)
    img = img + noise
    return np.clip(img, 0.0, 1.0)


def voronoi_rgb(height: int, width: int, config: int, channels: int = 3) -> np.ndarray:
    """A (channels, height, width) float64 image, channel c drawn with seed 1000*config + c."""
    return np.stack([voronoi_image(height, width, config_seed(config, c)) for c in range(channels)])


def joint_pair(height: int, width: int, index: int, noise_sigma: float = 0.05):
    """A (target, guidance) pair for joint filtering, both float64 (height, width).

    The guidance is the generator above with seed 4000+index; the target is the
    guidance plus N(0, noise_sigma^2) noise drawn with seed 4500+index, not clipped.
    """
    guide = voronoi_image(height, width, 4000 + int(index))
    rng = np.random.default_rng(4500 + int(index))
    target = guide + rng.normal(0.0, noise_sigma, size=(height, width))
    return target, guide


def quantized(img: np.ndarray, levels: int = 64) -> np.ndarray:
    """img rounded to the nearest multiple of 1/levels (an image stored with a few bits per
    sample).  With levels a power of two every sample, every difference of samples and
    every small multiple of those is exact in binary floating point, FP32 included."""
    return np.round(np.asarray(img, dtype=np.float64) * levels) / levels
