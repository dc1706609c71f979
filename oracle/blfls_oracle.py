"""FP64 CPU oracle for BLF-LS (Liu et al., "Embedding Bilateral Filter in Least
Squares for Efficient Edge-preserving Image Smoothing", arXiv 1812.07122).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow definition that the
GPU library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never calls it and
shares no code with it.

Notation (the paper calls the input g; here, as in the library, the input is f):
  f        input image, one channel, shape (H, W), float64
  p_x, p_y forward-difference gradient fields of f (Section II-B, Eq. (4) text)
  q_x, q_y the fields the range kernel compares: p itself (self-guided), the
           gradients of a guidance image (Section III-D, joint filtering), or the
           gradients of the previous output (Section III-D, rolling guidance)
  g_x, g_y the bilateral-filtered fields, g = BLF(p) (Eq. (1), Eq. (7))
  u        output, the minimiser of Eq. (7), given by Eq. (8)

Readings taken where the paper is silent (each one is listed in the design notes):
  * boundaries are circular everywhere: the Fourier solve of Eq. (6)/(8) only
    diagonalises circulant difference operators, so the gradients, the filter
    window and the solve all wrap;
  * the window is the square of Chebyshev radius r around s, r = ceil(3 sigma_s)
    unless given; a window wider than the image sums the periodic copies offset
    by offset, and the spatial weight uses the offset, not the wrapped distance;
  * both kernels of Eq. (1) are exp(-x^2 / (2 sigma^2)); spatial distance is
    Euclidean over the offset (dx, dy);
  * each field is filtered on its own, the range kernel comparing scalar values
    of the same axis (Eq. (7): f_BLF applied to each gradient field);
  * colour channels are processed independently;
  * sigma_r = inf switches the range kernel off (weight 1);
  * the optional normalisation of the experiments section (images and gradients
    mapped to [0, 1] before smoothing and back after) is applied per channel and
    per field, literally, when ``normalize=True``;
  * iterations > 1 follow the rolling-guidance extension: iteration k filters
    the input's gradients with range weights from the gradients of u_{k-1}, and
    u_0 is the guidance image if one is given (optionally Gaussian-smoothed
    first, sigma_guide > 0), else the input itself.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "default_radius",
    "grad_x", "grad_y", "grad_x_adjoint", "grad_y_adjoint",
    "bilateral_filter", "bilateral_filter_bruteforce", "bilateral_filter_at",
    "difference_otf", "ls_solve", "blfls_solve",
    "dense_difference_matrices", "dense_blfls_solve",
    "gaussian_blur", "smooth", "smooth_channel",
]


def default_radius(sigma_s: float) -> int:
    """Window radius when none is given: ceil(3 sigma_s)."""
    return int(math.ceil(3.0 * float(sigma_s)))


# ---------------------------------------------------------------------------
# Difference operators D_x, D_y and their adjoints D_x^T, D_y^T
# (Section II-B: forward differences; their transposes are the backward ones)
# ---------------------------------------------------------------------------

def grad_x(f: np.ndarray) -> np.ndarray:
    """(D_x f)(i, j) = f(i, j+1) - f(i, j), indices mod W."""
    return np.roll(f, -1, axis=-1) - f


def grad_y(f: np.ndarray) -> np.ndarray:
    """(D_y f)(i, j) = f(i+1, j) - f(i, j), indices mod H."""
    return np.roll(f, -1, axis=-2) - f


def grad_x_adjoint(v: np.ndarray) -> np.ndarray:
    """(D_x^T v)(i, j) = v(i, j-1) - v(i, j), indices mod W."""
    return np.roll(v, 1, axis=-1) - v


def grad_y_adjoint(v: np.ndarray) -> np.ndarray:
    """(D_y^T v)(i, j) = v(i-1, j) - v(i, j), indices mod H."""
    return np.roll(v, 1, axis=-2) - v


# ---------------------------------------------------------------------------
# Bilateral filter, Eq. (1)
# ---------------------------------------------------------------------------

def bilateral_filter(p: np.ndarray, q: np.ndarray | None, sigma_s: float, sigma_r: float,
                     radius: int) -> np.ndarray:
    """Eq. (1) on one 2-D field p, range weights from the field q (q=None: q=p).

    out(s) = sum_d G_s(d) G_r(q(s+d) - q(s)) p(s+d) / sum_d G_s(d) G_r(q(s+d) - q(s)),
    summed over every offset d = (dy, dx) of the square [-r, r]^2, s+d wrapping.
    G_s(d) = exp(-(dx^2 + dy^2) / (2 sigma_s^2)); G_r(t) = exp(-t^2 / (2 sigma_r^2)),
    or 1 when sigma_r is infinite.
    """
    p = np.asarray(p, dtype=np.float64)
    q = p if q is None else np.asarray(q, dtype=np.float64)
    r = int(radius)
    num = np.zeros_like(p)
    den = np.zeros_like(p)
    range_on = math.isfinite(sigma_r)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            # value at s + d for every s: shift the plane by -d
            p_t = np.roll(p, (-dy, -dx), axis=(-2, -1))
            w = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma_s * sigma_s))
            if range_on:
                q_t = np.roll(q, (-dy, -dx), axis=(-2, -1))
                w = w * np.exp(-((q_t - q) ** 2) / (2.0 * sigma_r * sigma_r))
            num += w * p_t
            den += w
    return num / den


def bilateral_filter_bruteforce(p, q, sigma_s, sigma_r, radius):
    """Eq. (1) by explicit loops over pixels and window taps (tiny inputs only)."""
    p = np.asarray(p, dtype=np.float64)
    q = p if q is None else np.asarray(q, dtype=np.float64)
    H, W = p.shape
    out = np.empty_like(p)
    for i in range(H):
        for j in range(W):
            num = 0.0
            den = 0.0
            for dy in range(-radius, radius + 1):
                for dx in range(-radius, radius + 1):
                    ti, tj = (i + dy) % H, (j + dx) % W
                    ws = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma_s ** 2))
                    if math.isfinite(sigma_r):
                        wr = math.exp(-(q[ti, tj] - q[i, j]) ** 2 / (2.0 * sigma_r ** 2))
                    else:
                        wr = 1.0
                    num += ws * wr * p[ti, tj]
                    den += ws * wr
            out[i, j] = num / den
    return out


def bilateral_filter_at(p, q, sigma_s, sigma_r, radius, rows, cols):
    """Eq. (1) evaluated only at the pixels (rows[k], cols[k]); same definition as
    ``bilateral_filter`` (circular window, periodic summation), vectorised over
    the listed pixels instead of over the image, for checks on large images."""
    p = np.asarray(p, dtype=np.float64)
    q = p if q is None else np.asarray(q, dtype=np.float64)
    H, W = p.shape
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    r = int(radius)
    d = np.arange(-r, r + 1)
    ti = (rows[:, None, None] + d[None, :, None]) % H        # (n, 2r+1, 1) window rows
    tj = (cols[:, None, None] + d[None, None, :]) % W        # (n, 1, 2r+1) window columns
    w = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * sigma_s * sigma_s))[None]
    if math.isfinite(sigma_r):
        qs = q[rows, cols][:, None, None]
        w = w * np.exp(-((q[ti, tj] - qs) ** 2) / (2.0 * sigma_r * sigma_r))
    return np.sum(w * p[ti, tj], axis=(1, 2)) / np.sum(w, axis=(1, 2))


# ---------------------------------------------------------------------------
# Fourier-domain least-squares solves, Eq. (6) and Eq. (8)
# ---------------------------------------------------------------------------

def difference_otf(H: int, W: int):
    """F(1), F(d_x), F(d_y): DFTs of the delta and of the two difference kernels.

    Applying D_x is circular convolution with the image kx having kx[0,0] = -1 and
    kx[0,W-1] = +1 (so that (kx * f)(i,j) = f(i,j+1) - f(i,j)); likewise ky.
    """
    delta = np.zeros((H, W))
    delta[0, 0] = 1.0
    kx = np.zeros((H, W))
    kx[0, 0] = -1.0
    kx[0, (W - 1) % W] += 1.0
    ky = np.zeros((H, W))
    ky[0, 0] = -1.0
    ky[(H - 1) % H, 0] += 1.0
    return np.fft.fft2(delta), np.fft.fft2(kx), np.fft.fft2(ky)


def ls_solve(f: np.ndarray, lam: float) -> np.ndarray:
    """Eq. (6): u = F^-1( F(f) / (F(1) + lam (conj(F(dx)) F(dx) + conj(F(dy)) F(dy))) )."""
    f = np.asarray(f, dtype=np.float64)
    F1, Fx, Fy = difference_otf(*f.shape)
    den = F1 + lam * (np.conj(Fx) * Fx + np.conj(Fy) * Fy)
    return np.real(np.fft.ifft2(np.fft.fft2(f) / den))


def blfls_solve(f: np.ndarray, gx: np.ndarray, gy: np.ndarray, lam: float) -> np.ndarray:
    """Eq. (8), term by term:

    u = F^-1( (F(f) + lam sum_* conj(F(d_*)) F(g_*)) / (F(1) + lam sum_* conj(F(d_*)) F(d_*)) ).
    """
    f = np.asarray(f, dtype=np.float64)
    F1, Fx, Fy = difference_otf(*f.shape)
    num = np.fft.fft2(f) + lam * (np.conj(Fx) * np.fft.fft2(gx) + np.conj(Fy) * np.fft.fft2(gy))
    den = F1 + lam * (np.conj(Fx) * Fx + np.conj(Fy) * Fy)
    return np.real(np.fft.ifft2(num / den))


def dense_difference_matrices(H: int, W: int):
    """Explicit (HW x HW) matrices of D_x, D_y on row-major flattened images."""
    n = H * W
    Mx = np.zeros((n, n))
    My = np.zeros((n, n))
    for i in range(H):
        for j in range(W):
            s = i * W + j
            Mx[s, i * W + (j + 1) % W] += 1.0
            Mx[s, s] -= 1.0
            My[s, ((i + 1) % H) * W + j] += 1.0
            My[s, s] -= 1.0
    return Mx, My


def dense_blfls_solve(f, gx, gy, lam):
    """The normal equations of Eq. (7) solved directly (tiny images only):

    (I + lam (Mx^T Mx + My^T My)) u = f + lam (Mx^T gx + My^T gy).
    """
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    Mx, My = dense_difference_matrices(H, W)
    A = np.eye(H * W) + lam * (Mx.T @ Mx + My.T @ My)
    b = f.ravel() + lam * (Mx.T @ np.ravel(gx) + My.T @ np.ravel(gy))
    return np.linalg.solve(A, b).reshape(H, W)


# ---------------------------------------------------------------------------
# The method: BLF on the gradients, then the Eq. (8) solve (Section III-A),
# with the extensions of Section III-D
# ---------------------------------------------------------------------------

def gaussian_blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Circular Gaussian smoothing, radius ceil(3 sigma), normalised weights."""
    img = np.asarray(img, dtype=np.float64)
    if sigma <= 0:
        return img.copy()
    r = default_radius(sigma)
    acc = np.zeros_like(img)
    tot = 0.0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
            acc += w * np.roll(img, (-dy, -dx), axis=(-2, -1))
            tot += w
    return acc / tot


def _normalise_unit(v: np.ndarray):
    """Map v affinely onto [0, 1]; returns (mapped, lo, span).  A constant v maps to 0."""
    lo = float(v.min())
    span = float(v.max()) - lo
    if span > 0.0:
        return (v - lo) / span, lo, span
    return v - lo, lo, 1.0


def _filter_field(p, q, sigma_s, sigma_r, radius, normalize):
    if not normalize:
        return bilateral_filter(p, q, sigma_s, sigma_r, radius)
    # experiments section: fields taken to [0, 1], filtered, then mapped back
    pn, plo, pspan = _normalise_unit(p)
    qn = pn if q is None else _normalise_unit(q)[0]
    return bilateral_filter(pn, qn, sigma_s, sigma_r, radius) * pspan + plo


def smooth_channel(f, lam, sigma_s, sigma_r, radius=-1, iterations=1, guide=None,
                   normalize=False, sigma_guide=0.0, return_fields=False):
    """BLF-LS on one channel (Section III-A two-step procedure, Section III-D extensions).

    Step 1 filters p_x, p_y with Eq. (1); step 2 solves Eq. (8).  ``guide`` switches
    to joint filtering; ``iterations`` > 1 is rolling guidance.
    """
    f = np.asarray(f, dtype=np.float64)
    r = default_radius(sigma_s) if radius is None or radius < 0 else int(radius)
    lo, span = 0.0, 1.0
    if normalize:
        f, lo, span = _normalise_unit(f)
    px, py = grad_x(f), grad_y(f)
    if guide is not None:
        h = np.asarray(guide, dtype=np.float64)
        if normalize:
            h = _normalise_unit(h)[0]
        if sigma_guide > 0:
            h = gaussian_blur(h, sigma_guide)
        prev = h
    elif sigma_guide > 0:
        prev = gaussian_blur(f, sigma_guide)
    else:
        prev = None
    u = f
    gx = gy = None
    for _ in range(int(iterations)):
        if prev is None:
            qx = qy = None
        else:
            qx, qy = grad_x(prev), grad_y(prev)
        gx = _filter_field(px, qx, sigma_s, sigma_r, r, normalize)
        gy = _filter_field(py, qy, sigma_s, sigma_r, r, normalize)
        u = blfls_solve(f, gx, gy, lam)
        prev = u
    out = u * span + lo
    if return_fields:
        return out, gx * span, gy * span
    return out


def smooth(f, lam, sigma_s, sigma_r, radius=-1, iterations=1, guide=None, normalize=False,
           sigma_guide=0.0):
    """BLF-LS on a (H, W) or (C, H, W) image; channels are independent."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 2:
        return smooth_channel(f, lam, sigma_s, sigma_r, radius, iterations, guide, normalize,
                              sigma_guide)
    g = None if guide is None else np.asarray(guide, dtype=np.float64)
    outs = []
    for c in range(f.shape[0]):
        gc = None if g is None else (g[c] if g.ndim == 3 else g)
        outs.append(smooth_channel(f[c], lam, sigma_s, sigma_r, radius, iterations, gc,
                                   normalize, sigma_guide))
    return np.stack(outs)
