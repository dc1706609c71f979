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
  * NC-LS (Section III-D) replaces the BLF by the normalized-convolution filter
    of the domain transform on the same fields and guides; its borders do not
    wrap and it runs three iterations (see the NC section below);
  * AMF-LS (Section III-D) replaces it by the adaptive-manifold filter, whose
    recursive passes start at the borders (see the AMF section below);
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
    "nc_schedule", "nc_increments", "nc_box_pass", "nc_filter", "nc_filter_bruteforce",
    "nc_decision_margin",
    "GRID_PAD", "GRID_ZMAX", "grid_cell", "grid_range", "grid_bin_margin", "grid_filter",
    "grid_filter_bruteforce",
    "AMF_MAX_HEIGHT", "AMF_TAU", "amf_tree_height", "amf_rf_line_rows", "amf_blur",
    "amf_filter", "amf_filter_dense",
    "TM_FLOOR", "tonemap",
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
# Normalized-convolution filter of the domain transform (Section III-D: NC-LS
# embeds it in place of the BLF; its definition is Gastal and Oliveira,
# "Domain Transform for Edge-Aware Image and Video Processing", 2011)
# ---------------------------------------------------------------------------
#
# Along a row, the domain transform maps pixel j to ct(j) = sum_{t <= j} d(t)
# with increments d(t) = 1 + (sigma_s / sigma_r) |q(t) - q(t-1)|, q the guide
# field; the NC filter replaces each value by the mean of the values whose
# transformed coordinate lies within r of its own (a box in the transformed
# domain), and iterates horizontal then vertical passes with shrinking boxes.
# Readings (listed in the design notes): the filtered signal is the gradient
# field and the guide is the field itself or the guide image's field of the
# same axis (as for the BLF); windows stop at the image borders (the filter
# is defined on a finite signal; only the solve is circular); three
# iterations.  Everything here is FP64, window membership included: the
# transformed distance between j and m is the sum of the increments between
# them, and m is in j's window when that sum is at most r.  Membership is a
# discontinuous function of the guide, so ``nc_decision_margin`` reports how
# far the closest decision lies from its threshold; a lower-precision
# implementation reproduces these windows exactly when its own rounding of the
# distances stays below that margin.

def nc_schedule(sigma_s: float, n_iter: int = 3):
    """Box radii of the n_iter passes: sigma_k = sigma_s sqrt(3) 2^(n-k) / sqrt(4^n - 1)
    (the iterated boxes' variances sum to sigma_s^2) and r_k = sqrt(3) sigma_k (a box of
    half-width r has variance r^2 / 3)."""
    n = int(n_iter)
    out = []
    for k in range(1, n + 1):
        sk = float(sigma_s) * math.sqrt(3.0) * 2.0 ** (n - k) / math.sqrt(4.0 ** n - 1.0)
        out.append(math.sqrt(3.0) * sk)
    return out


def nc_increments(q: np.ndarray, a: float, inv_span=None):
    """Domain-transform increments of the guide field q: dh[i, j] = 1 + a |q[i, j] - q[i, j-1]|
    (column 0 unused) and dv[i, j] = 1 + a |q[i, j] - q[i-1, j]| (row 0 unused); with inv_span
    (normalised fields) the term is a |dq| inv_span."""
    q = np.asarray(q, dtype=np.float64)
    scale = float(a) * (1.0 if inv_span is None else float(inv_span))
    dh = np.ones_like(q)
    dv = np.ones_like(q)
    dh[:, 1:] = 1.0 + scale * np.abs(q[:, 1:] - q[:, :-1])
    dv[1:, :] = 1.0 + scale * np.abs(q[1:, :] - q[:-1, :])
    return dh, dv


def _nc_walks(d: np.ndarray, r: float):
    """Outward walks along the rows of d: for k = 1, 2, ... yields (k, sign, dist, live),
    dist the sum of the increments between j and j + sign k (inf past the border) and live
    whether every distance up to that step is within r."""
    Hn, Wn = d.shape
    R = int(math.floor(r)) + 1          # increments are >= 1: no window reaches past R
    for sgn in (1, -1):
        dist = np.zeros((Hn, Wn))
        live = np.ones((Hn, Wn), dtype=bool)
        for k in range(1, min(R, Wn - 1) + 1):
            inc = np.full((Hn, Wn), np.inf)
            if sgn > 0:
                inc[:, :Wn - k] = d[:, k:]            # to the right: d[j+1], ..., d[j+k]
            else:
                inc[:, k:] = d[:, 1:Wn - k + 1]       # to the left: d[j], ..., d[j-k+1]
            dist = dist + inc
            live &= dist <= r
            yield k, sgn, dist, live


def nc_box_pass(F: np.ndarray, d: np.ndarray, r: float, axis: int) -> np.ndarray:
    """One transformed-domain box pass along `axis` (1: rows, 0: columns).  The output at j
    is the mean of F over the m on the same line with transformed distance
    dist(j, m) <= r, dist being the sum of the increments d between j and m; no wrap at
    the borders."""
    F = np.asarray(F, dtype=np.float64)
    if axis == 0:
        return nc_box_pass(F.T, d.T, r, 1).T
    Wn = F.shape[1]
    num = F.copy()
    cnt = np.ones_like(F)
    for k, sgn, _dist, live in _nc_walks(d, float(r)):
        vals = np.zeros_like(F)
        if sgn > 0:
            vals[:, :Wn - k] = F[:, k:]
        else:
            vals[:, k:] = F[:, :Wn - k]
        num += np.where(live, vals, 0.0)
        cnt += live
    return num / cnt


def _nc_params(sigma_s, sigma_r):
    # the sigmas arrive as the library's FP32 parameters; a and the radii follow in FP64
    s = float(np.float32(sigma_s))
    a = 0.0 if math.isinf(sigma_r) else s / float(np.float32(sigma_r))
    return s, a


def nc_filter(p: np.ndarray, q, sigma_s: float, sigma_r: float, n_iter: int = 3, inv_span=None) -> np.ndarray:
    """NC filter of field p guided by q (None: p itself): n_iter rounds of a horizontal then a
    vertical box pass with radii nc_schedule(sigma_s, n_iter); the increments come from the
    guide once (the domain transform is not recomputed between passes).  sigma_r = inf
    switches the range term off (increments 1: plain iterated box filters)."""
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    s, a = _nc_params(sigma_s, sigma_r)
    dh, dv = nc_increments(qq, a, inv_span)
    F = p
    for r in nc_schedule(s, n_iter):
        F = nc_box_pass(F, dh, r, 1)
        F = nc_box_pass(F, dv, r, 0)
    return F


def nc_decision_margin(q, sigma_s: float, sigma_r: float, n_iter: int = 3, inv_span=None) -> float:
    """Smallest |dist - r_k| over the window-membership decisions nc_filter takes for the
    guide field q (every step of every walk up to and including its first step past r_k,
    both axes, every pass): how far the closest decision lies from its threshold."""
    qq = np.asarray(q, dtype=np.float64)
    s, a = _nc_params(sigma_s, sigma_r)
    dh, dv = nc_increments(qq, a, inv_span)
    best = math.inf
    for r in nc_schedule(s, n_iter):
        for d in (dh, dv.T):
            alive = np.ones(d.shape, dtype=bool)
            prev_sgn = None
            for _k, sgn, dist, live in _nc_walks(d, float(r)):
                if sgn != prev_sgn:
                    alive = np.ones(d.shape, dtype=bool)
                    prev_sgn = sgn
                decided = alive & np.isfinite(dist)     # steps still walked (inside the image)
                if decided.any():
                    best = min(best, float(np.min(np.abs(dist[decided] - r))))
                alive = live.copy()
    return best


def nc_filter_bruteforce(p, q, sigma_s, sigma_r, n_iter=3):
    """Pixel-by-pixel loops over the same definition (tiny inputs only): for each pixel walk
    outward along the line, adding the increments, and average the values reached within r."""
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    Hn, Wn = p.shape
    s, a = _nc_params(sigma_s, sigma_r)

    def incr(x1, x0):
        return 1.0 + a * abs(x1 - x0)

    def line_pass(vals, guide, r):
        n = len(vals)
        out = [0.0] * n
        for j in range(n):
            tot, cnt = vals[j], 1
            dist = 0.0
            for m in range(j + 1, n):
                dist += incr(guide[m], guide[m - 1])
                if not dist <= r:
                    break
                tot += vals[m]
                cnt += 1
            dist = 0.0
            for m in range(j - 1, -1, -1):
                dist += incr(guide[m + 1], guide[m])
                if not dist <= r:
                    break
                tot += vals[m]
                cnt += 1
            out[j] = tot / cnt
        return out

    F = [list(row) for row in p]
    for r in nc_schedule(s, n_iter):
        F = [line_pass(F[i], list(qq[i]), r) for i in range(Hn)]
        cols = [line_pass([F[i][j] for i in range(Hn)], [qq[i][j] for i in range(Hn)], r) for j in range(Wn)]
        F = [[cols[j][i] for j in range(Wn)] for i in range(Hn)]
    return np.array(F, dtype=np.float64)


# ---------------------------------------------------------------------------
# Bilateral-grid approximation of Eq. (1) (Paris and Durand, "A Fast
# Approximation of the Bilateral Filter using a Signal Processing Approach",
# 2006: the fast BLF the paper's experiments use, Section III-B)
# ---------------------------------------------------------------------------
#
# The filter is a 3-D linear convolution in (x, y, range) followed by a
# division: values p and ones are splatted into a grid of cells s pixels wide
# and one range cell deep, both grids are blurred with a Gaussian, and each
# pixel reads num / den back by trilinear interpolation at its own
# (x, y, q).  Readings (listed in the design notes):
#   * spatial cell s = max(1, floor(sigma_s + 1/2)) pixels: pixel x lies in cell
#     floor((x + floor(s/2)) / s) and is read back at x / s;
#   * range cell 1 / inv from min(q): inv = 1 / sigma_r, lowered if needed so
#     that at most GRID_ZMAX bins span [min q, max q]; a pixel's bin is
#     floor((q - min q) inv + 1/2), in FP64 like everything here (the bin is a
#     discontinuous function of q: ``grid_bin_margin`` reports how close the
#     closest pixel lies to a bin boundary); with the normalise flag inv is
#     divided by the field's span first;
#   * blur: Gaussian taps exp(-k^2 / (2 sigma^2)) for k in [-2, 2], sigma =
#     sigma_s / s cells along x and y and sigma_r inv cells along the range;
#     the range axis has two empty bins of padding at each end;
#   * the image is periodic (as in the exact filter): the grid is built over
#     the periodic extension, so every output sees the same neighbourhood of
#     cells whatever its position.

GRID_PAD = 2
GRID_ZMAX = 32


def grid_cell(sigma_s: float) -> int:
    """Spatial cell size: sigma_s (the sampling rate of the Paris-Durand grid) rounded to a
    whole number of pixels, halves up, at least 1: max(1, floor(sigma_s + 1/2)), from the
    library's FP32 sigma_s."""
    return max(1, int(math.floor(float(np.float32(sigma_s)) + 0.5)))


def _grid_scale(q: np.ndarray, sigma_r: float, inv_span=None):
    """Range origin, span and bins per unit of the guide field q (FP64): inv = 1 / sigma_r
    (times inv_span when normalised), lowered to (GRID_ZMAX - 1) / span when more bins than
    GRID_ZMAX would be needed."""
    q = np.asarray(q, dtype=np.float64)
    qmin = float(q.min())
    span = float(q.max()) - qmin
    inv = 0.0 if math.isinf(sigma_r) else 1.0 / float(np.float32(sigma_r))
    if inv_span is not None:
        inv *= float(inv_span)
    capped = span * inv > GRID_ZMAX - 1
    if capped:
        inv = (GRID_ZMAX - 1) / span
    return qmin, span, inv, capped


def grid_range(q: np.ndarray, sigma_r: float, inv_span=None):
    """Range origin and scale of the guide field q: (qmin, inv, bin of every pixel, bins in
    use); the bin is floor((q - qmin) inv + 1/2)."""
    q = np.asarray(q, dtype=np.float64)
    qmin, _span, inv, _capped = _grid_scale(q, sigma_r, inv_span)
    z = np.floor((q - qmin) * inv + 0.5).astype(np.int64)
    return qmin, inv, z, int(z.max()) + 1


def grid_bin_margin(q: np.ndarray, sigma_r: float, inv_span=None) -> float:
    """How close the grid's integer decisions come to their thresholds for the guide field
    q: the smallest distance of (q - qmin) inv + 1/2 from an integer over the pixels, and of
    span inv from GRID_ZMAX - 1 (the cap decision), in bins."""
    q = np.asarray(q, dtype=np.float64)
    qmin, span, inv, _capped = _grid_scale(q, sigma_r, inv_span)
    raw = 0.0 if math.isinf(sigma_r) else 1.0 / float(np.float32(sigma_r))
    if inv_span is not None:
        raw *= float(inv_span)
    t = (q - qmin) * inv + 0.5
    return min(float(np.min(np.abs(t - np.round(t)))), abs(span * raw - (GRID_ZMAX - 1)))


def _grid_taps(sigma_cells: float):
    k = np.arange(-GRID_PAD, GRID_PAD + 1, dtype=np.float64)
    if sigma_cells <= 0.0:
        return (k == 0).astype(np.float64)
    return np.exp(-(k * k) / (2.0 * sigma_cells * sigma_cells))


def grid_filter(p: np.ndarray, q, sigma_s: float, sigma_r: float, inv_span=None) -> np.ndarray:
    """Bilateral-grid approximation of Eq. (1) on field p with range values q (None: p)."""
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    H, W = p.shape
    s = grid_cell(sigma_s)
    qmin, inv, zb, nz = grid_range(qq, sigma_r, inv_span)
    sig_xy = float(np.float32(sigma_s)) / s
    # the range Gaussian, sigma_r in the (normalised) guide's units, measured in cells
    sig_z = 0.0 if math.isinf(sigma_r) else float(np.float32(sigma_r)) * float(inv)
    if inv_span is not None and sig_z > 0.0:
        sig_z /= float(inv_span)
    # periodic extension by m pixels: enough for every cell within 3 of an output's cell
    m = 4 * s + s // 2 + 1
    ys = np.arange(-m, H + m)
    xs = np.arange(-m, W + m)
    cy = (ys + s // 2) // s
    cx = (xs + s // 2) // s
    oy, ox = cy.min(), cx.min()
    gy, gx, gz = cy.max() - oy + 1, cx.max() - ox + 1, nz + 2 * GRID_PAD
    num = np.zeros((gz, gy, gx))
    den = np.zeros((gz, gy, gx))
    Y, X = np.meshgrid(ys % H, xs % W, indexing="ij")
    CY, CX = np.meshgrid(cy - oy, cx - ox, indexing="ij")
    np.add.at(num, (zb[Y, X] + GRID_PAD, CY, CX), p[Y, X])
    np.add.at(den, (zb[Y, X] + GRID_PAD, CY, CX), 1.0)
    for axis, taps in ((2, _grid_taps(sig_xy)), (1, _grid_taps(sig_xy)), (0, _grid_taps(sig_z))):
        for arr in (num, den):
            out = np.zeros_like(arr)
            n = arr.shape[axis]
            for k, w in zip(range(-GRID_PAD, GRID_PAD + 1), taps):
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                src[axis] = slice(max(0, k), n + min(0, k))
                dst[axis] = slice(max(0, -k), n - max(0, k))
                out[tuple(dst)] += w * arr[tuple(src)]
            arr[...] = out
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    fz = (qq - qmin) * float(inv) + GRID_PAD
    fy = yy / s - oy
    fx = xx / s - ox
    z0, y0, x0 = np.floor(fz).astype(np.int64), np.floor(fy).astype(np.int64), np.floor(fx).astype(np.int64)
    az, ay, ax = fz - z0, fy - y0, fx - x0
    vn = np.zeros_like(p)
    vd = np.zeros_like(p)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (az if dz else 1 - az) * (ay if dy else 1 - ay) * (ax if dx else 1 - ax)
                vn += w * num[z0 + dz, y0 + dy, x0 + dx]
                vd += w * den[z0 + dz, y0 + dy, x0 + dx]
    return vn / vd


def grid_filter_bruteforce(p, q, sigma_s, sigma_r):
    """The same approximation as one sum per output over the pixels of the periodic
    extension (tiny inputs): the output is sum_j T(i, j) p_j / sum_j T(i, j), T(i, j) the
    trilinear read at pixel i's grid position of the blurred unit splat of pixel j."""
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    H, W = p.shape
    s = grid_cell(sigma_s)
    qmin, inv, zb, nz = grid_range(qq, sigma_r)
    ts = _grid_taps(float(np.float32(sigma_s)) / s)
    tz = _grid_taps(0.0 if math.isinf(sigma_r) else float(np.float32(sigma_r)) * float(inv))
    m = 4 * s + s // 2 + 1

    def tap(taps, d):
        return taps[d + GRID_PAD] if abs(d) <= GRID_PAD else 0.0

    out = np.zeros_like(p)
    for i in range(H):
        for j in range(W):
            fz, fy, fx = (qq[i, j] - qmin) * float(inv), i / s, j / s
            z0, y0, x0 = math.floor(fz), math.floor(fy), math.floor(fx)
            num = den = 0.0
            for a in range(-m, H + m):
                for b in range(-m, W + m):
                    cz, cy, cx = int(zb[a % H, b % W]), (a + s // 2) // s, (b + s // 2) // s
                    t = 0.0
                    for dz in (0, 1):
                        for dy in (0, 1):
                            for dx in (0, 1):
                                w = ((fz - z0) if dz else 1 - (fz - z0)) * ((fy - y0) if dy else 1 - (fy - y0)) * \
                                    ((fx - x0) if dx else 1 - (fx - x0))
                                if w != 0.0:
                                    t += w * tap(tz, z0 + dz - cz) * tap(ts, y0 + dy - cy) * tap(ts, x0 + dx - cx)
                    num += t * p[a % H, b % W]
                    den += t
            out[i, j] = num / den
    return out


# ---------------------------------------------------------------------------
# Adaptive-manifold filter (Section III-D: AMF-LS embeds it in place of the
# BLF; its definition is Gastal and Oliveira, "Adaptive Manifolds for
# Real-Time High-Dimensional Filtering", 2012)
# ---------------------------------------------------------------------------
#
# The AMF approximates a Gaussian bilateral filter of p with range source q by
# filtering on a few smooth images eta_k ("manifolds") that sample the range:
# every pixel is splatted onto each manifold with the Gaussian weight
# psi_k = exp(-(eta_k - q)^2 / (2 sigma_r'^2)), the splatted values (psi p and
# psi) are blurred along the manifold by a recursive filter whose steps lengthen
# with the manifold's own range differences, and each pixel reads the blurred
# values back with the same weight: g = sum_k psi_k B_k(psi_k p) / sum_k psi_k
# B_k(psi_k).  The manifolds form a binary tree: the root is a spatial low-pass
# of q; the two children of a manifold are low-passes of q over the pixels
# below and above it, each pixel weighted by 1 - psi (how poorly the parent
# represents it).  Readings (listed in the design notes):
#   * the range is a scalar, so the split of a cluster is the sign of q - eta;
#   * sigma_r' = sigma_r / sqrt(2) in the splat, the slice and the blur's range
#     term (the splat and slice weights multiply to the sigma_r Gaussian);
#   * the blur is the domain transform's first-order recursive filter:
#     y_j = (1 - a^{d_j}) x_j + a^{d_j} y_{j-1}, a = exp(-sqrt(2) / sigma_s), then
#     the same from the right (step j -> j-1 uses d_j), along rows and then
#     along columns, once; d_j = 1 + (sigma_s / sigma_r') |eta_j - eta_{j-1}| on a
#     manifold and d_j = 1 for the low-passes; lines start at the image borders
#     (no wrap), y_0 = x_0;
#   * everything at full resolution (no downsampled manifolds);
#   * tree height max(2, ceil(H_s L)), H_s = floor(log2 sigma_s) - 1,
#     L = 1 - sigma_r, each clamped at 0, at most AMF_MAX_HEIGHT; 2^height - 1
#     manifolds;
#   * a child manifold is absent at pixels where its low-passed weight is below
#     AMF_TAU (no cluster pixel within reach): there it takes no splat and no
#     children, and the blur steps across it with d = 1;
#   * pixels far from every manifold keep their value: g = p + alpha (num / den
#     - p) with alpha = max_k psi_k, and g = p where den = 0;
#   * with the normalisation flag the range differences (eta - q and the
#     manifold steps) are scaled by 1/span(q), the guide field mapped to [0, 1];
#   * sigma_r = inf: psi = 1, no children, d = 1: the normalised recursive
#     filter of p.

AMF_MAX_HEIGHT = 6
AMF_TAU = 1e-20


def amf_tree_height(sigma_s: float, sigma_r: float) -> int:
    """max(2, ceil(H_s L)), H_s = floor(log2 sigma_s) - 1 and L = 1 - sigma_r clamped at 0,
    capped at AMF_MAX_HEIGHT; the sigmas are the FP32 parameters, the arithmetic FP64."""
    s = float(np.float32(sigma_s))
    r = float(np.float32(sigma_r))
    hs = max(0.0, math.floor(math.log2(s)) - 1.0)
    lr = 0.0 if math.isinf(r) else max(0.0, 1.0 - r)
    return int(min(AMF_MAX_HEIGHT, max(2, math.ceil(hs * lr))))


def amf_rf_line_rows(X, alpha):
    """Recursive filter along each row of every array in X: alpha[i, j] is the step
    coefficient between columns j-1 and j (alpha[:, 0] unused); left to right, then right to
    left."""
    out = []
    W = alpha.shape[1]
    for x in X:
        y = np.array(x, dtype=np.float64, copy=True)
        for j in range(1, W):
            y[:, j] = (1.0 - alpha[:, j]) * y[:, j] + alpha[:, j] * y[:, j - 1]
        for j in range(W - 2, -1, -1):
            y[:, j] = (1.0 - alpha[:, j + 1]) * y[:, j] + alpha[:, j + 1] * y[:, j + 1]
        out.append(y)
    return out


def _amf_alpha(eta, sigma_s, sigma_r, axis, inv_span):
    """Step coefficients a^d along `axis` (1: rows, 0: columns) over manifold eta; sigma_r = inf
    gives the plain low-pass (d = 1).  Absent samples (NaN) step as if flat."""
    a_log = -math.sqrt(2.0) / sigma_s
    shape = eta.shape
    if math.isinf(sigma_r):
        return np.full(shape, math.exp(a_log))
    diff = np.zeros(shape)
    if axis == 1:
        diff[:, 1:] = eta[:, 1:] - eta[:, :-1]
    else:
        diff[1:, :] = eta[1:, :] - eta[:-1, :]
    diff = np.where(np.isnan(diff), 0.0, np.abs(diff)) * (1.0 if inv_span is None else float(inv_span))
    sr1 = sigma_r / math.sqrt(2.0)
    return np.exp(a_log * (1.0 + (sigma_s / sr1) * diff))


def amf_blur(X, eta, sigma_s, sigma_r, inv_span=None):
    """Rows then columns recursive filtering of the arrays in X over manifold eta (None: the
    plain low-pass)."""
    shape = X[0].shape
    ref = np.zeros(shape) if eta is None else eta
    ah = _amf_alpha(ref, sigma_s, math.inf if eta is None else sigma_r, 1, inv_span)
    av = _amf_alpha(ref, sigma_s, math.inf if eta is None else sigma_r, 0, inv_span)
    Y = amf_rf_line_rows(X, ah)
    return [z.T for z in amf_rf_line_rows([y.T for y in Y], av.T)]


def amf_filter(p: np.ndarray, q, sigma_s: float, sigma_r: float, height: int = 0,
               inv_span=None, return_manifolds=False):
    """Adaptive-manifold filter of field p with range source q (None: p itself).  height 0
    takes amf_tree_height(sigma_s, sigma_r).  The sigmas are taken as FP32 values."""
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    s = float(np.float32(sigma_s))
    r = float(np.float32(sigma_r))
    ht = amf_tree_height(s, r) if not height else int(height)
    scale = 1.0 if inv_span is None else float(inv_span)
    inf = math.isinf(r)
    k = 0.0 if inf else 1.0 / (r * r)          # psi = exp(-(eta - q)^2 / (2 (r / sqrt 2)^2))
    num = np.zeros_like(p)
    den = np.zeros_like(p)
    amax = np.zeros_like(p)
    manifolds = []
    stack = [(amf_blur([qq], None, s, r)[0], 1)]
    while stack:
        eta, level = stack.pop()
        manifolds.append(eta)
        present = ~np.isnan(eta)
        dq = np.where(present, (eta - qq) * scale, 0.0)
        psi = np.where(present, np.exp(-k * dq * dq), 0.0)
        bn, bd = amf_blur([psi * p, psi], eta, s, r, inv_span)
        num += psi * bn
        den += psi * bd
        amax = np.maximum(amax, psi)
        if level < ht:
            for below in (True, False):
                side = (qq < eta) if below else (qq >= eta)
                w = np.where(present & side, 1.0 - psi, 0.0)
                hq, hw = amf_blur([w * qq, w], None, s, r)
                child = np.full_like(p, np.nan)
                ok = hw >= AMF_TAU
                child[ok] = hq[ok] / hw[ok]
                stack.append((child, level + 1))
    safe = np.where(den > 0.0, den, 1.0)
    g = np.where(den > 0.0, p + amax * (num / safe - p), p)
    return (g, manifolds) if return_manifolds else g


def amf_filter_dense(p, q, sigma_s, sigma_r, height=0, inv_span=None):
    """The same filter through explicit linear operators (tiny inputs only): each recursive
    pass is the dense matrix of its closed form, y = B F x with
    F[i, k] = (1 - c_k) prod_{m=k+1..i} c_m (F[i, 0] = prod_{m=1..i} c_m) and
    B[i, k] = (1 - c_{k+1}) prod_{m=i+1..k} c_m (B[i, n-1] = prod_{m=i+1..n-1} c_m); the
    tree is walked breadth first with per-pixel loops."""
    p = np.asarray(p, dtype=np.float64)
    qq = p if q is None else np.asarray(q, dtype=np.float64)
    Hn, Wn = p.shape
    s = float(np.float32(sigma_s))
    r = float(np.float32(sigma_r))
    ht = amf_tree_height(s, r) if not height else int(height)
    scale = 1.0 if inv_span is None else float(inv_span)
    a = math.exp(-math.sqrt(2.0) / s)

    def line_op(c):
        n = len(c)
        F = np.zeros((n, n))
        B = np.zeros((n, n))
        for i in range(n):
            for kk in range(i + 1):
                w = 1.0 if kk == 0 else 1.0 - c[kk]
                for m in range(kk + 1, i + 1):
                    w *= c[m]
                F[i, kk] = w
            for kk in range(i, n):
                w = 1.0 if kk == n - 1 else 1.0 - c[kk + 1]
                for m in range(i + 1, kk + 1):
                    w *= c[m]
                B[i, kk] = w
        return B @ F

    def coef(e0, e1):
        if e0 is None or math.isinf(r) or math.isnan(e0) or math.isnan(e1):
            return a
        return a ** (1.0 + (s / (r / math.sqrt(2.0))) * abs(e1 - e0) * scale)

    def blur2d(x, eta):
        y = np.zeros((Hn, Wn))
        for i in range(Hn):
            c = [0.0] + [coef(None if eta is None else eta[i, j - 1], None if eta is None else eta[i, j])
                         for j in range(1, Wn)]
            y[i, :] = line_op(c) @ x[i, :]
        z = np.zeros((Hn, Wn))
        for j in range(Wn):
            c = [0.0] + [coef(None if eta is None else eta[i - 1, j], None if eta is None else eta[i, j])
                         for i in range(1, Hn)]
            z[:, j] = line_op(c) @ y[:, j]
        return z

    num = np.zeros((Hn, Wn))
    den = np.zeros((Hn, Wn))
    amax = np.zeros((Hn, Wn))
    level = [blur2d(qq, None)]
    for depth in range(1, ht + 1):
        nxt = []
        for eta in level:
            psi = np.zeros((Hn, Wn))
            for i in range(Hn):
                for j in range(Wn):
                    if math.isnan(eta[i, j]):
                        continue
                    d = (eta[i, j] - qq[i, j]) * scale
                    psi[i, j] = 1.0 if math.isinf(r) else math.exp(-d * d / (r * r))
            bn = blur2d(psi * p, eta)
            bd = blur2d(psi, eta)
            num += psi * bn
            den += psi * bd
            amax = np.maximum(amax, psi)
            if depth < ht:
                for below in (True, False):
                    w = np.zeros((Hn, Wn))
                    for i in range(Hn):
                        for j in range(Wn):
                            e = eta[i, j]
                            if not math.isnan(e) and ((qq[i, j] < e) if below else (qq[i, j] >= e)):
                                w[i, j] = 1.0 - psi[i, j]
                    hq = blur2d(w * qq, None)
                    hw = blur2d(w, None)
                    child = np.full((Hn, Wn), np.nan)
                    for i in range(Hn):
                        for j in range(Wn):
                            if hw[i, j] >= AMF_TAU:
                                child[i, j] = hq[i, j] / hw[i, j]
                    nxt.append(child)
        level = nxt
    g = p.copy()
    for i in range(Hn):
        for j in range(Wn):
            if den[i, j] > 0.0:
                g[i, j] = p[i, j] + amax[i, j] * (num[i, j] / den[i, j] - p[i, j])
    return g


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


def _field_inv_span(p, q, sigma_r, normalize):
    """The normalisation of the experiments section maps the guide field to [0, 1], which
    scales its differences by 1 / span (None: no normalisation, range kernel off, or a
    constant field, which keeps sigma_r)."""
    if not (normalize and math.isfinite(sigma_r)):
        return None
    g = np.asarray(p if q is None else q, dtype=np.float64)
    span = float(g.max()) - float(g.min())
    return 1.0 / span if span > 0 else None


def _filter_field(p, q, sigma_s, sigma_r, radius, normalize, filt="blf", nc_iterations=3, amf_height=0,
                  engine="numpy"):
    if filt == "grid":
        # the bilateral-grid approximation in place of the exact filter
        return grid_filter(p, q, sigma_s, sigma_r, _field_inv_span(p, q, sigma_r, normalize))
    if filt == "amf":
        # AMF-LS (Section III-D): the adaptive-manifold filter in place of the BLF
        # (amf_height 0: the default tree-height rule)
        return amf_filter(p, q, sigma_s, sigma_r, amf_height, _field_inv_span(p, q, sigma_r, normalize))
    if filt == "nc":
        # NC-LS (Section III-D): the NC filter in place of the BLF.  With the
        # normalisation of the experiments section the guide field is mapped to
        # [0, 1], which scales its differences (and so the increments' range
        # term) by 1/span; the filtered field's own affine map commutes with
        # the averaging.
        inv = _field_inv_span(p, q, sigma_r, normalize)
        return nc_filter(p, q, sigma_s, sigma_r, nc_iterations, inv)
    blf = bilateral_filter
    if engine == "c":
        # the same definition as plain C loops (oracle/blf_oracle.c), for large images
        from .c_blf import bilateral_filter_c as blf
    if not normalize:
        return blf(p, q, sigma_s, sigma_r, radius)
    # experiments section: fields taken to [0, 1], filtered, then mapped back
    pn, plo, pspan = _normalise_unit(p)
    qn = pn if q is None else _normalise_unit(q)[0]
    return blf(pn, qn, sigma_s, sigma_r, radius) * pspan + plo


def smooth_channel(f, lam, sigma_s, sigma_r, radius=-1, iterations=1, guide=None,
                   normalize=False, sigma_guide=0.0, return_fields=False, filter="blf", nc_iterations=3,
                   amf_height=0, detail_gain=0.0, engine="numpy"):
    """BLF-LS on one channel (Section III-A two-step procedure, Section III-D extensions).

    Step 1 filters p_x, p_y with Eq. (1) (``filter="nc"``: the NC filter of the domain
    transform, NC-LS; ``filter="grid"``: the bilateral-grid approximation of Eq. (1);
    ``filter="amf"``: the adaptive-manifold filter, AMF-LS); step 2 solves Eq. (8).  ``guide`` switches to joint filtering;
    ``iterations`` > 1 is rolling guidance.  ``detail_gain`` m != 0 returns the detail-enhanced
    u + m (f - u) of the experiments section (the detail layer f - u boosted m times).
    ``engine="c"`` evaluates Eq. (1) with the C loops of ``blf_oracle.c`` (same definition,
    for images where the NumPy loops take minutes).
    """
    f = np.asarray(f, dtype=np.float64)
    f_in = f
    r = default_radius(sigma_s) if radius is None or radius < 0 else int(radius)
    nc = filter in ("nc", "grid", "amf")   # these normalise through the guide field's span
    lo, span = 0.0, 1.0
    if normalize and not nc:
        f, lo, span = _normalise_unit(f)
    px, py = grad_x(f), grad_y(f)
    if guide is not None:
        h = np.asarray(guide, dtype=np.float64)
        if normalize and not nc:
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
        gx = _filter_field(px, qx, sigma_s, sigma_r, r, normalize, filter, nc_iterations, amf_height, engine)
        gy = _filter_field(py, qy, sigma_s, sigma_r, r, normalize, filter, nc_iterations, amf_height, engine)
        u = blfls_solve(f, gx, gy, lam)
        prev = u
    out = u * span + lo
    if detail_gain:
        out = out + detail_gain * (f_in - out)
    if return_fields:
        return out, gx * span, gy * span
    return out


def smooth(f, lam, sigma_s, sigma_r, radius=-1, iterations=1, guide=None, normalize=False,
           sigma_guide=0.0, filter="blf", nc_iterations=3, amf_height=0, detail_gain=0.0, engine="numpy"):
    """BLF-LS (or NC-LS, grid BLF-LS, AMF-LS with ``filter="nc"``, ``"grid"``, ``"amf"``) on a
    (H, W) or (C, H, W) image; channels are independent."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 2:
        return smooth_channel(f, lam, sigma_s, sigma_r, radius, iterations, guide, normalize,
                              sigma_guide, filter=filter, nc_iterations=nc_iterations,
                              amf_height=amf_height, detail_gain=detail_gain, engine=engine)
    g = None if guide is None else np.asarray(guide, dtype=np.float64)
    outs = []
    for c in range(f.shape[0]):
        gc = None if g is None else (g[c] if g.ndim == 3 else g)
        outs.append(smooth_channel(f[c], lam, sigma_s, sigma_r, radius, iterations, gc,
                                   normalize, sigma_guide, filter=filter, nc_iterations=nc_iterations,
                                   amf_height=amf_height, detail_gain=detail_gain, engine=engine))
    return np.stack(outs)


# ---------------------------------------------------------------------------
# HDR tone mapping in the log domain (experiments section: the framework of
# Durand and Dorsey 2002, with BLF-LS as the base/detail decomposition)
# ---------------------------------------------------------------------------
#
# Readings (listed in the design notes): the intensity is the weighted sum
# (20 R + 40 G + B) / 61, floored at TM_FLOOR; its base layer is the BLF-LS
# output of log10(intensity) and the detail layer the difference; the base is
# compressed linearly so that its range spans log10(contrast) with its maximum
# at 0 (a constant base is only shifted); the output intensity is
# 10^(compressed base + detail) and each channel keeps its ratio to the input
# intensity.  Linear output, no display gamma.

TM_FLOOR = 1e-6


def tonemap(rgb: np.ndarray, lam, sigma_s, sigma_r, contrast=5.0, **smooth_kw) -> np.ndarray:
    """Tone-map a (3, H, W) linear HDR image; smooth_kw go to smooth() (normalize, filter, ...)."""
    rgb = np.asarray(rgb, dtype=np.float64)
    inten = np.maximum((20.0 * rgb[0] + 40.0 * rgb[1] + rgb[2]) / 61.0, TM_FLOOR)
    L = np.log10(inten)
    base = smooth(L, lam, sigma_s, sigma_r, **smooth_kw)
    detail = L - base
    lo, hi = float(base.min()), float(base.max())
    cf = math.log10(contrast) / (hi - lo) if hi > lo else 1.0
    out_log = (base - hi) * cf + detail
    return rgb / inten * 10.0 ** out_log
