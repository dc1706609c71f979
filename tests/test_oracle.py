"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with an
independent route to the same number (an explicit dense solve, brute-force
loops, a hand derivation, a closed form, an invariant the method must keep).
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image

RNG = np.random.default_rng(12345)


def _rand(H, W, rng=RNG):
    return rng.uniform(0.0, 1.0, size=(H, W))


# -- independent operators written for the tests (explicit loops, no np.roll) --

def _dx_loop(f):
    H, W = f.shape
    out = np.empty_like(f)
    for i in range(H):
        for j in range(W):
            out[i, j] = f[i, (j + 1) % W] - f[i, j]
    return out


def _dy_loop(f):
    H, W = f.shape
    out = np.empty_like(f)
    for i in range(H):
        for j in range(W):
            out[i, j] = f[(i + 1) % H, j] - f[i, j]
    return out


# ---------------------------------------------------------------------------
# Difference operators (Section II-B: forward differences and their adjoints)
# ---------------------------------------------------------------------------

def test_gradients_match_loops():
    f = _rand(5, 7)
    assert np.array_equal(oracle.grad_x(f), _dx_loop(f))
    assert np.array_equal(oracle.grad_y(f), _dy_loop(f))


def test_adjoints_are_transposes():
    # <D v, w> == <v, D^T w> for random v, w pins the adjoint's sign and direction
    v, w = _rand(6, 9), _rand(6, 9)
    assert np.isclose(np.sum(oracle.grad_x(v) * w), np.sum(v * oracle.grad_x_adjoint(w)), atol=1e-13)
    assert np.isclose(np.sum(oracle.grad_y(v) * w), np.sum(v * oracle.grad_y_adjoint(w)), atol=1e-13)


def test_difference_otf_closed_form():
    # F(1) is the DFT of the delta: all ones (Section II-C).  The DFT of the
    # forward-difference kernel is exp(2 pi i k / N) - 1, |.|^2 = 4 sin^2(pi k / N).
    H, W = 6, 10
    F1, Fx, Fy = oracle.difference_otf(H, W)
    assert np.allclose(F1, 1.0, atol=1e-14)
    kx = np.arange(W)[None, :]
    ky = np.arange(H)[:, None]
    assert np.allclose(Fx, np.exp(2j * np.pi * kx / W) - 1.0 + 0 * ky, atol=1e-13)
    assert np.allclose(Fy, np.exp(2j * np.pi * ky / H) - 1.0 + 0 * kx, atol=1e-13)
    assert np.allclose(np.abs(Fx) ** 2, 4 * np.sin(np.pi * kx / W) ** 2 + 0 * ky, atol=1e-13)


# ---------------------------------------------------------------------------
# P1: Eq. (8) Fourier solve == dense direct solve of the normal equations
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", [(1, 1), (1, 5), (2, 2), (3, 4), (5, 7), (7, 5), (11, 3), (12, 12), (4, 9)])
@pytest.mark.parametrize("lam", [0.0, 0.3, 20.0, 1024.0])
def test_P1_fft_solve_equals_dense(H, W, lam):
    rng = np.random.default_rng(H * 100 + W)
    f, gx, gy = _rand(H, W, rng), rng.normal(size=(H, W)), rng.normal(size=(H, W))
    u_fft = oracle.blfls_solve(f, gx, gy, lam)
    u_dense = oracle.dense_blfls_solve(f, gx, gy, lam)
    assert np.max(np.abs(u_fft - u_dense)) < 1e-10 * (1 + lam)


def test_dense_matrices_match_loop_operators():
    H, W = 4, 6
    Mx, My = oracle.dense_difference_matrices(H, W)
    f = _rand(H, W)
    assert np.allclose((Mx @ f.ravel()).reshape(H, W), _dx_loop(f), atol=1e-15)
    assert np.allclose((My @ f.ravel()).reshape(H, W), _dy_loop(f), atol=1e-15)


# ---------------------------------------------------------------------------
# P2: normal-equation stencil residual at a larger size (operators applied, not inverted)
# ---------------------------------------------------------------------------

def test_P2_stencil_residual():
    H, W, lam = 96, 130, 50.0
    rng = np.random.default_rng(7)
    f = voronoi_image(H, W, 7)
    gx, gy = rng.normal(0, 0.1, (H, W)), rng.normal(0, 0.1, (H, W))
    u = oracle.blfls_solve(f, gx, gy, lam)

    def dxT(v):
        out = np.empty_like(v)
        out[:, 1:] = v[:, :-1] - v[:, 1:]
        out[:, 0] = v[:, -1] - v[:, 0]
        return out

    def dyT(v):
        out = np.empty_like(v)
        out[1:, :] = v[:-1, :] - v[1:, :]
        out[0, :] = v[-1, :] - v[0, :]
        return out

    def dx(v):
        out = np.empty_like(v)
        out[:, :-1] = v[:, 1:] - v[:, :-1]
        out[:, -1] = v[:, 0] - v[:, -1]
        return out

    def dy(v):
        out = np.empty_like(v)
        out[:-1, :] = v[1:, :] - v[:-1, :]
        out[-1, :] = v[0, :] - v[-1, :]
        return out

    res = (u - f) + lam * (dxT(dx(u) - gx) + dyT(dy(u) - gy))
    assert np.max(np.abs(res)) < 1e-10


# ---------------------------------------------------------------------------
# P3: vectorised Eq. (1) == brute-force loops, including windows wider than the image
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("H,W,r,ss,sr", [
    (6, 7, 2, 1.0, 0.3), (5, 5, 1, 0.7, 0.05), (3, 5, 4, 1.5, 0.2),  # window > image
    (1, 6, 2, 1.0, 0.5), (4, 4, 0, 1.0, 0.1), (5, 3, 3, 2.0, math.inf)])
@pytest.mark.parametrize("joint", [False, True])
def test_P3_blf_bruteforce(H, W, r, ss, sr, joint):
    rng = np.random.default_rng(H * 31 + W * 7 + r)
    p = rng.normal(0, 0.3, (H, W))
    q = rng.normal(0, 0.3, (H, W)) if joint else None
    a = oracle.bilateral_filter(p, q, ss, sr, r)
    b = oracle.bilateral_filter_bruteforce(p, q, ss, sr, r)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("joint,sr,r", [(False, 0.2, 3), (True, 0.1, 5), (False, math.inf, 2), (False, 0.3, 9)])
def test_P3_blf_at_pixels_matches_full(joint, sr, r):
    rng = np.random.default_rng(99)
    p = rng.normal(0, 0.3, (13, 17))
    q = rng.normal(0, 0.3, (13, 17)) if joint else None
    full = oracle.bilateral_filter(p, q, 1.5, sr, r)
    rows = rng.integers(0, 13, 40)
    cols = rng.integers(0, 17, 40)
    at = oracle.bilateral_filter_at(p, q, 1.5, sr, r, rows, cols)
    assert np.max(np.abs(at - full[rows, cols])) < 1e-13


# ---------------------------------------------------------------------------
# Hand-derived example: a 1x4 step image, r=1, sigma_s=1
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.0, 1.0, 20.0, 1024.0])
def test_hand_derived_1x4(lam):
    # f = [0,0,1,1] -> p_x = [0,1,0,-1], p_y = 0.  With H = 1 the three window rows
    # dy = -1, 0, 1 all fall on row 0, so each column offset dx carries the
    # weight sum c_dx = sum_dy exp(-(dx^2 + dy^2)/2):  a = exp(-1/2),
    # c_0 = 1 + 2a,  c_1 = a + 2a^2.
    a = math.exp(-0.5)
    c0, c1 = 1 + 2 * a, a + 2 * a * a
    f = np.array([[0.0, 0.0, 1.0, 1.0]])
    # range kernel off: g_x = [0, b, 0, -b], b = c0 / (c0 + 2 c1) = 1 / (1 + 2a)
    b = 1.0 / (1.0 + 2.0 * a)
    u, gx, gy = oracle.smooth_channel(f, lam, 1.0, math.inf, radius=1, return_fields=True)
    assert np.allclose(gx, [[0, b, 0, -b]], atol=1e-15)
    assert np.allclose(gy, 0.0, atol=1e-15)
    # normal equations: (I + lam Dx^T Dx) u = f + lam Dx^T g_x, with
    # Dx^T g_x = [-b,-b,b,b] = b e, e = [-1,-1,1,1], and Dx^T Dx e = 2 e.
    # Hence u = 1/2 + gamma e, gamma = (1/2 + lam b) / (1 + 2 lam).
    gamma = (0.5 + lam * b) / (1.0 + 2.0 * lam)
    assert np.allclose(u, [[0.5 - gamma, 0.5 - gamma, 0.5 + gamma, 0.5 + gamma]], atol=1e-12)
    # range kernel on, sigma_r = 1: the neighbours of p = +-1 differ by 1 -> weight a,
    # the neighbours of p = 0 cancel -> b' = c0 / (c0 + 2 a c1)
    u2, gx2, _ = oracle.smooth_channel(f, lam, 1.0, 1.0, radius=1, return_fields=True)
    b2 = c0 / (c0 + 2 * a * c1)
    assert np.allclose(gx2, [[0, b2, 0, -b2]], atol=1e-15)
    gamma2 = (0.5 + lam * b2) / (1.0 + 2.0 * lam)
    assert np.allclose(u2, [[0.5 - gamma2, 0.5 - gamma2, 0.5 + gamma2, 0.5 + gamma2]], atol=1e-12)


# ---------------------------------------------------------------------------
# P4-P6, P8: special cases and invariants of the whole method
# ---------------------------------------------------------------------------

def test_P4_lambda_zero_is_identity():
    f = voronoi_image(40, 56, 3)
    u = oracle.smooth(f, 0.0, 2.0, 0.1)
    assert np.max(np.abs(u - f)) < 1e-13


def test_P5_constant_image_unchanged():
    f = np.full((24, 30), 0.37)
    for lam in (1.0, 1024.0):
        assert np.max(np.abs(oracle.smooth(f, lam, 2.0, 0.1) - f)) < 1e-12


def test_P6_identity_filter_keeps_f():
    # r = 0 makes the filter the identity, g = D f, and (I + lam D^T D) f = f + lam D^T D f
    f = voronoi_image(32, 48, 5)
    for lam in (0.5, 20.0, 1024.0):
        u = oracle.smooth(f, lam, 3.0, 0.1, radius=0)
        assert np.max(np.abs(u - f)) < 1e-10


def test_P8_mean_preserved():
    f = voronoi_image(48, 64, 11)
    u = oracle.smooth(f, 20.0, 2.0, 0.1)
    assert abs(u.mean() - f.mean()) < 1e-13


# ---------------------------------------------------------------------------
# P7: range kernel off => Gaussian-filtered gradients; closed form in Fourier space
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("H,W,ss,r", [(32, 40, 1.5, 5), (9, 7, 2.0, 6)])
def test_P7_sigma_r_infinite_closed_form(H, W, ss, r):
    lam = 30.0
    f = voronoi_image(H, W, 21)
    u = oracle.smooth(f, lam, ss, math.inf, radius=r)
    # normalised periodic truncated Gaussian as an image (offsets summed mod size)
    K = np.zeros((H, W))
    tot = 0.0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2 * ss * ss))
            K[dy % H, dx % W] += w
            tot += w
    G = np.fft.fft2(K / tot)  # real: the kernel is symmetric
    kx = np.arange(W)[None, :]
    ky = np.arange(H)[:, None]
    S = 4 * np.sin(np.pi * kx / W) ** 2 + 4 * np.sin(np.pi * ky / H) ** 2
    U = np.fft.fft2(f) * (1 + lam * S * G) / (1 + lam * S)
    assert np.max(np.abs(np.real(np.fft.ifft2(U)) - u)) < 1e-12


# ---------------------------------------------------------------------------
# P9: g == 0 gives the LS model, Eq. (5)/(6); P14: LS cannot enlarge gradients
# ---------------------------------------------------------------------------

def test_P9_zero_fields_give_ls():
    f = voronoi_image(10, 12, 2)
    z = np.zeros_like(f)
    for lam in (0.5, 8.0):
        dense = oracle.dense_blfls_solve(f, z, z, lam)
        assert np.max(np.abs(oracle.ls_solve(f, lam) - dense)) < 1e-12
        assert np.max(np.abs(oracle.blfls_solve(f, z, z, lam) - dense)) < 1e-12


def test_P14_ls_shrinks():
    f = voronoi_image(64, 64, 9)
    for lam in (1.0, 100.0):
        u = oracle.ls_solve(f, lam)
        assert np.linalg.norm(_dx_loop(u)) <= np.linalg.norm(_dx_loop(f)) + 1e-12
        assert np.linalg.norm(_dy_loop(u)) <= np.linalg.norm(_dy_loop(f)) + 1e-12
        assert np.linalg.norm(u) <= np.linalg.norm(f) + 1e-12


# ---------------------------------------------------------------------------
# P10: the gradients of u approach BLF(grad f) as lambda grows (Fig. 5(b) trend)
# ---------------------------------------------------------------------------

def test_P10_msd_decreases_with_lambda():
    f = voronoi_image(48, 48, 13)
    msd = []
    for lam in (1.0, 4.0, 32.0, 256.0, 1024.0, 8192.0):
        u, gx, gy = oracle.smooth_channel(f, lam, 2.0, 0.1, return_fields=True)
        msd.append(np.mean((_dx_loop(u) - gx) ** 2 + (_dy_loop(u) - gy) ** 2))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(msd, msd[1:]))
    assert msd[-1] < 0.5 * msd[0]
    # the filtered fields are not an exact gradient field, so the floor is the
    # residual of their least-squares projection onto gradients (lambda -> inf)
    u, gx, gy = oracle.smooth_channel(f, 1e10, 2.0, 0.1, return_fields=True)
    floor = np.mean((_dx_loop(u) - gx) ** 2 + (_dy_loop(u) - gy) ** 2)
    assert floor <= msd[-1] * (1 + 1e-9) and msd[-1] - floor < 0.05 * (msd[0] - floor)


# ---------------------------------------------------------------------------
# P11: symmetries
# ---------------------------------------------------------------------------

def test_P11_symmetries():
    f = voronoi_image(24, 36, 17)
    lam, ss, sr = 20.0, 2.0, 0.1
    u = oracle.smooth(f, lam, ss, sr)
    # transpose swaps the axes (and so the two fields)
    assert np.max(np.abs(oracle.smooth(f.T.copy(), lam, ss, sr) - u.T)) < 1e-12
    # circular shift
    sh = (5, -7)
    assert np.max(np.abs(oracle.smooth(np.roll(f, sh, (0, 1)), lam, ss, sr) - np.roll(u, sh, (0, 1)))) < 1e-12
    # negation
    assert np.max(np.abs(oracle.smooth(-f, lam, ss, sr) + u)) < 1e-12
    # affine map with sigma_r scaled by |a|
    a, b = -2.5, 0.75
    ua = oracle.smooth(a * f + b, lam, ss, sr * abs(a))
    assert np.max(np.abs(ua - (a * u + b))) < 1e-11


# ---------------------------------------------------------------------------
# P12: lambda -> infinity: grad u is the least-squares fit to g; the mean stays
# ---------------------------------------------------------------------------

def test_P12_large_lambda_limit():
    H, W = 20, 28
    f = voronoi_image(H, W, 19)
    u, gx, gy = oracle.smooth_channel(f, 1e9, 2.0, 0.1, return_fields=True)
    kx = np.arange(W)[None, :]
    ky = np.arange(H)[:, None]
    ex = np.exp(2j * np.pi * kx / W) - 1 + 0 * ky
    ey = np.exp(2j * np.pi * ky / H) - 1 + 0 * kx
    S = np.abs(ex) ** 2 + np.abs(ey) ** 2
    S[0, 0] = 1.0
    U = (np.conj(ex) * np.fft.fft2(gx) + np.conj(ey) * np.fft.fft2(gy)) / S
    U[0, 0] = f.sum()
    lim = np.real(np.fft.ifft2(U))
    assert np.max(np.abs(u - lim)) < 1e-6


# ---------------------------------------------------------------------------
# P13: variants that reduce to the plain method
# ---------------------------------------------------------------------------

def test_P13_joint_with_self_guide_and_single_iteration():
    f = voronoi_image(30, 26, 23)
    u = oracle.smooth(f, 20.0, 2.0, 0.1)
    assert np.max(np.abs(oracle.smooth(f, 20.0, 2.0, 0.1, guide=f) - u)) < 1e-14
    assert np.max(np.abs(oracle.smooth(f, 20.0, 2.0, 0.1, iterations=1) - u)) < 1e-14


def test_rolling_guidance_composes():
    # iteration 2 is the joint filter guided by iteration 1's output
    f = voronoi_image(30, 26, 29)
    u1 = oracle.smooth(f, 20.0, 2.0, 0.1)
    u2 = oracle.smooth(f, 20.0, 2.0, 0.1, iterations=2)
    assert np.max(np.abs(u2 - oracle.smooth(f, 20.0, 2.0, 0.1, guide=u1))) < 1e-14
    u3 = oracle.smooth(f, 20.0, 2.0, 0.1, iterations=3)
    assert np.max(np.abs(u3 - oracle.smooth(f, 20.0, 2.0, 0.1, guide=u2))) < 1e-14


def test_normalisation_is_a_range_rescale():
    # mapping a field to [0,1] before Eq. (1) and back after equals the raw filter
    # with sigma_r scaled by the field's span (the weights see only differences)
    f = voronoi_image(28, 34, 31) * 0.6 + 0.1
    lam, ss, sr = 20.0, 2.0, 0.2
    un = oracle.smooth(f, lam, ss, sr, normalize=True)
    px, py = _dx_loop(f), _dy_loop(f)
    r = oracle.default_radius(ss)
    gx = oracle.bilateral_filter_bruteforce(px, None, ss, sr * (px.max() - px.min()), r)
    gy = oracle.bilateral_filter_bruteforce(py, None, ss, sr * (py.max() - py.min()), r)
    assert np.max(np.abs(un - oracle.dense_blfls_solve(f, gx, gy, lam))) < 1e-10


def test_multichannel_is_per_channel():
    f = np.stack([voronoi_image(16, 20, s) for s in (1, 2, 3)])
    u = oracle.smooth(f, 20.0, 1.5, 0.1)
    for c in range(3):
        assert np.array_equal(u[c], oracle.smooth(f[c], 20.0, 1.5, 0.1))


def test_gaussian_blur_normalised_and_symmetric():
    img = np.zeros((15, 15))
    img[7, 7] = 1.0
    b = oracle.gaussian_blur(img, 1.2)
    assert abs(b.sum() - 1.0) < 1e-14
    assert np.allclose(b, b.T) and np.allclose(b, b[::-1, ::-1])
    assert b[7, 7] == b.max()


@pytest.mark.parametrize("sigma", [0.7, 1.2, 1.7, 2.5])
def test_gaussian_blur_is_the_library_gaussian_on_a_torus(sigma):
    """The initial guide's smoothing (Section III-D) against scipy's Gaussian filter with
    the same radius ceil(3 sigma) and wrap-around borders: an independent implementation
    of the normalised sampled Gaussian (separable, so its 2-D normalisation is the product
    of the 1-D ones)."""
    from scipy import ndimage
    img = np.random.default_rng(31).random((23, 29))
    r = int(math.ceil(3.0 * sigma))
    ref = ndimage.gaussian_filter(img, sigma, mode="wrap", radius=r)
    assert np.max(np.abs(oracle.gaussian_blur(img, sigma) - ref)) < 1e-14


@pytest.mark.parametrize("sigma", [0.9, 1.7, 2.5])
def test_gaussian_blur_impulse_support_and_variance(sigma):
    """Impulse response: nonzero exactly on the square of radius ceil(3 sigma), rank one
    (Euclidean distance makes the 2-D Gaussian separable), and a second moment per axis
    of sigma^2 up to the truncation at 3 sigma (which removes less than 3% of it)."""
    n = 41
    img = np.zeros((n, n))
    img[n // 2, n // 2] = 1.0
    b = oracle.gaussian_blur(img, sigma)
    r = int(math.ceil(3.0 * sigma))
    k = np.arange(n) - n // 2
    inside = (np.abs(k)[:, None] <= r) & (np.abs(k)[None, :] <= r)
    assert np.all(b[inside] > 0) and np.all(b[~inside] == 0)
    s = np.linalg.svd(b, compute_uv=False)
    assert s[1] < 1e-12 * s[0]
    var_y = float(np.sum(b * (k[:, None] ** 2)))
    assert 0.97 * sigma ** 2 < var_y <= sigma ** 2 * (1 + 1e-9)


@pytest.mark.parametrize("sigma_s,s", [(0.3, 1), (1.0, 1), (1.49, 1), (1.5, 2), (2.5, 3), (3.0, 3),
                                       (7.6, 8), (8.0, 8), (8.5, 9), (20.0, 20)])
def test_grid_cell_hand_derived(sigma_s, s):
    """Cell size: sigma_s rounded to whole pixels, halves up, at least one pixel."""
    assert oracle.grid_cell(sigma_s) == s


def test_grid_range_hand_derived_bins():
    """Bins worked by hand: q = (0, 0.25, 0.26, 0.74, 1) with sigma_r = 0.5 gives inv = 2,
    t = (0, 0.5, 0.52, 1.48, 2) and bins floor(t + 1/2) = (0, 1, 1, 1, 2) (a half rounds
    up); a field spanning [-1, 1] with sigma_r = 0.01 would need 200 bins, so inv drops
    to 31 / 2 = 15.5 and q = (-1, -0.5, 0, 0.5, 1) fall in bins (0, 8, 16, 23, 31): t = (0,
    7.75, 15.5, 23.25, 31), so 32 bins."""
    q = np.array([[0.0, 0.25, 0.26, 0.74, 1.0]])
    qmin, inv, z, nz = oracle.grid_range(q, 0.5)
    assert qmin == 0.0 and abs(inv - 2.0) < 1e-7 and nz == 3
    assert z.tolist() == [[0, 1, 1, 1, 2]]
    q = np.array([[-1.0, -0.5, 0.0, 0.5, 1.0]])
    qmin, inv, z, nz = oracle.grid_range(q, 0.01)
    assert qmin == -1.0 and inv == 15.5 and nz == oracle.GRID_ZMAX
    assert z.tolist() == [[0, 8, 16, 23, 31]]
    # the same field with normalisation (inv_span = 1/2) and sigma_r = 0.25: 2 bins per unit
    qmin, inv, z, nz = oracle.grid_range(q, 0.25, 0.5)
    assert abs(inv - 2.0) < 1e-7 and z.tolist() == [[0, 1, 2, 3, 4]] and nz == 5


def test_grid_bin_margin_hand_derived():
    """t + 1/2 = (0.5, 1.0, 1.02, 1.98, 2.5) for the first field above: the closest
    decision is the exact half (margin 0); without it, 0.02."""
    q = np.array([[0.0, 0.25, 0.26, 0.74, 1.0]])
    assert oracle.grid_bin_margin(q, 0.5) < 1e-7
    q = np.array([[0.0, 0.26, 0.74, 1.0]])
    assert abs(oracle.grid_bin_margin(q, 0.5) - 0.02) < 1e-7
    # the cap decision: span 2 at inv 15.4 is 30.8 bins, 0.2 from the cap at 31
    q = np.array([[-1.0, 1.0]])
    assert abs(oracle.grid_bin_margin(q, 1.0 / 15.4) - 0.2) < 1e-6


def test_nc_decision_margin_by_loops():
    """The NC filter's smallest decision margin against explicit walks over every pixel,
    direction and pass (tiny field)."""
    rng = np.random.default_rng(5)
    q = rng.random((5, 7))
    ss, sr = 2.0, 0.7
    s32, r32 = float(np.float32(ss)), float(np.float32(sr))
    a = s32 / r32
    best = math.inf
    for rad in oracle.nc_schedule(s32, 3):
        for line_set in (q, q.T):
            for line in line_set:
                n = len(line)
                for j in range(n):
                    for step in (1, -1):
                        dist = 0.0
                        m = j
                        while 0 <= m + step < n:
                            nxt = m + step
                            dist += 1.0 + a * abs(line[nxt] - line[m])
                            best = min(best, abs(dist - rad))
                            m = nxt
                            if dist > rad:
                                break
    assert abs(oracle.nc_decision_margin(q, ss, sr, 3) - best) < 1e-12


@pytest.mark.parametrize("H,W,r,sr,joint", [(5, 7, 2, 0.3, False), (4, 6, 5, 0.2, True), (3, 3, 4, math.inf, False),
                                            (6, 5, 1, 0.05, True)])
def test_c_blf_matches_pixel_loops(H, W, r, sr, joint):
    """The C loops of Eq. (1) (oracle/blf_oracle.c) against the Python pixel loops,
    windows wider than the image included."""
    from oracle.c_blf import bilateral_filter_c
    rng = np.random.default_rng(H * W + r)
    p = rng.random((H, W))
    q = rng.random((H, W)) if joint else None
    a = bilateral_filter_c(p, q, 1.3, sr, r)
    b = oracle.bilateral_filter_bruteforce(p, q, 1.3, sr, r)
    assert np.max(np.abs(a - b)) < 1e-14


def test_c_engine_gives_the_numpy_result():
    f = voronoi_image(40, 52, 12)
    g = voronoi_image(40, 52, 13)
    for kw in (dict(), dict(guide=g), dict(iterations=2, sigma_guide=1.0), dict(normalize=True)):
        a = oracle.smooth(f, 30.0, 2.0, 0.08, engine="c", **kw)
        b = oracle.smooth(f, 30.0, 2.0, 0.08, **kw)
        assert np.max(np.abs(a - b)) < 1e-13, kw
