"""CPU check of the symmetric-pair filter's work split (no GPU): a float64 model of
the kernel's bookkeeping (lanes = columns of a band of at most 64, blocks of K rows,
partner sums kept per lane, source sums shifted one lane per column-offset step and
stored when they leave the band, the merge pass) reproduces Eq. (1) of the oracle
to rounding, for several band layouts.  A pair {s, s + d}, d in {dy > 0} u {dy = 0,
dx > 0}, must be evaluated exactly once and its weight must reach both pixels: a
pair lost at a band edge, a carry-over row added twice or a shift in the wrong
direction changes the result by far more than rounding.  The model takes the
kernel's loop order (dx = r..1 with the sources to the left, then dx = -r..0 with
the sources to the right, the own column last) but not its arithmetic order.
"""
import math

import numpy as np
import pytest

import oracle

LOG2E = 1.4426950408889634
HUGE = 1e30


def _bounds(n, nb):
    return [(i * n) // nb for i in range(nb + 1)]


def pair_model(p, q, sigma_s, sigma_r, r, R, K, joint, nbx, nby):
    """Residual BLF(p) - p of one field by the pair decomposition (q: range source)."""
    H, W = p.shape
    c = math.sqrt(LOG2E / (2 * sigma_r * sigma_r)) if math.isfinite(sigma_r) else 0.0
    qq = c * q
    pw = np.array([[-(dx * dx + dy * dy) * LOG2E / (2 * sigma_s * sigma_s) if max(dx, dy) <= r else -np.inf
                    for dy in range(R + 1)] for dx in range(R + 1)])
    T = -(-H // K)
    cb = _bounds(W, nbx)
    rb = _bounds(T, nby)
    L, NJ = 64, K + R
    lane = np.arange(L)
    main, left, right = {}, {}, {}
    for by in range(nby):
        Y0, nblk = rb[by] * K, rb[by + 1] - rb[by]
        Y1 = min(H, Y0 + nblk * K)
        for bx in range(nbx):
            x0, wb = cb[bx], cb[bx + 1] - cb[bx]
            ok = lane < wb
            xo = np.where(ok, x0 + lane, x0) % W
            M = np.zeros((nblk * K + R, L, 2))
            OL = np.zeros((nblk, R, K, 2))
            OR = np.zeros((nblk, R, K, 2))
            A = np.zeros((NJ, L, 2))
            for b in range(nblk):
                y = Y0 + b * K
                cols = (x0 - R + np.arange(L + 2 * R)) % W
                sq = np.array([qq[y + k, cols] if y + k < Y1 else np.full(L + 2 * R, HUGE) for k in range(K)])
                sp = np.array([p[y + k, cols] if y + k < Y1 else np.zeros(L + 2 * R) for k in range(K)])
                vq = np.array([np.where(ok, qq[(y + j) % H, xo], -HUGE) for j in range(NJ)])
                vp = np.array([np.where(ok, p[(y + j) % H, xo], 0.0) for j in range(NJ)])

                def step(B, off, dx, dy0):
                    for dy in range(dy0, R + 1):
                        for k in range(K):
                            j = k + dy
                            d = sq[k, R + lane + off] - vq[j]
                            with np.errstate(over="ignore"):
                                e = np.exp2(pw[dx, dy] - d * d)
                            an, bn = (e * sp[k, R + lane + off], e * vp[j]) if joint else (e * d, e * d)
                            A[j, :, 0] += an
                            A[j, :, 1] += e
                            B[k, :, 0] += bn
                            B[k, :, 1] += e

                sgn = 1.0 if joint else -1.0
                B = np.zeros((K, L, 2))
                for dx in range(r, 0, -1):          # sources dx columns to the left
                    step(B, -dx, dx, 0)
                    OL[b, dx - 1] = B[:, 0, :]     # leaves through lane 0
                    B = np.concatenate([B[:, 1:], np.zeros((K, 1, 2))], axis=1)
                A[:K, :, 0] += sgn * B[:, :, 0]
                A[:K, :, 1] += B[:, :, 1]
                B = np.zeros((K, L, 2))
                for m in range(r, -1, -1):          # sources m columns to the right, own column last
                    if m < r:
                        OR[b, m] = B[:, wb - 1, :]  # the previous step's sums leave through the last lane
                        B = np.concatenate([np.zeros((K, 1, 2)), B[:, :-1]], axis=1)
                    step(B, m, m, 1)
                A[:K, :, 0] += sgn * B[:, :, 0]
                A[:K, :, 1] += B[:, :, 1]
                M[b * K:b * K + K] = A[:K]
                A = np.concatenate([A[K:], np.zeros((K, L, 2))], axis=0)
            M[nblk * K:] = A[:R]
            main[bx, by], left[bx, by], right[bx, by] = M, OL, OR
    out = np.empty((H, W))
    sgn = 1.0 if joint else -1.0
    for Y in range(H):
        t = Y // K
        by = ((t + 1) * nby - 1) // T
        Y0 = rb[by] * K
        ly = Y - Y0
        bya = (by - 1) % nby
        Y0a, nblka = rb[bya] * K, rb[bya + 1] - rb[bya]
        hba = min(H, Y0a + nblka * K) - Y0a
        la = (Y - Y0a) % H
        if la < hba:
            la += H
        for x in range(W):
            bx = ((x + 1) * nbx - 1) // W
            x0, wb = cb[bx], cb[bx + 1] - cb[bx]
            lx = x - x0
            v = main[bx, by][ly, lx].copy()
            if la < nblka * K + R:
                v += main[bx, bya][la, lx]
            bxr = (bx + 1) % nbx
            dr = (cb[bxr] - x) % W or W
            if dr <= r:
                o = left[bxr, by][ly // K, dr - 1, ly % K]
                v += (sgn * o[0], o[1])
            bxl = (bx - 1) % nbx
            dl = (x - (cb[bxl + 1] - 1)) % W or W
            if dl <= r:
                o = right[bxl, by][ly // K, dl - 1, ly % K]
                v += (sgn * o[0], o[1])
            den = 1.0 + v[1]
            out[Y, x] = (p[Y, x] + v[0]) / den - p[Y, x] if joint else v[0] / (c * den)
    return out


@pytest.mark.parametrize("H,W,ss,sr,r,R,K,joint,nbx,nby", [
    (34, 70, 3.0, 0.3, 9, 9, 8, False, 2, 2),     # two bands each way, last block of 2 rows
    (30, 70, 3.0, 0.3, 9, 9, 8, True, 2, 1),      # joint, one row band (carry-over wraps onto itself)
    (28, 20, 2.0, 0.5, 8, 9, 8, False, 1, 1),     # one band each way, r below its class
    (60, 130, 5.0, 0.2, 12, 12, 4, False, 3, 3),  # K = 4, ragged column bands (43, 43, 44)
    (45, 90, 4.0, math.inf, 10, 12, 4, True, 2, 2),  # range kernel off (joint form)
])
def test_pair_decomposition_equals_eq1(H, W, ss, sr, r, R, K, joint, nbx, nby):
    rng = np.random.default_rng(H * W + r)
    p = rng.random((H, W))
    q = rng.random((H, W)) if joint else p
    got = pair_model(p, q, ss, sr, r, R, K, joint, nbx, nby)
    ref = oracle.bilateral_filter(p, q if joint else None, ss, sr, r) - p
    assert np.max(np.abs(got - ref)) < 1e-12
