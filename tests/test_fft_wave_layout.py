"""CPU checks of the index algebra behind the wave-resident Fourier passes
(one transform of length N = 64 L per wave, lane l holding elements l + 64 m).

The factorisation X[k1 + L k2] = sum_l W_64^(l k2) W_N^(l k1) sum_m x[l + 64 m]
W_L^(m k1), with the 64-point DFTs over the lanes split 8 x 8 and the inverse
retracing the steps with conjugate twiddles, is replayed here lane by lane in
NumPy and compared with numpy.fft; the LDS slot map of the exchanges is checked
to be a bijection per block and free of bank conflicts for the three access
patterns the kernels use (16 lanes at a time, 8-byte elements over 32 banks of
4 bytes: a 16-lane group is conflict-free when its 16 slots differ mod 16).
"""
import numpy as np
import pytest


def wslot(k1, row, col):
    return k1 * 64 + (((row + k1) & 7) << 3) + (col ^ row)


def dft(v, sg):
    r = len(v)
    t = np.arange(r)
    return np.array([np.sum(v * np.exp(sg * 2j * np.pi * t * k / r)) for k in range(r)])


def w(n, e):
    return np.exp(-2j * np.pi * np.asarray(e) / n)


def four_step_forward(x, L):
    """Lane-level replay: returns X in the registers' layout {(k1, k2a, k2b): value}."""
    N = 64 * L
    T = np.zeros(L * 64, complex)
    for l in range(64):
        a = dft(np.array([x[l + 64 * m] for m in range(L)]), -1) * w(N, l * np.arange(L))
        for k1 in range(L):
            T[wslot(k1, l >> 3, l & 7)] = a[k1]
    for p in range(8 * L):                 # 8-point DFTs over l2, twiddle W_64^(l1 k2a)
        k1, l1 = p >> 3, p & 7
        b = dft(np.array([T[wslot(k1, r, l1)] for r in range(8)]), -1) * w(64, l1 * np.arange(8))
        for r in range(8):
            T[wslot(k1, r, l1)] = b[r]
    out = {}
    for p in range(8 * L):                 # 8-point DFTs over l1
        k1, k2a = p >> 3, p & 7
        d = dft(np.array([T[wslot(k1, k2a, c)] for c in range(8)]), -1)
        for k2b in range(8):
            out[(k1, k2a, k2b)] = d[k2b]
    return out


def four_step_inverse(regs, L):
    N = 64 * L
    T = np.zeros(L * 64, complex)
    for p in range(8 * L):
        k1, k2a = p >> 3, p & 7
        d = dft(np.array([regs[(k1, k2a, k2b)] for k2b in range(8)]), 1)
        for c in range(8):
            T[wslot(k1, k2a, c)] = d[c]
    for p in range(8 * L):
        k1, l1 = p >> 3, p & 7
        e = dft(np.array([T[wslot(k1, r, l1)] for r in range(8)]) * np.conj(w(64, l1 * np.arange(8))), 1)
        for r in range(8):
            T[wslot(k1, r, l1)] = e[r]
    y = np.zeros(N, complex)
    for l in range(64):
        z = np.array([T[wslot(k1, l >> 3, l & 7)] for k1 in range(L)]) * np.conj(w(N, l * np.arange(L)))
        e = dft(z, 1)
        for m in range(L):
            y[l + 64 * m] = e[m]
    return y


@pytest.mark.parametrize("L", [8, 16])
def test_four_step_forward_and_inverse(L):
    N = 64 * L
    rng = np.random.default_rng(L)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    regs = four_step_forward(x, L)
    X = np.fft.fft(x)
    got = np.zeros(N, complex)
    for (k1, k2a, k2b), v in regs.items():
        got[k1 + L * (k2a + 8 * k2b)] = v
    assert np.max(np.abs(got - X)) < 1e-9 * np.max(np.abs(X))
    # a spectral scale between the two transforms, as the column pass applies the divide
    s = 1.0 / (1.0 + rng.random(N))
    scaled = {key: v * s[key[0] + L * (key[1] + 8 * key[2])] for key, v in regs.items()}
    y = four_step_inverse(scaled, L)
    ref = np.fft.ifft(X * s) * N
    assert np.max(np.abs(y - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("L", [8, 16])
def test_slot_map_is_a_bijection(L):
    slots = {wslot(k1, r, c) for k1 in range(L) for r in range(8) for c in range(8)}
    assert slots == set(range(64 * L))


@pytest.mark.parametrize("L", [8, 16])
def test_exchanges_are_free_of_bank_conflicts(L):
    for q in range(L // 8):
        for g in range(4):                       # 16-lane groups of the wave
            lanes = range(16 * g, 16 * g + 16)
            pairs = [(p >> 3, p & 7) for p in (l + 64 * q for l in lanes)]
            for fixed in range(8):
                # column reads and writes: (k1, l1) pairs, one row per instruction
                assert len({wslot(k1, fixed, l1) % 16 for k1, l1 in pairs}) == 16
                # row reads: (k1, k2a) pairs, one column per instruction
                assert len({wslot(k1, k2a, fixed) % 16 for k1, k2a in pairs}) == 16
    for k1 in range(L):
        # lane-order transposes: lane l at (l >> 3, l & 7), one block per instruction
        for g in range(4):
            got = [wslot(k1, l >> 3, l & 7) % 16 for l in range(16 * g, 16 * g + 16)]
            assert len(set(got)) == 16
