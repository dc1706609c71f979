"""GPU parity of the symmetric-pair filter path (one exp per unordered pair of taps
of Eq. (1)) against the FP64 oracle, through the C ABI.

The path cuts each image into bands of at most 64 columns and whole blocks of
rows; one wave sweeps a band, the partial sums that leave a band (sources whose
partner lies in a neighbouring band, rows past the band) go to a merge pass.
The cases below put every one of those hand-overs to work: several column and
row bands, ragged widths and heights, a last block cut by the image edge, one
band that wraps onto itself in either direction, radius classes 8 to 32 with r
below its class, joint fields, the range kernel off, normalising, rolling
guidance and 16-bit field storage; blocks of eight rows (classes 8 and 9) and of four
(classes 10 and up).  Radius classes below 8 and images too small
for bands at least R wide and R + K - 1 tall take the tile kernel (the other
GPU tests); the workspace test shows which path a request takes.
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image, voronoi_rgb, joint_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_MIXED = 2e-3


def blfls():
    import paper_1812_07122_amd as b
    return b


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _smooth(f, guide=None, **kw):
    f32 = np.asarray(f, dtype=np.float32)
    g32 = None if guide is None else np.asarray(guide, dtype=np.float32)
    u = blfls().smooth(_gpu(f32), guide=None if g32 is None else _gpu(g32), **kw)
    torch.cuda.synchronize()
    return (u.cpu().numpy().astype(np.float64), f32.astype(np.float64),
            None if g32 is None else g32.astype(np.float64))


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


@pytest.mark.parametrize("H,W,ss,r,pair", [
    (64, 200, 3.0, 9, True),      # R = 9: 4 column bands of 50, 8-row blocks
    (72, 90, 8.0, 24, True),      # R = 24: 2 x 2 bands, 4-row blocks
    (40, 20, 2.0, 9, True),       # one column band of 20 >= R
    (64, 200, 1.0, 3, False),     # radius class 3: the tile kernel
    (12, 200, 3.0, 9, False),     # 12 rows < R + K - 1: the tile kernel
    (64, 16, 3.0, 9, True),       # one band of 16 >= 9 columns
    (64, 16, 6.0, 18, False),     # 16 columns < R = 20
])
def test_path_selection_by_workspace(H, W, ss, r, pair):
    """A request on the pair path needs the partial-sum records beyond the plan's
    workspace; a tile-kernel request needs exactly the plan's."""
    b = blfls()
    plan = b.Plan(H, W, 1)
    prm = b.make_params(10.0, ss, 0.1, r)
    need = plan.workspace_for(prm)
    assert (need > plan.workspace_bytes) == pair, (need, plan.workspace_bytes)


@pytest.mark.parametrize("H,W,ss,sr,r,lam", [
    (40, 72, 3.0, 0.3, 9, 20.0),       # 2 column bands of 36, 5 blocks: one row band
    (36, 120, 2.7, 0.4, 8, 10.0),      # class 8, two bands of 60
    (45, 250, 2.7, 0.4, 8, 10.0),      # 4 bands of 62-63 (unaligned starts), last block of 5 rows
    (64, 200, 4.0, 0.1, 12, 30.0),     # class 12
    (25, 20, 2.0, 0.5, 9, 5.0),        # one band each way: sums wrap onto the band itself
    (96, 300, 8.0, 0.05, 24, 50.0),    # class 24 (4-row blocks), the headline's weights
    (72, 90, 10.0, 0.1, 30, 20.0),     # class 32, r = 30 < R: rows and columns past r weigh 0
    (80, 128, 7.0, 0.1, 22, 20.0),     # class 24, r = 22
    (160, 64, 5.0, 0.1, 16, 20.0),     # class 16, one column band of 64, several row bands
    (54, 150, 6.0, 0.15, 20, 40.0),    # class 20, H = 54: last block of 2 rows
    (90, 256, 9.0, 0.1, 28, 20.0),     # class 28
    (48, 160, 3.3, 0.2, 10, 15.0),     # class 10, the smallest with 4-row blocks
    (75, 150, 4.7, 0.15, 14, 25.0),    # class 14, 3 x 3 bands, a last block of 3 rows
    (64, 1200, 4.0, 0.1, 12, 20.0),    # two merge segments of 1024 columns, the second partial
])
def test_pair_path_parity(H, W, ss, sr, r, lam):
    f = voronoi_image(H, W, 1000 + H + W + r)
    u, fin, _ = _smooth(f, lam=lam, sigma_s=ss, sigma_r=sr, radius=r)
    ref = oracle.smooth(fin, lam, ss, sr, radius=r)
    err = float(np.max(np.abs(u - ref)))
    print(f"pair {H}x{W} r={r}: max-abs {err:.3e}")
    assert err <= TOL_FP32


@pytest.mark.parametrize("H,W,ss,r", [(40, 72, 3.0, 9), (72, 90, 10.0, 30), (64, 200, 8.0, 24),
                                      (64, 128, 4.0, 12), (80, 96, 5.3, 16)])
def test_pair_path_joint(H, W, ss, r):
    t, g = joint_pair(H, W, 5)
    u, tin, gin = _smooth(t, g, lam=30.0, sigma_s=ss, sigma_r=0.1, radius=r)
    ref = oracle.smooth(tin, 30.0, ss, 0.1, radius=r, guide=gin)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_pair_path_range_off_normalize_rolling():
    f = voronoi_image(96, 128, 77)
    u, fin, _ = _smooth(f, lam=20.0, sigma_s=3.0, sigma_r=math.inf)
    assert np.max(np.abs(u - oracle.smooth(fin, 20.0, 3.0, math.inf))) <= TOL_FP32
    u, fin, _ = _smooth(f, lam=20.0, sigma_s=3.0, sigma_r=0.3, normalize=True)
    assert np.max(np.abs(u - oracle.smooth(fin, 20.0, 3.0, 0.3, normalize=True))) <= TOL_FP32
    u, fin, _ = _smooth(f, lam=20.0, sigma_s=3.0, sigma_r=0.1, iterations=2, sigma_guide=1.5)
    ref = oracle.smooth(fin, 20.0, 3.0, 0.1, iterations=2, sigma_guide=1.5)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_pair_path_16_bit_fields(precision):
    f = voronoi_rgb(128, 160, 9)
    u, fin, _ = _smooth(f, lam=30.0, sigma_s=4.0, sigma_r=0.1, precision=precision)
    ref = oracle.smooth(fin, 30.0, 4.0, 0.1)
    err = float(np.max(np.abs(u - ref)))
    assert err <= TOL_MIXED and _psnr(u, ref) >= 50.0, (err, _psnr(u, ref))


def test_pair_path_channels_bitwise_independent_and_repeatable():
    """The decomposition depends on the image shape only: a channel of an RGB call
    equals, bit for bit, the same channel filtered alone, and calls repeat exactly."""
    f = voronoi_rgb(96, 200, 4).astype(np.float32)
    u3, _, _ = _smooth(f, lam=20.0, sigma_s=4.0, sigma_r=0.1)
    u3b, _, _ = _smooth(f, lam=20.0, sigma_s=4.0, sigma_r=0.1)
    assert np.array_equal(u3, u3b)
    for c in range(3):
        u1, _, _ = _smooth(f[c], lam=20.0, sigma_s=4.0, sigma_r=0.1)
        assert np.array_equal(u1, u3[c])


def test_pair_path_served_graphs_equal_direct_calls():
    """Served steps replay captured graphs of the persistent pair kernels (band items
    drawn from a counter, any band of any request in any order): every result equals
    its direct call bit for bit, for radius classes 12 and 24, self and joint."""
    import time
    b = blfls()
    reqs = []
    for k in range(12):
        H, W = [(72, 90), (96, 128), (64, 200)][k % 3]
        f = voronoi_image(H, W, 2100 + k)
        prm = dict(lam=[20.0, 50.0][k % 2], sigma_s=[4.0, 8.0][(k // 2) % 2], sigma_r=0.1)
        guide = voronoi_image(H, W, 2200 + k) if k % 4 == 3 else None
        reqs.append((f, guide, prm))
    server = b.Server(arena_bytes=256 << 20, max_slots=6, precision="fp32")
    pending = []
    for f, guide, prm in reqs:
        g = None if guide is None else _gpu(guide)
        pending.append(server.submit(_gpu(f), guide=g, **prm))
    deadline = time.time() + 60
    for t, u in pending:
        while True:
            state, status = server.poll(t)
            if state in (b.DONE, b.FAILED):
                break
            assert time.time() < deadline
            time.sleep(0.001)
        assert state == b.DONE and status == 0
    server.stream.synchronize()
    stats = server.stats()
    assert stats["graph_steps"] >= 1
    server.close()
    for (f, guide, prm), (_, u) in zip(reqs, pending):
        g = None if guide is None else _gpu(guide)
        alone = b.smooth(_gpu(f), guide=g, **prm)
        torch.cuda.synchronize()
        assert torch.equal(alone, u), prm


def _smooth235(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def test_pair_path_random_layouts():
    """Seeded random shapes (H and W/2 with factors 2, 3, 5 only), radius classes 8-32,
    self- and joint-guided, three range scales: every case element by element against
    the oracle.  Most take the pair path; the rest (bands narrower than R, images
    shorter than R + K - 1) the tile kernel, counted in the message."""
    b = blfls()
    heights = [n for n in range(16, 241) if _smooth235(n)]
    widths = [2 * n for n in range(8, 161) if _smooth235(n)]
    rng = np.random.default_rng(2024)
    on_pair = 0
    for case in range(24):
        H, W = int(rng.choice(heights)), int(rng.choice(widths))
        r = int(rng.integers(8, 33))
        joint = bool(rng.integers(0, 2))
        sr = float(rng.choice([0.05, 0.1, 0.3]))
        lam = float(rng.uniform(5, 60))
        plan = b.Plan(H, W, 1)
        on_pair += plan.workspace_for(b.make_params(lam, r / 3.0, sr, r)) > plan.workspace_bytes
        plan.close()
        print(f"case {case}: {H}x{W} r={r} joint={joint} sigma_r={sr}", flush=True)
        f = voronoi_image(H, W, 7000 + case)
        g = joint_pair(H, W, 7100 + case)[1] if joint else None
        u, fin, gin = _smooth(f, g, lam=lam, sigma_s=r / 3.0, sigma_r=sr, radius=r)
        ref = oracle.smooth(fin, lam, r / 3.0, sr, radius=r, guide=gin)
        err = float(np.max(np.abs(u - ref)))
        assert err <= TOL_FP32, (H, W, r, joint, err)
    print(f"{on_pair} of 24 cases on the pair path")
    assert on_pair >= 16


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_served_random_mixes_equal_direct_calls(precision):
    """Seeded random requests (radius classes 2-32 on both filter paths, RGB and
    grey, self- and joint-guided, normalising, one or two rolling iterations)
    served in one mix: each result equals the same request run alone, bit for bit."""
    import time
    b = blfls()
    heights = [n for n in range(24, 200) if _smooth235(n)]
    widths = [2 * n for n in range(16, 150) if _smooth235(n)]
    rng = np.random.default_rng(31 if precision == "fp32" else 32)
    reqs = []
    for k in range(16):
        H, W, C = int(rng.choice(heights)), int(rng.choice(widths)), int(rng.choice([1, 3]))
        r = int(rng.integers(2, 33))
        prm = dict(lam=float(rng.uniform(5, 100)), sigma_s=r / 3.0, sigma_r=float(rng.uniform(0.03, 0.3)),
                   radius=r, iterations=int(rng.integers(1, 3)), normalize=bool(rng.integers(0, 4) == 0))
        f = np.stack([voronoi_image(H, W, 8000 + 3 * k + c) for c in range(C)])
        g = np.stack([voronoi_image(H, W, 8500 + 3 * k + c) for c in range(C)]) if rng.integers(0, 3) == 0 else None
        reqs.append((_gpu(f), None if g is None else _gpu(g), prm))
    server = b.Server(arena_bytes=512 << 20, max_slots=8, precision=precision)
    pending = [server.submit(f, guide=g, **prm) for f, g, prm in reqs]
    deadline = time.time() + 60
    for t, _ in pending:
        while True:
            state, status = server.poll(t)
            if state in (b.DONE, b.FAILED):
                break
            assert time.time() < deadline
            time.sleep(0.001)
        assert state == b.DONE and status == 0
    server.stream.synchronize()
    server.close()
    for (f, g, prm), (_, u) in zip(reqs, pending):
        alone = b.smooth(f, guide=g, precision=precision, **prm)
        torch.cuda.synchronize()
        assert torch.equal(alone, u), prm
