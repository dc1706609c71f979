"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are FP32 on the device; the oracle runs on float64(float32(input)) so
input rounding is not charged to the GPU.  Plain FP32 results must agree to
max-abs 1e-5 (FP32 filter weights and transforms; the filter-field error is
amplified by at most sqrt(lambda)/2 through the solve).  The 16-bit field
storage paths must agree to max-abs 2e-3 and PSNR >= 50 dB.
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image, voronoi_rgb, joint_pair, config_seed

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_MIXED = 2e-3


def blfls():
    import paper_1812_07122_amd as b
    return b


def _to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _run(f64, guide64=None, **kw):
    f32 = np.asarray(f64, dtype=np.float32)
    g = None if guide64 is None else _to_gpu(guide64)
    u = blfls().smooth(_to_gpu(f32), guide=g, **kw)
    torch.cuda.synchronize()
    ref_in = f32.astype(np.float64)
    ref_guide = None if guide64 is None else np.asarray(guide64, dtype=np.float32).astype(np.float64)
    return u.cpu().numpy().astype(np.float64), ref_in, ref_guide


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


@pytest.mark.parametrize("lam", [1024.0, 20.0])
def test_grayscale_256(lam):
    f = voronoi_image(256, 256, config_seed(0, 0))
    u, fin, _ = _run(f, lam=lam, sigma_s=3.0, sigma_r=0.1)
    ref = oracle.smooth(fin, lam, 3.0, 0.1)
    err = np.max(np.abs(u - ref))
    print(f"256x256 lam={lam}: max-abs {err:.3e}")
    assert err <= TOL_FP32


@pytest.mark.parametrize("H,W,ss,sr,lam", [
    (96, 100, 2.0, 0.1, 20.0),     # ragged tiles in both directions
    (45, 50, 1.0, 0.05, 50.0),     # odd H (3^2 5), W/2 = 25
    (6, 10, 3.0, 0.2, 20.0),       # window wider than the image (periodic copies)
    (1, 2, 1.0, 0.1, 5.0),         # one row, W/2 = 1
    (2, 4, 2.0, 0.1, 5.0),
    (160, 30, 1.5, 0.08, 100.0),   # tall, W < one tile
    (36, 270, 2.5, 0.1, 30.0),     # W/2 = 135 = 3^3 5
])
def test_ragged_and_tiny(H, W, ss, sr, lam):
    f = voronoi_image(H, W, 11 + H + W)
    u, fin, _ = _run(f, lam=lam, sigma_s=ss, sigma_r=sr)
    ref = oracle.smooth(fin, lam, ss, sr)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


@pytest.mark.parametrize("r", [1, 2, 3, 5, 7, 11, 13, 17, 21, 25, 30, 32])
def test_every_radius_class(r):
    H, W = 72, 90
    f = voronoi_image(H, W, 300 + r)
    ss = max(r / 3.0, 0.5)
    u, fin, _ = _run(f, lam=20.0, sigma_s=ss, sigma_r=0.1, radius=r)
    ref = oracle.smooth(fin, 20.0, ss, 0.1, radius=r)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_rgb_channels_independent():
    f = voronoi_rgb(64, 96, 1)
    u, fin, _ = _run(f, lam=20.0, sigma_s=2.0, sigma_r=0.1)
    ref = oracle.smooth(fin, 20.0, 2.0, 0.1)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_four_channels():
    f = np.stack([voronoi_image(40, 48, s) for s in range(4)])
    u, fin, _ = _run(f, lam=10.0, sigma_s=1.5, sigma_r=0.1)
    assert np.max(np.abs(u - oracle.smooth(fin, 10.0, 1.5, 0.1))) <= TOL_FP32


def test_joint_guide():
    target, guide = joint_pair(128, 128, 0)
    u, fin, gin = _run(target, guide, lam=30.0, sigma_s=4.0, sigma_r=0.08)
    ref = oracle.smooth(fin, 30.0, 4.0, 0.08, guide=gin)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


@pytest.mark.parametrize("n", [2, 3])
def test_rolling_guidance_iterations(n):
    f = voronoi_image(80, 96, 41)
    u, fin, _ = _run(f, lam=20.0, sigma_s=2.0, sigma_r=0.1, iterations=n)
    ref = oracle.smooth(fin, 20.0, 2.0, 0.1, iterations=n)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_rolling_with_gaussian_initial_guide():
    f = voronoi_image(72, 90, 43)
    u, fin, _ = _run(f, lam=20.0, sigma_s=2.0, sigma_r=0.05, iterations=2, sigma_guide=1.5)
    ref = oracle.smooth(fin, 20.0, 2.0, 0.05, iterations=2, sigma_guide=1.5)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_normalize_flag():
    f = voronoi_image(64, 80, 47) * 0.5 + 0.2
    u, fin, _ = _run(f, lam=20.0, sigma_s=2.0, sigma_r=0.1, normalize=True)
    ref = oracle.smooth(fin, 20.0, 2.0, 0.1, normalize=True)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_normalize_with_guide_and_iterations():
    target, guide = joint_pair(64, 64, 3)
    u, fin, gin = _run(target, guide, lam=20.0, sigma_s=2.0, sigma_r=0.2, normalize=True, iterations=2)
    ref = oracle.smooth(fin, 20.0, 2.0, 0.2, guide=gin, normalize=True, iterations=2)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_range_kernel_off():
    f = voronoi_image(50, 60, 53)
    u, fin, _ = _run(f, lam=30.0, sigma_s=2.0, sigma_r=math.inf)
    assert np.max(np.abs(u - oracle.smooth(fin, 30.0, 2.0, math.inf))) <= TOL_FP32


def test_exact_special_cases():
    f = voronoi_image(64, 64, 59).astype(np.float32)
    # lambda = 0, identity filter (r = 0) and a constant image return f bitwise (residual form)
    u0, _, _ = _run(f, lam=0.0, sigma_s=2.0, sigma_r=0.1)
    assert np.array_equal(u0.astype(np.float32), f)
    ur, _, _ = _run(f, lam=1024.0, sigma_s=2.0, sigma_r=0.1, radius=0)
    assert np.array_equal(ur.astype(np.float32), f)
    c = np.full((32, 40), 0.375, dtype=np.float32)
    uc, _, _ = _run(c, lam=500.0, sigma_s=3.0, sigma_r=0.1)
    assert np.array_equal(uc.astype(np.float32), c)


def test_mean_preserved():
    f = voronoi_image(128, 160, 61)
    u, fin, _ = _run(f, lam=1024.0, sigma_s=3.0, sigma_r=0.1)
    assert abs(u.mean() - fin.mean()) < 1e-6


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_mixed_precision_fields(precision):
    f = voronoi_image(256, 256, config_seed(0, 0))
    u, fin, _ = _run(f, lam=50.0, sigma_s=3.0, sigma_r=0.05, precision=precision)
    ref = oracle.smooth(fin, 50.0, 3.0, 0.05)
    err = np.max(np.abs(u - ref))
    psnr = _psnr(u, ref)
    print(f"{precision}: max-abs {err:.3e} psnr {psnr:.1f} dB")
    assert err <= TOL_MIXED and psnr >= 50.0


def test_pitched_buffers_and_side_stream():
    b = blfls()
    H, W, pitch = 48, 64, 80
    f = voronoi_image(H, W, 67).astype(np.float32)
    fbuf = torch.zeros((H, pitch), dtype=torch.float32, device="cuda")
    fbuf[:, :W] = torch.from_numpy(f).cuda()
    ubuf = torch.full((H, pitch), -7.0, dtype=torch.float32, device="cuda")
    plan = b.Plan(H, W, 1)
    prm = b.make_params(20.0, 2.0, 0.1)
    s = torch.cuda.Stream()
    import ctypes
    with torch.cuda.stream(s):
        st = b.lib().blfls_smooth(plan._handle, ctypes.byref(prm), ctypes.c_void_p(fbuf.data_ptr()), None,
                                  ctypes.c_void_p(ubuf.data_ptr()), pitch, ctypes.c_void_p(plan.workspace_ptr),
                                  ctypes.c_void_p(s.cuda_stream))
    assert st == 0
    s.synchronize()
    out = ubuf.cpu().numpy()
    assert np.all(out[:, W:] == -7.0)  # padding untouched
    ref = oracle.smooth(f.astype(np.float64), 20.0, 2.0, 0.1)
    assert np.max(np.abs(out[:, :W] - ref)) <= TOL_FP32


def test_abi_errors_on_device():
    import ctypes
    b = blfls()
    L = b.lib()
    plan = b.Plan(32, 32, 1)
    f = torch.zeros((32, 32), device="cuda")
    prm = b.make_params(20.0, 2.0, 0.1)
    ws = ctypes.c_void_p(plan.workspace_ptr)
    # u aliasing f
    assert L.blfls_smooth(plan._handle, ctypes.byref(prm), ctypes.c_void_p(f.data_ptr()), None,
                          ctypes.c_void_p(f.data_ptr()), 32, ws, None) == -1
    u = torch.zeros_like(f)
    bad = [b.make_params(-1.0, 2.0, 0.1), b.make_params(20.0, 0.0, 0.1), b.make_params(20.0, 2.0, 0.0),
           b.make_params(20.0, 2.0, 0.1, radius=33), b.make_params(20.0, 2.0, 0.1, iterations=0),
           b.make_params(float("nan"), 2.0, 0.1)]
    for p in bad:
        assert L.blfls_smooth(plan._handle, ctypes.byref(p), ctypes.c_void_p(f.data_ptr()), None,
                              ctypes.c_void_p(u.data_ptr()), 32, ws, None) == -1
    # misaligned workspace, short pitch
    assert L.blfls_smooth(plan._handle, ctypes.byref(prm), ctypes.c_void_p(f.data_ptr()), None,
                          ctypes.c_void_p(u.data_ptr()), 32, ctypes.c_void_p(plan.workspace_ptr + 4), None) == -1
    assert L.blfls_smooth(plan._handle, ctypes.byref(prm), ctypes.c_void_p(f.data_ptr()), None,
                          ctypes.c_void_p(u.data_ptr()), 16, ws, None) == -1
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# Full-size workload: 1024 x 1024 RGB, lambda = 20, sigma_s = 3, sigma_r = 0.1
# ---------------------------------------------------------------------------

def _stencil_residual_at(u, f, gx, gy, lam, rows, cols):
    """(u - f) + lam (D_x^T (D_x u - g_x) + D_y^T (D_y u - g_y)) at the listed pixels,
    given g_* at (i, j), (i, j-1) and (i-1, j) for each listed pixel."""
    H, W = u.shape
    i, j = rows, cols
    jm, jp = (j - 1) % W, (j + 1) % W
    im, ip = (i - 1) % H, (i + 1) % H
    dxu_here = u[i, jp] - u[i, j]
    dxu_left = u[i, j] - u[i, jm]
    dyu_here = u[ip, j] - u[i, j]
    dyu_up = u[i, j] - u[im, j]
    ex_here, ex_left = dxu_here - gx[0], dxu_left - gx[1]
    ey_here, ey_up = dyu_here - gy[0], dyu_up - gy[1]
    return (u[i, j] - f[i, j]) + lam * ((ex_left - ex_here) + (ey_up - ey_here))


def test_rgb_1024_full_size():
    lam, ss, sr = 20.0, 3.0, 0.1
    f = voronoi_rgb(1024, 1024, 1)
    u, fin, _ = _run(f, lam=lam, sigma_s=ss, sigma_r=sr)
    # channel 0 element by element against the whole oracle
    ref0 = oracle.smooth(fin[0], lam, ss, sr)
    err0 = np.max(np.abs(u[0] - ref0))
    print(f"1024x1024 channel 0: max-abs {err0:.3e}")
    assert err0 <= TOL_FP32
    # every channel: the normal equations of Eq. (7) hold at sampled pixels, with the
    # filtered fields evaluated there by the oracle, pixel by pixel
    rng = np.random.default_rng(2024)
    rows = rng.integers(0, 1024, 400)
    cols = rng.integers(0, 1024, 400)
    r = oracle.default_radius(ss)
    for c in range(3):
        px, py = oracle.grad_x(fin[c]), oracle.grad_y(fin[c])
        gx = [oracle.bilateral_filter_at(px, None, ss, sr, r, rows, cols),
              oracle.bilateral_filter_at(px, None, ss, sr, r, rows, (cols - 1) % 1024)]
        gy = [oracle.bilateral_filter_at(py, None, ss, sr, r, rows, cols),
              oracle.bilateral_filter_at(py, None, ss, sr, r, (rows - 1) % 1024, cols)]
        res = _stencil_residual_at(u[c], fin[c], gx, gy, lam, rows, cols)
        # a u error e moves the residual by at most (1 + 8 lam) |e|
        assert np.max(np.abs(res)) <= (1 + 8 * lam) * TOL_FP32


def _sampled_normal_equations(u, f, g, lam, ss, sr, n, seed):
    """Max |residual| of the normal equations of Eq. (7) at n random pixels, with the filtered
    fields there (and at the left / upper neighbours) evaluated by the oracle pixel by pixel."""
    H, W = f.shape
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, H, n)
    cols = rng.integers(0, W, n)
    r = oracle.default_radius(ss)
    px, py = oracle.grad_x(f), oracle.grad_y(f)
    qx = qy = None
    if g is not None:
        qx, qy = oracle.grad_x(g), oracle.grad_y(g)
    gx = [oracle.bilateral_filter_at(px, qx, ss, sr, r, rows, cols),
          oracle.bilateral_filter_at(px, qx, ss, sr, r, rows, (cols - 1) % W)]
    gy = [oracle.bilateral_filter_at(py, qy, ss, sr, r, rows, cols),
          oracle.bilateral_filter_at(py, qy, ss, sr, r, (rows - 1) % H, cols)]
    return float(np.max(np.abs(_stencil_residual_at(u, f, gx, gy, lam, rows, cols))))


@pytest.mark.timeout(900)
def test_uhd_rgb_full_size_every_precision():
    """The 3840x2160 RGB workload (lambda = 50, sigma_s = 8: r = 24, sigma_r = 0.05) in the
    launch bench.py times: one whole channel element by element against the oracle (its C
    loops of Eq. (1), then the Eq. (8) solve) in FP32 (<= 1e-5), BF16 and FP16 field
    storage (<= 2e-3, >= 50 dB); every channel's normal equations at sampled pixels as a
    diagnostic of where an error would sit (filter or solve)."""
    lam, ss, sr = 50.0, 8.0, 0.05
    f = voronoi_rgb(2160, 3840, 2)
    f32 = np.asarray(f, dtype=np.float32)
    outs = {}
    for prec in ("fp32", "bf16", "fp16"):
        u = blfls().smooth(_to_gpu(f32), lam=lam, sigma_s=ss, sigma_r=sr, precision=prec)
        torch.cuda.synchronize()
        outs[prec] = u.cpu().numpy().astype(np.float64)
    fin = f32.astype(np.float64)
    for c in range(3):
        res = _sampled_normal_equations(outs["fp32"][c], fin[c], None, lam, ss, sr, 100, 77 + c)
        print(f"3840x2160 channel {c}: max normal-equation residual {res:.3e}")
    ref = oracle.smooth(fin[0], lam, ss, sr, engine="c")
    for prec, tol in (("fp32", TOL_FP32), ("bf16", TOL_MIXED), ("fp16", TOL_MIXED)):
        err = float(np.max(np.abs(outs[prec][0] - ref)))
        psnr = _psnr(outs[prec][0], ref)
        print(f"3840x2160 channel 0 {prec}: max-abs {err:.3e}, PSNR {psnr:.1f} dB")
        assert err <= tol
        if prec != "fp32":
            assert psnr >= 50.0


@pytest.mark.timeout(600)
def test_joint_2048_full_size_fp16_and_fp32():
    """One pair of the guided 2048x2048 workload (lambda = 30, sigma_s = 4: r = 12,
    sigma_r = 0.08) element by element against the oracle: FP16 field storage as the
    workload runs it (<= 2e-3, >= 50 dB) and plain FP32 (<= 1e-5)."""
    lam, ss, sr = 30.0, 4.0, 0.08
    t, g = joint_pair(2048, 2048, 0)
    tin = np.asarray(t, dtype=np.float32).astype(np.float64)
    gin = np.asarray(g, dtype=np.float32).astype(np.float64)
    ref = oracle.smooth(tin, lam, ss, sr, guide=gin, engine="c")
    for prec, tol in (("fp16", TOL_MIXED), ("fp32", TOL_FP32)):
        u, _, _ = _run(t, g, lam=lam, sigma_s=ss, sigma_r=sr, precision=prec)
        err = float(np.max(np.abs(u - ref)))
        psnr = _psnr(u, ref)
        print(f"2048x2048 joint {prec}: max-abs {err:.3e}, PSNR {psnr:.1f} dB")
        assert err <= tol
        if prec == "fp16":
            assert psnr >= 50.0


def test_largest_plan_sampled():
    # the largest transform sizes a plan accepts: W/2 = H = 4096
    lam, ss, sr = 10.0, 1.0, 0.1
    f = voronoi_image(4096, 8192, 5)
    u, fin, _ = _run(f, lam=lam, sigma_s=ss, sigma_r=sr)
    res = _sampled_normal_equations(u, fin, None, lam, ss, sr, 300, 83)
    print(f"4096x8192: max normal-equation residual {res:.3e}")
    assert res <= (1 + 8 * lam) * TOL_FP32
    assert abs(float(u.mean()) - float(fin.mean())) < 1e-6


# ---------------------------------------------------------------------------
# Serving: every result equals the same request run alone
# ---------------------------------------------------------------------------

def test_server_results_equal_alone():
    import time
    b = blfls()
    rng = np.random.default_rng(5)
    shapes = [(32, 48, 1), (64, 64, 3), (40, 30, 1), (96, 80, 3), (48, 50, 1), (64, 128, 1)]
    reqs = []
    for k in range(12):
        H, W, C = shapes[k % len(shapes)]
        f = np.stack([voronoi_image(H, W, 700 + 10 * k + c) for c in range(C)])
        prm = dict(lam=float(rng.uniform(5, 100)), sigma_s=float(rng.choice([1.0, 2.0, 4.0])),
                   sigma_r=float(rng.uniform(0.03, 0.2)))
        guide = np.stack([voronoi_image(H, W, 900 + k + c) for c in range(C)]) if k % 5 == 4 else None
        reqs.append((f, guide, prm))
    server = b.Server(arena_bytes=256 << 20, max_slots=5, precision="fp32")
    tickets = []
    for f, guide, prm in reqs:
        g = None if guide is None else _to_gpu(guide)
        t, u = server.submit(_to_gpu(f), guide=g, **prm)
        tickets.append((t, u))
    outs = []
    deadline = time.time() + 60
    for t, u in tickets:
        while True:
            state, status = server.poll(t)
            if state in (b.DONE, b.FAILED):
                break
            assert time.time() < deadline, "server did not finish"
            time.sleep(0.001)
        assert state == b.DONE and status == 0
        outs.append(u)
    server.stream.synchronize()
    stats = server.stats()
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    # BLF-LS steps of these sizes replay captured graphs of persistent launches
    assert stats["graph_steps"] >= 1 and stats["graph_steps"] + stats["direct_steps"] == stats["steps"]
    server.close()
    for (f, guide, prm), u in zip(reqs, outs):
        g = None if guide is None else _to_gpu(guide)
        alone = b.smooth(_to_gpu(f), guide=g, **prm)
        torch.cuda.synchronize()
        assert torch.equal(alone, u)
        ref = oracle.smooth(f.astype(np.float32).astype(np.float64), prm["lam"], prm["sigma_s"], prm["sigma_r"],
                            guide=None if guide is None else guide.astype(np.float32).astype(np.float64))
        assert np.max(np.abs(u.cpu().numpy() - ref)) <= TOL_FP32


# ---------------------------------------------------------------------------
# Graph capture of the synchronous path
# ---------------------------------------------------------------------------

def test_smooth_captured_in_graph_replays_match_eager():
    """blfls_smooth queues only kernels (descriptor upload by kernel argument, no
    memset or host copy), so it can be captured; every replay must equal the eager
    result for the inputs present at replay time."""
    b = blfls()
    H, W, C = 96, 128, 3
    plan = b.Plan(H, W, C)
    prm = dict(lam=20.0, sigma_s=2.0, sigma_r=0.1)
    static_f = torch.zeros((C, H, W), device="cuda")
    static_u = torch.zeros_like(static_f)
    # warm up on a side stream, then capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.smooth(static_f, out=static_u, **prm)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.smooth(static_f, out=static_u, **prm)
    for k in range(4):
        img = torch.from_numpy(voronoi_rgb(H, W, 20 + k).astype(np.float32)).cuda()
        static_f.copy_(img)
        g.replay()
        torch.cuda.synchronize()
        eager = plan.smooth(img, **prm)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(static_u, eager), f"replay {k} differs from eager"


def test_server_graph_path_all_features_bitwise():
    """Steps mixing Gaussian guides, normalisation, rolling iterations, joint
    filtering and three radius classes run as captured graphs; replays with new
    work must give exactly the synchronous result of each request."""
    import time
    b = blfls()
    reqs = []
    for k in range(18):
        H, W = [(40, 48), (64, 80), (72, 90)][k % 3]
        f = voronoi_image(H, W, 1200 + k)
        prm = dict(lam=[10.0, 50.0, 200.0][k % 3], sigma_s=[1.0, 2.0, 4.0][(k // 3) % 3],
                   sigma_r=0.08, iterations=1 + k % 2, normalize=(k % 4 == 1),
                   sigma_guide=(1.0 if k % 5 == 2 else 0.0))
        guide = voronoi_image(H, W, 1300 + k) if k % 6 == 3 else None
        reqs.append((f, guide, prm))
    server = b.Server(arena_bytes=256 << 20, max_slots=4, precision="fp32")
    pending = []
    for f, guide, prm in reqs:  # several steps: the same signatures replay their graphs
        g = None if guide is None else _to_gpu(guide)
        t, u = server.submit(_to_gpu(f), guide=g, **prm)
        pending.append((t, u))
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
    assert server.stats()["steps"] >= 3
    server.close()
    for (f, guide, prm), (_, u) in zip(reqs, pending):
        g = None if guide is None else _to_gpu(guide)
        alone = b.smooth(_to_gpu(f), guide=g, **prm)
        torch.cuda.synchronize()
        assert torch.equal(alone, u), prm


def test_server_rejects_and_backpressure():
    b = blfls()
    server = b.Server(arena_bytes=48 << 20, max_slots=2, queue_capacity=2, precision="fp32")
    f = _to_gpu(voronoi_image(64, 64, 5))
    with pytest.raises(b.BlflsError) as e:
        server.submit(_to_gpu(voronoi_image(2048, 2048, 5)), lam=20.0, sigma_s=2.0, sigma_r=0.1)  # never fits
    assert e.value.status == -3
    with pytest.raises(b.BlflsError) as e:
        server.submit(f, lam=-1.0, sigma_s=2.0, sigma_r=0.1)
    assert e.value.status == -1
    with pytest.raises(b.BlflsError) as e:
        server.submit(_to_gpu(voronoi_image(63, 64, 5)), lam=20.0, sigma_s=2.0, sigma_r=0.1)
    assert e.value.status == -2
    # a full queue answers E_AGAIN and accepts again once it drains
    tickets = []
    again = 0
    for _ in range(50):
        try:
            tickets.append(server.submit(f, lam=20.0, sigma_s=2.0, sigma_r=0.1)[0])
        except b.BlflsError as err:
            assert err.status == -4
            again += 1
    assert again > 0
    import time
    for t in tickets:
        while server.poll(t)[0] not in (b.DONE, b.FAILED):
            time.sleep(0.001)
    with pytest.raises(b.BlflsError) as e:
        server.poll(tickets[0])  # retired by the poll that reported DONE
    assert e.value.status == -6
    server.close()


def test_binding_validates_out_guide_and_server_inputs():
    """Wrong shapes, dtypes, strides or devices of out, guide or a served image raise
    ValueError before anything is queued."""
    b = blfls()
    f = _to_gpu(voronoi_image(64, 80, 6))
    plan = b.Plan(64, 80, 1)
    for bad in (torch.empty(32, 80, device="cuda"), torch.empty(64, 80, device="cuda", dtype=torch.float64),
                torch.empty(80, 64, device="cuda").t(), torch.empty(64, 80)):
        with pytest.raises(ValueError):
            plan.smooth(f, 20.0, 2.0, 0.1, out=bad)
        with pytest.raises(ValueError):
            plan.smooth(f, 20.0, 2.0, 0.1, guide=bad)
    with pytest.raises(ValueError):
        plan.smooth(f, 20.0, 2.0, 0.1, out=f)
    server = b.Server(arena_bytes=64 << 20, max_slots=2)
    for bad in (f.double(), torch.empty(80, 64, device="cuda").t(), f.cpu()):
        with pytest.raises(ValueError):
            server.submit(bad, lam=20.0, sigma_s=2.0, sigma_r=0.1)
    with pytest.raises(ValueError):
        server.submit(f, guide=torch.empty(32, 80, device="cuda"), lam=20.0, sigma_s=2.0, sigma_r=0.1)
    with pytest.raises(ValueError):
        server.submit(f, out=torch.empty(64, 81, device="cuda"), lam=20.0, sigma_s=2.0, sigma_r=0.1)
    server.close()
    plan.close()


def test_server_orders_inputs_still_being_written_on_the_callers_stream():
    """An image produced by GPU work still queued on the caller's stream when it is
    submitted: the server's stream waits for that work, so the result equals the same
    request run alone."""
    import time
    b = blfls()
    img = voronoi_image(512, 512, 8)
    server = b.Server(arena_bytes=256 << 20, max_slots=2)
    big = torch.eye(4096, device="cuda")
    for _ in range(20):                 # milliseconds of queued work (the products stay the identity)
        big = big @ big
    f = _to_gpu(img) + big[0, :1] * 0.0   # written only after the products
    t, u = server.submit(f, lam=20.0, sigma_s=2.0, sigma_r=0.1)
    deadline = time.time() + 60
    while server.poll(t)[0] not in (b.DONE, b.FAILED):
        assert time.time() < deadline
        time.sleep(0.001)
    server.stream.synchronize()
    alone = b.smooth(_to_gpu(img), lam=20.0, sigma_s=2.0, sigma_r=0.1)
    torch.cuda.synchronize()
    assert torch.equal(alone, u)
    server.close()


def _psnr_peak(a, b, peak):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(peak * peak / mse)


@pytest.mark.parametrize("k,filt", [(65535.0, "blf"), (65536.0, "blf"), (65536.0, "nc"), (65536.0, "grid"),
                                    (65536.0, "amf"), (2.0 ** 24, "blf")])
def test_fp16_fields_follow_the_data_range(k, filt):
    """FP16 field storage of images with 16-bit sample values and beyond: the residual
    fields reach the gradients' span, above the FP16 maximum 65504, so each field is
    stored times the power of two that brings its span to 2^15 and the solve multiplies
    it back.  The result is finite and matches the oracle within k times the mixed
    bar (2e-3 k, 50 dB against the peak k).  The filters' windows and bins see the
    image and sigma_r scaled alike (k a power of two: the same decisions)."""
    from synth import quantized
    f = quantized(voronoi_image(72, 96, 61)) * k
    prm = dict(lam=30.0, sigma_s=3.0, sigma_r=0.0713 * k)
    kw = {} if filt == "blf" else {"filter": filt}
    u, fin, _ = _run(f, precision="fp16", **prm, **kw)
    for q in (oracle.grad_x(fin), oracle.grad_y(fin)):   # decisions far from their thresholds
        if filt == "nc":
            assert oracle.nc_decision_margin(q, prm["sigma_s"], prm["sigma_r"]) >= 1e-3
        if filt == "grid":
            assert oracle.grid_bin_margin(q, prm["sigma_r"]) >= 1e-4
    ref = oracle.smooth(fin, **prm, **kw)
    assert np.all(np.isfinite(u))
    err = float(np.max(np.abs(u - ref)))
    psnr = _psnr_peak(u, ref, k)
    print(f"FP16 fields, scale {k:g}, {filt}: max-abs {err:.3e} ({err / k:.2e} of the peak), {psnr:.1f} dB")
    assert err <= TOL_MIXED * k and psnr >= 50.0


def test_fp16_fields_joint_and_served_at_16_bit_scale():
    """A guided request with 16-bit values through the server equals the same request
    run alone, bit for bit, and matches the oracle within the scaled mixed bar."""
    import time
    b = blfls()
    k = 65535.0
    t, g = joint_pair(96, 128, 9)
    t, g = t * k, g * k
    prm = dict(lam=30.0, sigma_s=3.0, sigma_r=0.08 * k)
    server = b.Server(arena_bytes=128 << 20, max_slots=2, precision="fp16")
    tk, u = server.submit(_to_gpu(t), guide=_to_gpu(g), **prm)
    deadline = time.time() + 60
    while server.poll(tk)[0] not in (b.DONE, b.FAILED):
        assert time.time() < deadline
        time.sleep(0.001)
    server.stream.synchronize()
    alone = b.smooth(_to_gpu(t), guide=_to_gpu(g), precision="fp16", **prm)
    torch.cuda.synchronize()
    assert torch.equal(alone, u)
    server.close()
    ua = alone.cpu().numpy().astype(np.float64)
    ref = oracle.smooth(np.asarray(t, np.float32).astype(np.float64), guide=np.asarray(g, np.float32).astype(np.float64),
                        **prm)
    assert np.all(np.isfinite(ua))
    assert float(np.max(np.abs(ua - ref))) <= TOL_MIXED * k and _psnr_peak(ua, ref, k) >= 50.0
