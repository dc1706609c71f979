"""GPU parity of NC-LS (Section III-D: the domain transform's normalized
convolution in place of the BLF) against the FP64 oracle, through the C ABI.

Window membership is a discontinuous function of the guide: the oracle decides
it in FP64, the kernel in FP32.  The two pick the same windows whenever the
kernel's rounding of a transformed distance stays below the distance between
that distance and the box radius.  The kernel sums at most 33 increments (box
radii up to 32), each and each partial sum rounded once, so its distances are
within 33 * 2^-23 * 33 < 1.3e-4 of the exact ones.  The inputs here are images
with 6-bit samples (multiples of 1/64, ``synth.quantized``), whose increments
fall on a coarse grid; every test asserts that the oracle's smallest decision
margin (``oracle.nc_decision_margin``) is at least MARGIN = 1e-3, so both
sides take every decision alike and then differ only by FP32 averaging and
transforms: max-abs 1e-5 for FP32 fields, 2e-3 and PSNR >= 50 dB for 16-bit
fields.

Rolling guidance takes iteration k's range source from the previous output,
which is not on such a grid and differs in its last bits between the two
sides; a decision close to its threshold can then go either way, moving one
sample in or out of a window, and the moves of one iteration change the next
iteration's guide.  The end-to-end rolling test therefore states a
distributional bar (most pixels at the FP32 tolerance, the rest within the
effect of such moves), and a separate test checks the rolling step's
definition exactly: iteration 2 equals, bit for bit, the GPU's own joint
filtering guided by its first iteration.
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_image, voronoi_rgb, joint_pair, quantized

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_MIXED = 2e-3
MARGIN = 1e-3


def _assert_margin(src, ss, sr, normalize=False, n_iter=3):
    """The oracle's decisions on the range source `src` (an image, one channel or a stack)
    all lie at least MARGIN from their thresholds."""
    src = np.asarray(src, dtype=np.float32).astype(np.float64)
    for ch in (src if src.ndim == 3 else [src]):
        for q in (oracle.grad_x(ch), oracle.grad_y(ch)):
            inv = None
            if normalize and math.isfinite(sr) and q.max() > q.min():
                inv = 1.0 / (q.max() - q.min())
            m = oracle.nc_decision_margin(q, ss, sr, n_iter, inv)
            assert m >= MARGIN, f"input too close to a window decision: margin {m:.2e}"


def blfls():
    import paper_1812_07122_amd as b
    return b


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _nc(f64, guide64=None, **kw):
    f32 = np.asarray(f64, dtype=np.float32)
    g = None if guide64 is None else _gpu(guide64)
    u = blfls().smooth(_gpu(f32), guide=g, filter="nc", **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), f32.astype(np.float64)


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


@pytest.mark.parametrize("H,W,ss,sr,lam", [
    (256, 256, 4.0, 0.05, 20.0),
    (96, 100, 2.0, 0.1, 50.0),      # ragged tiles
    (40, 300, 3.0, 0.05, 20.0),     # two 256-pixel row segments (the second of 44), ten 32-column tiles
    (36, 540, 2.0, 0.08, 30.0),     # three row segments; two 32-row tiles, the second of 4 rows
    (72, 90, 8.0, 0.02, 20.0),      # first box radius 12.1: halos of 12 rows around 32-row tiles
    (8, 12, 3.0, 0.05, 10.0),       # image smaller than one segment and one tile
    (2, 4, 1.0, 0.1, 5.0),
    (160, 30, 1.5, 0.08, 100.0),
    (80, 100, 21.0, 0.3, 20.0),     # first box radius 31.75: the largest halo
])
def test_nc_ls_parity(H, W, ss, sr, lam):
    f = quantized(voronoi_image(H, W, 500 + H + W))
    _assert_margin(f, ss, sr)
    u, fin = _nc(f, lam=lam, sigma_s=ss, sigma_r=sr)
    ref = oracle.smooth(fin, lam, ss, sr, filter="nc")
    err = float(np.max(np.abs(u - ref)))
    print(f"NC-LS {H}x{W} ss={ss} sr={sr}: max-abs {err:.3e}")
    assert err <= TOL_FP32


@pytest.mark.parametrize("rounds", [1, 2, 5])
def test_nc_rounds(rounds):
    f = quantized(voronoi_image(64, 80, 77 + rounds))
    _assert_margin(f, 3.0, 0.05, n_iter=rounds)
    u, fin = _nc(f, lam=20.0, sigma_s=3.0, sigma_r=0.05, filter_iterations=rounds)
    ref = oracle.smooth(fin, 20.0, 3.0, 0.05, filter="nc", nc_iterations=rounds)
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_nc_rgb_and_joint():
    f = quantized(voronoi_rgb(64, 96, 3))
    _assert_margin(f, 4.0, 0.05)
    u, fin = _nc(f, lam=30.0, sigma_s=4.0, sigma_r=0.05)
    ref = oracle.smooth(fin, 30.0, 4.0, 0.05, filter="nc")
    assert np.max(np.abs(u - ref)) <= TOL_FP32
    t, g = joint_pair(96, 128, 3)
    g = quantized(g)
    _assert_margin(g, 4.0, 0.08)
    u, tin = _nc(t, g, lam=30.0, sigma_s=4.0, sigma_r=0.08)
    ref = oracle.smooth(tin, 30.0, 4.0, 0.08, guide=np.asarray(g, np.float32).astype(np.float64), filter="nc")
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_nc_normalize_and_range_off():
    f = quantized(voronoi_image(72, 90, 91))
    _assert_margin(f, 3.0, 0.3, normalize=True)
    u, fin = _nc(f, lam=20.0, sigma_s=3.0, sigma_r=0.3, normalize=True)
    ref = oracle.smooth(fin, 20.0, 3.0, 0.3, normalize=True, filter="nc")
    assert np.max(np.abs(u - ref)) <= TOL_FP32
    u, fin = _nc(f, lam=20.0, sigma_s=3.0, sigma_r=math.inf)
    ref = oracle.smooth(fin, 20.0, 3.0, math.inf, filter="nc")
    assert np.max(np.abs(u - ref)) <= TOL_FP32


def test_nc_rolling_end_to_end():
    """Rolling NC-LS with the texture-removal settings (three iterations from a
    Gaussian-smoothed guide) against oracle.smooth(iterations=3), nothing of the GPU's
    fed to the oracle.  Iterations 2 and 3 decide windows from the previous output, so
    a decision within rounding of its threshold may go either way and moves a sample in
    or out of a window (a change of up to a gradient's size over the window's count in
    one filtered value, spread by the solve); the first iteration's moves change the
    next guide, so such differences compound.  Measured on the box: 94.7% of the pixels
    within 1e-5, max-abs 5.0e-3, 77.8 dB.  The bar: the FP32 tolerance at 90% of the
    pixels, 2e-2 everywhere and 70 dB (a wrong kernel lands near 30-40 dB); the exact
    checks are iteration 1 against the oracle and the step's definition below."""
    f = quantized(voronoi_image(128, 160, 93))
    prm = dict(lam=20.0, sigma_s=8.0, sigma_r=0.02, iterations=3, sigma_guide=2.5)
    u, fin = _nc(f, **prm)
    ref = oracle.smooth(fin, filter="nc", **prm)
    d = np.abs(u - ref)
    frac = float(np.mean(d <= TOL_FP32))
    print(f"rolling NC-LS n=3: {frac:.4f} of pixels within 1e-5, max-abs {d.max():.3e}, "
          f"PSNR {_psnr(u, ref):.1f} dB")
    assert frac >= 0.90 and d.max() <= 2e-2 and _psnr(u, ref) >= 70.0


def test_nc_rolling_step_is_the_gpu_joint_step_guided_by_the_previous_output():
    """Iteration 2 of rolling guidance is, bit for bit, the GPU's own joint filtering
    guided by its first iteration (the definition of the rolling step); iteration 1
    matches the oracle at the FP32 tolerance."""
    f = quantized(voronoi_image(96, 128, 93))
    _assert_margin(f, 4.0, 0.02)
    u1, fin = _nc(f, lam=20.0, sigma_s=4.0, sigma_r=0.02, iterations=1)
    u2, _ = _nc(f, lam=20.0, sigma_s=4.0, sigma_r=0.02, iterations=2)
    assert np.max(np.abs(u1 - oracle.smooth(fin, 20.0, 4.0, 0.02, filter="nc"))) <= TOL_FP32
    u2j, _ = _nc(f, u1, lam=20.0, sigma_s=4.0, sigma_r=0.02)
    assert np.max(np.abs(u2 - u2j)) == 0.0


def test_nc_exact_special_cases():
    f = voronoi_image(48, 64, 95)
    f32 = np.asarray(f, dtype=np.float32)
    u, _ = _nc(f, lam=0.0, sigma_s=3.0, sigma_r=0.05)
    assert np.array_equal(u.astype(np.float32), f32)
    c = np.full((32, 40), 0.4, dtype=np.float32)
    u, _ = _nc(c, lam=50.0, sigma_s=3.0, sigma_r=0.05)
    assert np.array_equal(u.astype(np.float32), c)


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_nc_mixed_precision_fields(precision):
    f = quantized(voronoi_rgb(128, 160, 4))
    _assert_margin(f, 6.0, 0.05)
    u, fin = _nc(f, lam=30.0, sigma_s=6.0, sigma_r=0.05, precision=precision)
    ref = oracle.smooth(fin, 30.0, 6.0, 0.05, filter="nc")
    err = float(np.max(np.abs(u - ref)))
    psnr = _psnr(u, ref)
    print(f"NC-LS {precision}: max-abs {err:.3e}, PSNR {psnr:.1f} dB")
    assert err <= TOL_MIXED and psnr >= 50.0


def test_nc_rgb_1024_channel_full_size():
    f = quantized(voronoi_rgb(1024, 1024, 1))
    _assert_margin(f[0], 8.0, 0.05)
    u, fin = _nc(f, lam=20.0, sigma_s=8.0, sigma_r=0.05)
    ref0 = oracle.smooth(fin[0], 20.0, 8.0, 0.05, filter="nc")
    err = float(np.max(np.abs(u[0] - ref0)))
    print(f"NC-LS 1024x1024 channel 0: max-abs {err:.3e}")
    assert err <= TOL_FP32


def test_nc_abi_errors():
    b = blfls()
    f = _gpu(voronoi_image(16, 16, 1))
    with pytest.raises(b.BlflsError) as e:
        b.smooth(f, lam=1.0, sigma_s=22.0, sigma_r=0.1, filter="nc")   # first box beyond 32 pixels
    assert e.value.status == -1
    with pytest.raises(b.BlflsError) as e:
        b.smooth(f, lam=1.0, sigma_s=2.0, sigma_r=0.1, filter="nc", filter_iterations=9)
    assert e.value.status == -1
    with pytest.raises(b.BlflsError) as e:
        b.smooth(f, lam=1.0, sigma_s=2.0, sigma_r=0.1, filter_iterations=3)   # BLF takes no rounds
    assert e.value.status == -1
