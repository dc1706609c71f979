"""GPU parity of AMF-LS (Section III-D: the adaptive-manifold filter in place of
the BLF) against the FP64 oracle, through the C ABI.

The filter is a chain of recursive passes and smooth weights; the GPU runs it
in FP32 (manifolds, weights and sums) and differs from the FP64 oracle only by
rounding: max-abs 1e-5 for FP32 fields, 2e-3 and PSNR >= 50 dB for 16-bit
fields.  The sizes span several row chunks, column workgroups and 16-row scan
segments with ragged tails; trees of height 1 to 4 are covered.  Rolling
guidance is compared end to end: the range source of iteration 2 is each
side's own first output, and the filter is smooth in it.
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


def _amf(f64, guide64=None, **kw):
    f32 = np.asarray(f64, dtype=np.float32)
    g = None if guide64 is None else _gpu(guide64)
    u = blfls().smooth(_gpu(f32), guide=g, filter="amf", **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), f32.astype(np.float64)


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


@pytest.mark.parametrize("H,W,ss,sr,lam", [
    (96, 128, 4.0, 0.05, 20.0),
    (72, 90, 8.0, 0.05, 20.0),      # ragged: 5 scan segments (4 x 16, 8), W below one column workgroup
    (270, 300, 3.0, 0.08, 30.0),    # 17 segments (the last 14 rows), 2 column workgroups, 2 values per row chunk
    (8, 12, 3.0, 0.05, 10.0),       # image smaller than one segment
    (2, 4, 1.0, 0.1, 5.0),
    (160, 30, 1.5, 0.08, 100.0),
    (80, 100, 16.0, 0.2, 20.0),     # default tree height 3: 7 manifolds
])
def test_amf_ls_parity(H, W, ss, sr, lam):
    f = voronoi_image(H, W, 900 + H + W)
    u, fin = _amf(f, lam=lam, sigma_s=ss, sigma_r=sr)
    ref = oracle.smooth(fin, lam, ss, sr, filter="amf")
    err = float(np.max(np.abs(u - ref)))
    print(f"AMF-LS {H}x{W} ss={ss} sr={sr}: max-abs {err:.3e}")
    assert err <= TOL_FP32


@pytest.mark.parametrize("height", [1, 3, 4])
def test_amf_tree_heights(height):
    f = voronoi_image(64, 80, 60 + height)
    u, fin = _amf(f, lam=20.0, sigma_s=3.0, sigma_r=0.05, filter_iterations=height)
    ref = oracle.smooth(fin, 20.0, 3.0, 0.05, filter="amf", amf_height=height)
    err = float(np.max(np.abs(u - ref)))
    print(f"AMF-LS height {height}: max-abs {err:.3e}")
    assert err <= TOL_FP32


def test_amf_rgb_and_joint():
    f = voronoi_rgb(64, 96, 7)
    u, fin = _amf(f, lam=30.0, sigma_s=4.0, sigma_r=0.05)
    assert np.max(np.abs(u - oracle.smooth(fin, 30.0, 4.0, 0.05, filter="amf"))) <= TOL_FP32
    t, g = joint_pair(96, 128, 7)
    u, tin = _amf(t, g, lam=30.0, sigma_s=4.0, sigma_r=0.08)
    gin = np.asarray(g, np.float32).astype(np.float64)
    assert np.max(np.abs(u - oracle.smooth(tin, 30.0, 4.0, 0.08, guide=gin, filter="amf"))) <= TOL_FP32


def test_amf_normalize_and_range_off():
    f = voronoi_image(72, 90, 97)
    u, fin = _amf(f, lam=20.0, sigma_s=3.0, sigma_r=0.3, normalize=True)
    assert np.max(np.abs(u - oracle.smooth(fin, 20.0, 3.0, 0.3, normalize=True, filter="amf"))) <= TOL_FP32
    u, fin = _amf(f, lam=20.0, sigma_s=3.0, sigma_r=math.inf)
    assert np.max(np.abs(u - oracle.smooth(fin, 20.0, 3.0, math.inf, filter="amf"))) <= TOL_FP32


def test_amf_rolling_end_to_end():
    """Two iterations of rolling guidance against oracle.smooth(iterations=2), nothing of
    the GPU's fed to the oracle; and iteration 2 equals, bit for bit, the GPU's own joint
    step guided by its first iteration."""
    f = voronoi_image(96, 128, 98)
    prm = dict(lam=20.0, sigma_s=4.0, sigma_r=0.02)
    u1, fin = _amf(f, iterations=1, **prm)
    u2, _ = _amf(f, iterations=2, **prm)
    assert np.max(np.abs(u1 - oracle.smooth(fin, filter="amf", **prm))) <= TOL_FP32
    err = float(np.max(np.abs(u2 - oracle.smooth(fin, filter="amf", iterations=2, **prm))))
    print(f"rolling AMF-LS n=2: max-abs {err:.3e}")
    assert err <= TOL_FP32
    u2j, _ = _amf(f, u1, **prm)
    assert np.max(np.abs(u2 - u2j)) == 0.0


def test_amf_exact_special_cases():
    f = voronoi_image(48, 64, 99)
    f32 = np.asarray(f, dtype=np.float32)
    u, _ = _amf(f, lam=0.0, sigma_s=4.0, sigma_r=0.05)
    assert np.array_equal(u.astype(np.float32), f32)
    c = np.full((32, 40), 0.4, dtype=np.float32)
    u, _ = _amf(c, lam=50.0, sigma_s=4.0, sigma_r=0.05)
    assert np.array_equal(u.astype(np.float32), c)


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_amf_mixed_precision_fields(precision):
    f = voronoi_rgb(128, 160, 8)
    u, fin = _amf(f, lam=30.0, sigma_s=6.0, sigma_r=0.05, precision=precision)
    ref = oracle.smooth(fin, 30.0, 6.0, 0.05, filter="amf")
    err = float(np.max(np.abs(u - ref)))
    psnr = _psnr(u, ref)
    print(f"AMF-LS {precision}: max-abs {err:.3e}, PSNR {psnr:.1f} dB")
    assert err <= TOL_MIXED and psnr >= 50.0


def test_amf_rgb_1024_channel_full_size():
    f = voronoi_rgb(1024, 1024, 1)
    u, fin = _amf(f, lam=20.0, sigma_s=12.0, sigma_r=0.02)
    ref0 = oracle.smooth(fin[0], 20.0, 12.0, 0.02, filter="amf")
    err = float(np.max(np.abs(u[0] - ref0)))
    print(f"AMF-LS 1024x1024 channel 0: max-abs {err:.3e}")
    assert err <= TOL_FP32


def test_amf_workspace_and_abi_errors():
    b = blfls()
    plan = b.Plan(16, 16, 1)
    base = plan.workspace_bytes
    need2 = plan.workspace_for(b.make_params(1.0, 2.0, 0.1, filter="amf", filter_iterations=2))
    need4 = plan.workspace_for(b.make_params(1.0, 2.0, 0.1, filter="amf", filter_iterations=4))
    # (6 + 2h) planes per field of 16 x 16 floats and the scan arrays, after the plan's own
    assert need2 >= base + 2 * 10 * 256 * 4 and need4 - need2 == 2 * 4 * 256 * 4
    assert plan.workspace_for(b.make_params(1.0, 2.0, 0.1, filter="nc")) == base
    f = _gpu(voronoi_image(16, 16, 1))
    with pytest.raises(b.BlflsError) as e:
        b.smooth(f, lam=1.0, sigma_s=2.0, sigma_r=0.1, filter="amf", filter_iterations=7)
    assert e.value.status == -1
