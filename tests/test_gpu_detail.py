"""GPU parity of the detail-enhanced output u + m (f - u) (the experiments
section's detail enhancement) against the FP64 oracle, through the C ABI.

The library folds the gain into the spectral divide of the last iteration
(u = f + delta, so u + m (f - u) = f + (1 - m) delta); rounding errors of delta
grow by |1 - m|, which stays well inside the FP32 bar at m = 5.  The served path
must give exactly the synchronous result.
"""
import time

import numpy as np
import pytest

import oracle
from synth import voronoi_image, voronoi_rgb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_MIXED = 2e-3


def blfls():
    import paper_1812_07122_amd as b
    return b


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _run(f64, **kw):
    f32 = np.asarray(f64, dtype=np.float32)
    u = blfls().smooth(_gpu(f32), **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), f32.astype(np.float64)


@pytest.mark.parametrize("filt,extra", [("blf", {}), ("nc", {}), ("grid", {}), ("amf", {})])
def test_detail_gain_matches_oracle(filt, extra):
    f = voronoi_rgb(64, 96, 11)
    e, fin = _run(f, lam=20.0, sigma_s=3.0, sigma_r=0.08, filter=filt, detail_gain=5.0)
    ref = oracle.smooth(fin, 20.0, 3.0, 0.08, filter=filt, detail_gain=5.0)
    err = float(np.max(np.abs(e - ref)))
    print(f"{filt} detail x5: max-abs {err:.3e}")
    assert err <= TOL_FP32


def test_detail_gain_rolling_boosts_the_last_iteration():
    f = voronoi_image(72, 90, 12)
    u, fin = _run(f, lam=20.0, sigma_s=3.0, sigma_r=0.05, iterations=3)
    e, _ = _run(f, lam=20.0, sigma_s=3.0, sigma_r=0.05, iterations=3, detail_gain=5.0)
    # the same three iterations; only the last solve's delta is scaled by 1 - m
    assert np.max(np.abs(e - (u + 5.0 * (fin - u)))) <= 4e-6
    e1, _ = _run(f, lam=20.0, sigma_s=3.0, sigma_r=0.05, iterations=3, detail_gain=1.0)
    assert np.array_equal(e1.astype(np.float32), fin.astype(np.float32))   # m = 1: delta scaled by 0


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_detail_gain_mixed_fields(precision):
    f = voronoi_rgb(96, 128, 13)
    e, fin = _run(f, lam=30.0, sigma_s=4.0, sigma_r=0.05, precision=precision, detail_gain=5.0)
    ref = oracle.smooth(fin, 30.0, 4.0, 0.05, detail_gain=5.0)
    err = float(np.max(np.abs(e - ref)))
    print(f"detail x5 {precision}: max-abs {err:.3e}")
    # 16-bit residual fields, errors of delta scaled by |1 - m| = 4
    assert err <= 4 * TOL_MIXED


def test_detail_gain_served_equals_direct():
    b = blfls()
    reqs = []
    for k in range(6):
        H, W = [(40, 48), (64, 80)][k % 2]
        f = voronoi_image(H, W, 1400 + k)
        prm = dict(lam=20.0, sigma_s=2.0, sigma_r=0.08, iterations=1 + k % 2,
                   detail_gain=[0.0, 5.0, -1.5][k % 3])
        reqs.append((f, prm))
    server = b.Server(arena_bytes=128 << 20, max_slots=3, precision="fp32")
    pending = [server.submit(_gpu(f), **prm) for f, prm in reqs]
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
    for (f, prm), (_, u) in zip(reqs, pending):
        alone = b.smooth(_gpu(f), **prm)
        torch.cuda.synchronize()
        assert torch.equal(alone, u), prm


def test_detail_gain_must_be_finite():
    b = blfls()
    f = _gpu(voronoi_image(16, 16, 1))
    with pytest.raises(b.BlflsError) as e:
        b.smooth(f, lam=1.0, sigma_s=2.0, sigma_r=0.1, detail_gain=float("nan"))
    assert e.value.status == -1
