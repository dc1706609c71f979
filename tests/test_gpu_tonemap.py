"""GPU parity of the log-domain tone mapping (the experiments section's HDR
application of BLF-LS) against the FP64 oracle, through the C ABI.

The output is the input's colour ratios c / I times 10^(compressed base +
detail).  The ratios reach 61 where one channel dominates (I weights blue by
1/61), so outputs are not confined to [0, 1] like u, and the FP32 bar is taken
relative to the output: |out - ref| <= 1e-5 max(1, |ref|) per element.  FP32
logarithms, exponentials and the division keep the relative error near 1e-6.
"""
import math

import numpy as np
import pytest

import oracle
from synth import voronoi_rgb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def blfls():
    import paper_1812_07122_amd as b
    return b


def _hdr(H, W, seed):
    return 10.0 ** (4.0 * voronoi_rgb(H, W, seed) - 2.0)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("H,W,filt,kw", [
    (96, 128, "blf", dict(lam=20.0, sigma_s=4.0, sigma_r=0.03)),
    (72, 90, "blf", dict(lam=50.0, sigma_s=8.0, sigma_r=0.05)),
    (64, 80, "nc", dict(lam=20.0, sigma_s=6.0, sigma_r=0.05)),
    (64, 80, "amf", dict(lam=20.0, sigma_s=8.0, sigma_r=0.03)),
])
def test_tonemap_matches_oracle(H, W, filt, kw):
    rgb = np.asarray(_hdr(H, W, 20 + H), dtype=np.float32)
    out = blfls().tonemap(_gpu(rgb), contrast=5.0, normalize=True, filter=filt, **kw)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.tonemap(rgb.astype(np.float64), kw["lam"], kw["sigma_s"], kw["sigma_r"], contrast=5.0,
                         normalize=True, filter=filt)
    err = float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))))
    print(f"tonemap {H}x{W} {filt}: max relative error {err:.3e}, output max {ref.max():.3f}")
    assert err <= 1e-5


def test_tonemap_full_hd():
    rgb = np.asarray(_hdr(1080, 1920, 3), dtype=np.float32)
    out = blfls().tonemap(_gpu(rgb), lam=20.0, sigma_s=8.0, sigma_r=0.03, contrast=5.0)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.tonemap(rgb.astype(np.float64), 20.0, 8.0, 0.03, contrast=5.0, normalize=True)
    err = float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))))
    print(f"tonemap 1920x1080: max relative error {err:.3e}, output max {ref.max():.3f}")
    assert err <= 1e-5


def test_tonemap_validation():
    b = blfls()
    rgb = _gpu(_hdr(16, 16, 1))
    with pytest.raises(b.BlflsError) as e:
        b.tonemap(rgb, contrast=1.0)
    assert e.value.status == -1
    plan = b.Plan(16, 16, 3)
    prm = b.make_params(20.0, 2.0, 0.1)
    out = torch.empty_like(rgb)
    st = b.lib().blfls_tonemap(plan._handle, prm, rgb.data_ptr(), out.data_ptr(), 16, 5.0, plan.workspace_ptr, None)
    assert st == -1 and b"C = 1" in b.lib().blfls_last_error()
