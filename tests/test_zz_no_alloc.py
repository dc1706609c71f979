"""blfls_smooth_noalloc (the entry point for callers that cannot allocate device
memory) against blfls_smooth with a caller workspace, through the C ABI.

Two calls in a row share the library's static per-GPU scratch: a 1024x1024 RGB
image, then a smaller joint-guided one; each must equal blfls_smooth on the same
inputs bit for bit (the same kernels on the same data; only the workspace's
address differs).  A plan whose workspace exceeds the scratch is refused on the
host before anything is queued.
"""
import numpy as np
import pytest

from synth import voronoi_image, voronoi_rgb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_noalloc_equals_smooth_twice_with_a_smaller_second_input():
    import paper_1812_07122_amd as b
    cases = [
        ((1024, 1024, 3), dict(lam=20.0, sigma_s=3.0, sigma_r=0.1), False),
        ((96, 128, 1), dict(lam=30.0, sigma_s=2.0, sigma_r=0.08, iterations=2), True),
    ]
    for (H, W, C), prm, joint in cases:
        f = _gpu(voronoi_rgb(H, W, 11, C) if C > 1 else voronoi_image(H, W, 11))
        g = _gpu(voronoi_rgb(H, W, 12, C) if C > 1 else voronoi_image(H, W, 12)) if joint else None
        plan = b.Plan(H, W, C)
        ref = plan.smooth(f, guide=g, **prm)
        out = torch.full_like(f, float("nan"))
        plan.smooth_noalloc(f, guide=g, out=out, **prm)
        torch.cuda.synchronize()
        print(f"{H}x{W}x{C}: noalloc vs smooth max-abs {float((out - ref).abs().max()):.3e}")
        assert torch.equal(out, ref), (H, W, C)
        plan.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    import paper_1812_07122_amd as b
    plan = b.Plan(2048, 2048, 3)
    f = torch.zeros((3, 2048, 2048), device="cuda")
    out = torch.empty_like(f)
    with pytest.raises(b.BlflsError) as e:
        plan.smooth_noalloc(f, lam=20.0, sigma_s=3.0, sigma_r=0.1, out=out)
    assert e.value.status == -3 and "scratch" in str(e.value)
    plan.close()
