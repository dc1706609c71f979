"""The server runs every filter: steps mixing BLF-LS, NC-LS, grid BLF-LS and
AMF-LS requests (uneven sizes, rolling iterations, normalisation, joint
filtering, detail gain) give each request exactly its synchronous result.
Steps holding a filter other than the BLF launch directly (the filter stage
per request, extrema and the Fourier solve batched across requests)."""
import time

import numpy as np
import pytest

from synth import voronoi_image, voronoi_rgb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def blfls():
    import paper_1812_07122_amd as b
    return b


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_server_runs_every_filter_bitwise():
    b = blfls()
    filters = ["blf", "nc", "grid", "amf"]
    reqs = []
    for k in range(16):
        H, W = [(40, 48), (64, 80), (72, 90), (32, 40)][k % 4]
        f = voronoi_rgb(H, W, 1500 + k) if k % 3 == 0 else voronoi_image(H, W, 1500 + k)
        prm = dict(lam=[10.0, 30.0][k % 2], sigma_s=[2.0, 3.0, 4.0][k % 3], sigma_r=0.06,
                   filter=filters[k % 4], iterations=1 + (k // 4) % 2, normalize=(k % 5 == 1),
                   detail_gain=(5.0 if k % 7 == 3 else 0.0))
        guide = voronoi_image(H, W, 1600 + k) if (k % 6 == 5 and f.ndim == 2) else None
        reqs.append((f, guide, prm))
    server = b.Server(arena_bytes=512 << 20, max_slots=6, precision="fp32")
    pending = []
    for f, guide, prm in reqs:
        g = None if guide is None else _gpu(guide)
        pending.append(server.submit(_gpu(f), guide=g, **prm))
    deadline = time.time() + 60
    for t, _ in pending:
        while True:
            state, status = server.poll(t)
            if state in (b.DONE, b.FAILED):
                break
            assert time.time() < deadline, "server did not finish"
            time.sleep(0.001)
        assert state == b.DONE and status == 0
    server.stream.synchronize()
    stats = server.stats()
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    server.close()
    for (f, guide, prm), (_, u) in zip(reqs, pending):
        g = None if guide is None else _gpu(guide)
        alone = b.smooth(_gpu(f), guide=g, **prm)
        torch.cuda.synchronize()
        assert torch.equal(alone, u), prm


def test_server_amf_workspace_admission():
    # an AMF request needs more arena than the plan's workspace: an arena that holds the
    # plan's workspace but not the manifold arrays refuses it at submit
    b = blfls()
    f = _gpu(voronoi_image(256, 256, 3))
    plan = b.Plan(256, 256, 1)
    need = plan.workspace_for(b.make_params(20.0, 3.0, 0.05, filter="amf", filter_iterations=4))
    small = b.Server(arena_bytes=(plan.workspace_bytes + need) // 2 + (16 << 20), max_slots=2, precision="fp32")
    try:
        with pytest.raises(b.BlflsError) as e:
            small.submit(f, 20.0, 3.0, 0.05, filter="amf", filter_iterations=4)
        assert e.value.status == -3
    finally:
        small.close()


@pytest.mark.parametrize("filt", ["nc", "grid", "amf"])
def test_four_channel_plans_for_every_filter(filt):
    # C = 4 (the largest plan): every filter's descriptors, item offsets and (AMF) workspace
    # arrays cover the fourth channel, each channel matching the oracle on its own
    import oracle
    b = blfls()
    f = np.stack([voronoi_image(48, 64, 1700 + c) for c in range(4)])
    f32 = f.astype(np.float32)
    u = b.smooth(_gpu(f32), lam=20.0, sigma_s=3.0, sigma_r=0.06, filter=filt)
    torch.cuda.synchronize()
    got = u.cpu().numpy().astype(np.float64)
    for c in range(4):
        ref = oracle.smooth(f32[c].astype(np.float64), 20.0, 3.0, 0.06, filter=filt)
        assert np.max(np.abs(got[c] - ref)) <= 1e-5, (filt, c)
