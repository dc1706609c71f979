"""The benchmark's contract on the CPU: it refuses more than one GPU, and the
algorithmic work counts behind its roofline objects are the ones its header and
docstrings state (taps of Eq. (1), bytes of the three passes of the Eq. (8)
solve, the AMF tree height of the library)."""
import hashlib
import math
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import bench_workloads  # noqa: E402


def _run(args, env=None):
    return subprocess.run([sys.executable, "bench.py", *args], cwd=ROOT, capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_a_distributed_launch_is_refused():
    r = _run(["--steps", "1"], env={**os.environ, "WORLD_SIZE": "2"})
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_fft_pass_bytes():
    # rows_fwd: two residual fields in, the half spectrum out (transposed);
    # cols: the half spectrum in and out; rows_inv: the spectrum and f in, u out
    H, W, C = 2160, 3840, 3
    spec = C * (W // 2 + 1) * H * 8
    for fb in (4, 2):
        rf, cl, ri = bench.fft_bytes(H, W, C, fb)
        assert rf == 2 * C * H * W * fb + spec
        assert cl == 2 * spec
        assert ri == spec + 2 * C * H * W * 4


def test_filter_roofline_against_the_published_fp32_peak():
    # one tap = one weight of Eq. (1) for one output of one field: 6 flops (difference,
    # exponent FMA, weighted-value FMA, weight sum) against 157.3 TFLOP/s
    assert bench.FP32_PEAK_TFLOPS == 157.3 and bench.BLF_FLOPS_PER_TAP == 6
    ro = bench.blf_roofline("pair", 2160, 3840, 3, 24, 10.0)
    taps = 3 * 2160 * 3840 * 2 * 49 ** 2
    assert ro["taps_per_launch"] == taps
    assert abs(ro["achieved"] - taps * 6 / 1e-2 / 1e12) < 1e-3
    assert abs(ro["frac"] - ro["achieved"] / 157.3) < 1e-4 and ro["unit"] == "TFLOP/s" and ro["bound"] == "alu"
    # the pair kernel issues one exp per unordered pair of taps, the tile kernel one per tap
    assert ro["exp_pipe"]["exps_per_tap"] == 0.5 and ro["kernel"].startswith("blf_pair_kernel<R=24>")
    assert abs(ro["exp_pipe"]["achieved_T_exp_s"] - taps * 0.5 / 1e-2 / 1e12) < 1e-3
    rt = bench.blf_roofline("tile", 1024, 1024, 3, 9, 1.0)
    assert rt["exp_pipe"]["exps_per_tap"] == 1.0 and rt["kernel"] == "blf_field_kernel<R=9>"
    # traffic only from a summary taken on the current kernel source
    assert ro["traffic"] is None
    # exponentials: a wave64 v_exp_f32 per 8 SIMD cycles, 256 CUs x 4 SIMDs at 2.4 GHz
    assert abs(bench.EXP_PEAK_T - 19.6608) < 1e-3
    assert 3 * 1024 * 1024 * 2 * 19 ** 2 == 2271215616


def test_interleaved_rounds_time_every_graph_exactly_steps_times():
    class G:
        def __init__(self):
            self.n = 0

        def replay(self):
            self.n += 1

    class Ev:
        def record(self):
            pass

        def elapsed_time(self, other):
            return 1.0

    class Cuda:
        Event = staticmethod(lambda enable_timing=True: Ev())

        @staticmethod
        def synchronize():
            pass

    class T:
        cuda = Cuda

    for steps in (1, 3, 7, 20):
        gs = {"a": G(), "b": G(), "c": G()}
        bench.time_interleaved(gs, steps, 2, T)
        assert all(g.n == steps + 2 for g in gs.values()), steps


def test_amf_byte_model_tree_height_matches_the_oracle():
    for ss in (1.0, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 64.0, 1e5):
        for sr in (1e-4, 0.01, 0.02, 0.05, 0.1, 0.3, 1.0, math.inf):
            assert bench_workloads.amf_tree_height(ss, sr) == oracle.amf_tree_height(ss, sr), (ss, sr)


def test_nc_byte_model():
    # per field and pass: field (or image) in, range source in, field out; the last
    # pass adds f in and the residual out in the field type
    assert bench_workloads.nc_bytes(4, 8, 1, 4, 1) == 2 * 32 * (12 * 2 + 4)
    assert bench_workloads.nc_bytes(4, 8, 3, 2, 3) == 2 * 3 * 32 * (12 * 2 * 3 + 2)


def test_traffic_is_read_only_while_the_kernel_source_matches(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1812_07122_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = csrc / "k.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "k.md").write_text(
        f"# summary\n\nsource_sha256: {digest}\nhbm_bytes_per_launch: 1.25e+07\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("k.hip", "k.md") == 1.25e7
    src.write_bytes(b"__global__ void k() { /* changed */ }\n")
    assert bench.traffic_from_profile("k.hip", "k.md") is None
    assert bench.traffic_from_profile("k.hip", "missing.md") is None


def test_committed_summaries_name_their_sources():
    # every PMC summary that feeds a roofline records the hash and the per-launch bytes
    for name, src in (("blf_filter_uhd_pmc.md", "blf_pair_kernel.hip"), ("blf_filter_rgb1024_pmc.md", "blf_pair_kernel.hip"),
                      ("nc_passes_rgb1024_pmc.md", "nc_kernels.hip"), ("amf_passes_rgb1024_pmc.md", "amf_kernels.hip")):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "source_sha256:" in text and "hbm_bytes_per_launch:" in text, name
        assert "rocprofv3 --pmc" in text, name
