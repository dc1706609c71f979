"""The symmetric-pair filter's work split (paper_1812_07122_amd/csrc/blfls_pair_geom.h:
bands, blocks, the partial-sum record layout) on the CPU, by the native test in
tests/native/pair_geometry_test.cpp over about 1.3 million image shapes and every
radius class; built with g++, plain and with AddressSanitizer +
UndefinedBehaviorSanitizer (host code only).  The kernels and the plan use the same
header, so the invariants checked here (bands at least R wide and R + K - 1 tall,
carried rows landing in the next band, records disjoint and within the workspace)
are the ones their indexing relies on."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "pair_geometry_test.cpp")
INC = os.path.join(ROOT, "paper_1812_07122_amd", "csrc")


@pytest.mark.parametrize("flavour,flags", [
    ("plain", ["-O2"]),
    ("asan_ubsan", ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]),
])
def test_pair_geometry_invariants(tmp_path, flavour, flags):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / f"pair_geometry_{flavour}")
    cmd = [gxx, "-std=c++17", "-Wall", "-Wextra", *flags, "-I", INC, SRC, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all pair geometry checks passed" in run.stdout
    assert "runtime error" not in run.stderr, run.stderr
