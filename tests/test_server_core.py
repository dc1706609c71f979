"""The server's scheduling core on the CPU, driven by a fake executor
(tests/native/server_core_test.cpp): admission by arena bytes and slots, FAILED
retirement, drain on stop, E_AGAIN, E_NOMEM, unknown tickets, the bounded latency
window.  Built three times with g++: plain, with ThreadSanitizer, and with
AddressSanitizer + UndefinedBehaviorSanitizer (host code only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "server_core_test.cpp")
INC = os.path.join(ROOT, "paper_1812_07122_amd", "csrc")


@pytest.mark.parametrize("flavour,flags", [
    ("plain", ["-O2"]),
    ("tsan", ["-O1", "-g", "-fsanitize=thread"]),
    ("asan_ubsan", ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]),
])
def test_server_core_with_a_fake_executor(tmp_path, flavour, flags):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / f"server_core_{flavour}")
    cmd = [gxx, "-std=c++17", "-Wall", "-Wextra", "-pthread", *flags, "-I", INC, SRC, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=180, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all server core checks passed" in run.stdout
    assert "WARNING: ThreadSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr
