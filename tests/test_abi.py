"""The C ABI on the CPU: every declared entry point is exported, and the host-side
validation that needs no GPU returns the documented statuses and messages."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1812_07122_amd as blfls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "blfls.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blfls_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = blfls.lib()
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(L, name), name
    bound = {n for n, _, _ in blfls.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def test_version():
    assert b"gfx950" in blfls.lib().blfls_version()


@pytest.mark.parametrize("shape,status,text", [
    ((1024, 1023, 3), -2, "W must be even"),
    ((7, 8, 1), -2, "factor into 2, 3 and 5"),
    ((22, 8, 1), -2, "factor into 2, 3 and 5"),
    ((8, 8, 5), -1, "C must be"),
    ((8, 8, 0), -1, "C must be"),
    ((0, 8, 1), -1, "H and W"),
    ((8, 16384, 1), -2, "at most 4096"),
])
def test_plan_rejects_bad_shapes(shape, status, text):
    L = blfls.lib()
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert L.blfls_plan(ctypes.byref(h), *shape, 0, ctypes.byref(ws)) == status
    assert text in L.blfls_last_error().decode()
    assert h.value is None


def test_null_arguments():
    L = blfls.lib()
    prm = blfls.make_params(20.0, 2.0, 0.1)
    assert L.blfls_smooth(None, ctypes.byref(prm), None, None, None, 8, None, None) == -1
    assert L.blfls_plan(None, 8, 8, 1, 0, None) == -1
    assert L.blfls_plan_destroy(None) == -1
    assert L.blfls_workspace_size(None, ctypes.byref(prm), None) == -1
    assert L.blfls_poll(None, 1, None, None) == -1
    assert L.blfls_submit(None, None, None) == -1
    assert L.blfls_server_destroy(None) == -1
    assert L.blfls_profile_read(None, 0) == -1


def test_server_create_validation():
    L = blfls.lib()
    h = ctypes.c_void_p()
    assert L.blfls_server_create(ctypes.byref(h), None, 1 << 30, 4, 16, 0, None) == -1
    assert L.blfls_server_create(ctypes.byref(h), ctypes.c_void_p(256), 1 << 30, 0, 16, 0, None) == -1
    assert L.blfls_server_create(ctypes.byref(h), ctypes.c_void_p(257), 1 << 30, 4, 16, 0, None) == -1
    assert L.blfls_server_create(ctypes.byref(h), ctypes.c_void_p(256), 1 << 30, 4, 16, 7, None) == -1
    assert L.blfls_server_create(ctypes.byref(h), ctypes.c_void_p(256), 1 << 20, 4, 16, 0, None) == -3


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(blfls, "_LIB_PATH", "/nonexistent/libblfls.so")
    monkeypatch.setattr(blfls, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        blfls.lib()


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors have the header's sizes and field offsets (compiled with gcc)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    import paper_1812_07122_amd as b
    checks = {
        "blfls_params": (b.Params, ["lambda", "sigma_s", "sigma_r", "radius", "iterations", "flags", "sigma_guide",
                                    "filter", "filter_iterations", "detail_gain"]),
        "blfls_request": (b.Request, ["H", "W", "C", "f", "guide", "u", "pitch", "params"]),
        "blfls_stats": (b.Stats, [n for n, _ in b.Stats._fields_]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "blfls.h"', "int main(void) {"]
    for struct, (_, fields) in checks.items():
        lines.append(f'  printf("{struct} %zu\\n", sizeof({struct}));')
        for fld in fields:
            lines.append(f'  printf("{struct}.{fld} %zu\\n", offsetof({struct}, {fld}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if line)
    for struct, (cls, fields) in checks.items():
        assert int(out[struct]) == ctypes.sizeof(cls), struct
        names = [n for n, _ in cls._fields_]
        for fld, py in zip(fields, names):
            assert int(out[f"{struct}.{fld}"]) == getattr(cls, py).offset, f"{struct}.{fld}"


def test_binding_rejects_tensors_it_cannot_pass_as_planar_float32_images():
    """The binding checks dtype, device, contiguity and shape before anything is queued
    (CPU tensors stand in for each mistake; the CUDA checks run in the GPU suite)."""
    torch = pytest.importorskip("torch")
    import paper_1812_07122_amd as b
    for bad in (torch.zeros(2, 3, 4, dtype=torch.float64), torch.zeros(2, 3, 4), np.zeros((3, 4), np.float32),
                torch.zeros(5)):
        with pytest.raises(ValueError):
            b._checked_image(bad, "f")
