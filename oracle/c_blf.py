"""Loader of the oracle's C bilateral filter (``blf_oracle.c``), built with gcc into
``oracle/libblf_oracle.so``.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the plain FP64 loops of
Eq. (1) for images too large for the NumPy version, parallel over rows with
OpenMP (``OMP_NUM_THREADS`` threads).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "blf_oracle.c")
LIB = os.path.join(HERE, "libblf_oracle.so")
_lib = None


def build() -> str:
    """Compile blf_oracle.c (IEEE FP64: no fast-math, baseline x86-64) into LIB."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.blf_oracle_fp64.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, dp]
        lib.blf_oracle_fp64.restype = ctypes.c_int
        _lib = lib
    return _lib


def bilateral_filter_c(p, q, sigma_s: float, sigma_r: float, radius: int) -> np.ndarray:
    """Eq. (1) on one 2-D field (same arguments and result as ``bilateral_filter``)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = p if q is None else np.ascontiguousarray(q, dtype=np.float64)
    if p.ndim != 2 or q.shape != p.shape:
        raise ValueError("p and q must be 2-D fields of one shape")
    H, W = p.shape
    out = np.empty_like(p)
    dp = ctypes.POINTER(ctypes.c_double)
    st = _load().blf_oracle_fp64(p.ctypes.data_as(dp), q.ctypes.data_as(dp), H, W, float(sigma_s),
                                 float(sigma_r), int(radius), out.ctypes.data_as(dp))
    if st != 0:
        raise ValueError(f"blf_oracle_fp64 rejected its arguments ({st})")
    return out
