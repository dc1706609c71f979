"""BLF-LS edge-preserving smoothing on AMD MI355X (gfx950).

Thin Python binding over the C ABI of ``libblfls.so`` (declared in
``include/blfls.h``).  It only marshals arguments: PyTorch supplies device
memory and streams; every step of the method runs in the library's HIP
kernels.  If the library is missing, every call raises: there is no CPU path.

    import torch, paper_1812_07122_amd as blfls
    u = blfls.smooth(f_cuda, lam=20.0, sigma_s=3.0, sigma_r=0.1)
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

__all__ = [
    "Params", "Plan", "Server", "BlflsError", "smooth", "lib", "library_path", "profile_enable", "profile_read",
    "FP32", "MIXED_BF16", "MIXED_FP16", "F_NORMALIZE", "MAX_RADIUS",
    "QUEUED", "RUNNING", "DONE", "FAILED",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libblfls.so")

FP32, MIXED_BF16, MIXED_FP16 = 0, 1, 2
F_NORMALIZE = 0x1
MAX_RADIUS = 32
QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3
_PRECISIONS = {"fp32": FP32, "bf16": MIXED_BF16, "fp16": MIXED_FP16,
               FP32: FP32, MIXED_BF16: MIXED_BF16, MIXED_FP16: MIXED_FP16}

STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_UNSUPPORTED", -3: "E_NOMEM", -4: "E_AGAIN",
                -5: "E_HIP", -6: "E_UNKNOWN_TICKET"}


class BlflsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"BLFLS_{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    """Mirror of ``blfls_params``."""
    _fields_ = [
        ("lambda_", ctypes.c_float),
        ("sigma_s", ctypes.c_float),
        ("sigma_r", ctypes.c_float),
        ("radius", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("sigma_guide", ctypes.c_float),
        ("filter", ctypes.c_int32),
        ("filter_iterations", ctypes.c_int32),
        ("detail_gain", ctypes.c_float),
    ]


class Request(ctypes.Structure):
    """Mirror of ``blfls_request``."""
    _fields_ = [
        ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
        ("f", ctypes.c_void_p), ("guide", ctypes.c_void_p), ("u", ctypes.c_void_p),
        ("pitch", ctypes.c_int64), ("params", Params),
    ]


class Stats(ctypes.Structure):
    """Mirror of ``blfls_stats``."""
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
        ("queued_now", ctypes.c_uint64), ("running_now", ctypes.c_uint64),
        ("steps", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
        ("arena_in_use", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
        ("step_ms_mean", ctypes.c_double),
        ("latency_samples", ctypes.c_uint64),
        ("latency_p50_ms", ctypes.c_double),
        ("latency_p99_ms", ctypes.c_double),
        ("latency_max_ms", ctypes.c_double),
        ("graph_steps", ctypes.c_uint64),
        ("direct_steps", ctypes.c_uint64),
    ]


STAGES = ["upload", "gauss", "minmax", "blf", "rows_fwd", "cols", "rows_inv"]


class Profile(ctypes.Structure):
    """Mirror of ``blfls_profile``."""
    _fields_ = [("ms", ctypes.c_double * 7), ("launches", ctypes.c_uint64 * 7)]


_lib = None
_lib_lock = threading.Lock()

# (name, restype, argtypes) of every entry point of include/blfls.h
SIGNATURES = [
    ("blfls_plan", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    ("blfls_plan_workspace_size", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    ("blfls_workspace_size", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    ("blfls_plan_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("blfls_tonemap", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]),
    ("blfls_tonemap_workspace_size", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params),
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    ("blfls_smooth", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    ("blfls_smooth_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("blfls_server_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_void_p]),
    ("blfls_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    ("blfls_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int)]),
    ("blfls_server_stats", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    ("blfls_server_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("blfls_profile_enable", ctypes.c_int, [ctypes.c_int]),
    ("blfls_profile_read", ctypes.c_int, [ctypes.POINTER(Profile), ctypes.c_int]),
    ("blfls_last_error", ctypes.c_char_p, []),
    ("blfls_version", ctypes.c_char_p, []),
]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load ``libblfls.so``; raises if it was not built (no fallback exists)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(
                    f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                    "or `python paper_1812_07122_amd/build.py` (the BLF-LS path has no CPU fallback)")
            L = ctypes.CDLL(_LIB_PATH)
            for name, res, args in SIGNATURES:
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        msg = lib().blfls_last_error()
        raise BlflsError(status, msg.decode() if msg else "")


FILTERS = {"blf": 0, "nc": 1, "grid": 2, "amf": 3}


def make_params(lam: float, sigma_s: float, sigma_r: float, radius: int = -1, iterations: int = 1,
                normalize: bool = False, sigma_guide: float = 0.0, filter: str = "blf",
                filter_iterations: int = 0, detail_gain: float = 0.0) -> Params:
    """``filter``: "blf" (BLF-LS), "nc" (NC-LS: the domain transform's normalized
    convolution in place of the BLF; ``filter_iterations`` rounds, 0 = 3), "grid" (the
    bilateral-grid approximation of the BLF) or "amf" (AMF-LS: the adaptive-manifold
    filter; ``filter_iterations`` is the manifold tree height, 0 = the default rule).
    ``detail_gain`` m != 0 returns the detail-enhanced u + m (f - u) instead of u."""
    if filter not in FILTERS:
        raise ValueError(f"filter must be one of {sorted(FILTERS)}")
    return Params(float(lam), float(sigma_s), float(sigma_r), int(radius), int(iterations),
                  F_NORMALIZE if normalize else 0, float(sigma_guide), FILTERS[filter], int(filter_iterations),
                  float(detail_gain))


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def profile_enable(enable: bool = True):
    """Record HIP events around each kernel family of blfls_smooth (diagnostics)."""
    _check(lib().blfls_profile_enable(1 if enable else 0))


def profile_read(reset: bool = True) -> dict:
    """{stage: (ms summed, launches)} of the recorded events (waits for them)."""
    pr = Profile()
    _check(lib().blfls_profile_read(ctypes.byref(pr), 1 if reset else 0))
    return {name: (pr.ms[i], int(pr.launches[i])) for i, name in enumerate(STAGES)}


def _checked_image(t, name: str, shape=None, device=None):
    """t viewed as (C, H, W) after checking that it is a contiguous float32 CUDA tensor of
    that shape on that device (raises ValueError before anything is queued)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dim() not in (2, 3):
        raise ValueError(f"{name} must be a 2-D (H, W) or 3-D (C, H, W) torch tensor")
    t3 = t.reshape(1, *t.shape) if t.dim() == 2 else t
    if t3.dtype != torch.float32 or not t3.is_cuda or not t3.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t3.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t3.shape)})")
    if device is not None and t3.device != torch.device(device):
        raise ValueError(f"{name} is on {t3.device}, expected {device}")
    return t3


def _new_or_checked_out(out, f3, shape, device):
    import torch
    if out is None:
        return torch.empty_like(f3)
    u = _checked_image(out, "out", shape, device)
    if u.data_ptr() == f3.data_ptr():
        raise ValueError("out must not be f")
    return u


class Plan:
    """A ``blfls_plan`` for (C, H, W) images at one precision, with its workspace."""

    def __init__(self, H: int, W: int, C: int = 1, precision="fp32", device=None):
        import torch
        self.H, self.W, self.C = int(H), int(W), int(C)
        self.precision = _PRECISIONS[precision]
        self._handle = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(dev):
            _check(lib().blfls_plan(ctypes.byref(self._handle), self.H, self.W, self.C, self.precision,
                                    ctypes.byref(ws)))
        self.device = dev
        self._alloc_workspace(int(ws.value))

    def _alloc_workspace(self, nbytes: int):
        import torch
        # 256-byte alignment: over-allocate and offset
        self.workspace_bytes = nbytes
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self.workspace_ptr = (base + 255) // 256 * 256

    def workspace_for(self, prm: Params) -> int:
        """Workspace bytes ``blfls_smooth`` needs for these parameters (larger for the AMF)."""
        n = ctypes.c_size_t()
        _check(lib().blfls_workspace_size(self._handle, ctypes.byref(prm), ctypes.byref(n)))
        return int(n.value)

    def smooth(self, f, lam: float, sigma_s: float, sigma_r: float, radius: int = -1, iterations: int = 1,
               guide=None, normalize: bool = False, sigma_guide: float = 0.0, out=None, stream=None,
               filter: str = "blf", filter_iterations: int = 0, detail_gain: float = 0.0):
        import torch
        shape = (self.C, self.H, self.W)
        f3 = _checked_image(f, "f", shape, self.device)
        g3 = None if guide is None else _checked_image(guide, "guide", shape, self.device)
        u = _new_or_checked_out(out, f3, shape, self.device)
        prm = make_params(lam, sigma_s, sigma_r, radius, iterations, normalize, sigma_guide, filter,
                          filter_iterations, detail_gain)
        need = self.workspace_for(prm)
        if need > self.workspace_bytes:
            # work queued earlier (on any stream) may still use the old buffer
            torch.cuda.synchronize(self.device)
            self._alloc_workspace(need)
        _check(lib().blfls_smooth(self._handle, ctypes.byref(prm), ctypes.c_void_p(f3.data_ptr()),
                                  ctypes.c_void_p(g3.data_ptr() if g3 is not None else 0),
                                  ctypes.c_void_p(u.data_ptr()), self.W, ctypes.c_void_p(self.workspace_ptr),
                                  ctypes.c_void_p(_stream_handle(stream))))
        return u.reshape(f.shape)

    def smooth_noalloc(self, f, lam: float, sigma_s: float, sigma_r: float, out, radius: int = -1,
                       iterations: int = 1, guide=None, normalize: bool = False, sigma_guide: float = 0.0,
                       stream=None, filter: str = "blf", filter_iterations: int = 0, detail_gain: float = 0.0):
        """``blfls_smooth_noalloc``: the same smoothing into the caller's ``out`` with the
        library's static per-GPU scratch as workspace (no device allocation by the library
        or by this call; calls that overlap on one GPU race)."""
        shape = (self.C, self.H, self.W)
        f3 = _checked_image(f, "f", shape, self.device)
        g3 = None if guide is None else _checked_image(guide, "guide", shape, self.device)
        if out is None:
            raise ValueError("out is required (the call allocates nothing)")
        u = _new_or_checked_out(out, f3, shape, self.device)
        prm = make_params(lam, sigma_s, sigma_r, radius, iterations, normalize, sigma_guide, filter,
                          filter_iterations, detail_gain)
        _check(lib().blfls_smooth_noalloc(self._handle, ctypes.byref(prm), ctypes.c_void_p(f3.data_ptr()),
                                          ctypes.c_void_p(g3.data_ptr() if g3 is not None else 0),
                                          ctypes.c_void_p(u.data_ptr()), self.W,
                                          ctypes.c_void_p(_stream_handle(stream))))
        return out

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _check(lib().blfls_plan_destroy(self._handle))
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plan_cache: dict = {}


def smooth(f, lam: float = 1024.0, sigma_s: float = 3.0, sigma_r: float = 0.1, radius: int = -1,
           iterations: int = 1, guide=None, normalize: bool = False, sigma_guide: float = 0.0,
           precision="fp32", out=None, stream=None, filter: str = "blf", filter_iterations: int = 0,
           detail_gain: float = 0.0):
    """BLF-LS of a float32 CUDA image of shape (H, W) or (C, H, W); returns u (same shape).

    lam is lambda of Eq. (7) (the paper's default is 1024), sigma_s / sigma_r the
    spatial and range sigmas of Eq. (1), radius -1 means ceil(3 sigma_s).
    filter="nc" runs NC-LS (Section III-D) with filter_iterations rounds (0 = 3);
    filter="grid" the bilateral-grid approximation; filter="amf" AMF-LS with a manifold
    tree of height filter_iterations (0 = the default rule).  detail_gain m != 0 returns
    u + m (f - u) (the experiments' detail enhancement uses m = 5).
    """
    C, H, W = tuple(_checked_image(f, "f").shape)
    key = (C, H, W, _PRECISIONS[precision], f.device.index)
    plan = _plan_cache.get(key)
    if plan is None:
        plan = Plan(H, W, C, precision, device=f.device)
        _plan_cache[key] = plan
    return plan.smooth(f, lam, sigma_s, sigma_r, radius, iterations, guide, normalize, sigma_guide, out, stream,
                       filter, filter_iterations, detail_gain)


def tonemap(rgb, lam: float = 20.0, sigma_s: float = 8.0, sigma_r: float = 0.03, contrast: float = 5.0,
            normalize: bool = True, out=None, stream=None, filter: str = "blf", **kw):
    """Log-domain HDR tone mapping of a float32 CUDA image of shape (3, H, W) (``blfls_tonemap``):
    the BLF-LS base of log10 intensity is compressed to ``contrast`` and recombined with the
    detail layer and the colour ratios.  ``normalize`` maps the log intensity to [0, 1] before
    smoothing (the experiments section's convention for sigma_r)."""
    import torch
    if rgb.dim() != 3 or rgb.shape[0] != 3 or rgb.dtype != torch.float32 or not rgb.is_cuda or not rgb.is_contiguous():
        raise ValueError("rgb must be a contiguous float32 CUDA tensor of shape (3, H, W)")
    _, H, W = rgb.shape
    key = (1, H, W, _PRECISIONS["fp32"], rgb.device.index)
    plan = _plan_cache.get(key)
    if plan is None:
        plan = Plan(H, W, 1, "fp32", device=rgb.device)
        _plan_cache[key] = plan
    prm = make_params(lam, sigma_s, sigma_r, normalize=normalize, filter=filter, **kw)
    n = ctypes.c_size_t()
    _check(lib().blfls_tonemap_workspace_size(plan._handle, ctypes.byref(prm), ctypes.byref(n)))
    if int(n.value) > plan.workspace_bytes:
        torch.cuda.synchronize(plan.device)
        plan._alloc_workspace(int(n.value))
    out = torch.empty_like(rgb) if out is None else out
    _check(lib().blfls_tonemap(plan._handle, ctypes.byref(prm), ctypes.c_void_p(rgb.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), W, float(contrast),
                               ctypes.c_void_p(plan.workspace_ptr), ctypes.c_void_p(_stream_handle(stream))))
    return out


class Server:
    """Continuous-batching server (``blfls_server_*``) over a caller-owned device arena."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, queue_capacity: int = 4096, precision="fp32",
                 stream=None, device=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = dev
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=dev)
        base = (self._arena.data_ptr() + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self._handle = ctypes.c_void_p()
        self._keep: dict = {}
        with torch.cuda.device(dev):
            _check(lib().blfls_server_create(ctypes.byref(self._handle), ctypes.c_void_p(base),
                                             int(arena_bytes), int(max_slots), int(queue_capacity),
                                             _PRECISIONS[precision], ctypes.c_void_p(int(self._stream.cuda_stream))))

    @property
    def stream(self):
        return self._stream

    def submit(self, f, lam: float, sigma_s: float, sigma_r: float, radius: int = -1, iterations: int = 1,
               guide=None, normalize: bool = False, sigma_guide: float = 0.0, out=None, filter: str = "blf",
               filter_iterations: int = 0, detail_gain: float = 0.0):
        """Queue one image; returns (ticket, u).  u is valid once poll(ticket) reports DONE.

        The server's stream is made to wait for the caller's current stream first, so inputs
        still being written there, and the memory of a new ``u`` allocated there, are
        ordered before the request's kernels.  Raises BlflsError with status E_AGAIN when
        the queue is full, ValueError for tensors that are not contiguous float32 CUDA
        images of one shape on the server's device.
        """
        import torch
        f3 = _checked_image(f, "f", None, self.device)
        C, H, W = tuple(f3.shape)
        g3 = None if guide is None else _checked_image(guide, "guide", (C, H, W), self.device)
        u = _new_or_checked_out(out, f3, (C, H, W), self.device)
        self._stream.wait_stream(torch.cuda.current_stream(self.device))
        req = Request(H, W, C, f3.data_ptr(), g3.data_ptr() if g3 is not None else 0, u.data_ptr(), W,
                      make_params(lam, sigma_s, sigma_r, radius, iterations, normalize, sigma_guide, filter,
                                  filter_iterations, detail_gain))
        ticket = ctypes.c_uint64()
        _check(lib().blfls_submit(self._handle, ctypes.byref(req), ctypes.byref(ticket)))
        self._keep[ticket.value] = (f, guide, u)
        return ticket.value, u.reshape(f.shape)

    def poll(self, ticket: int):
        """(state, status) of a ticket; DONE/FAILED retire it."""
        state = ctypes.c_int32()
        result = ctypes.c_int()
        _check(lib().blfls_poll(self._handle, ctypes.c_uint64(ticket), ctypes.byref(state), ctypes.byref(result)))
        if state.value in (DONE, FAILED):
            self._keep.pop(ticket, None)
        return state.value, result.value

    def stats(self) -> dict:
        st = Stats()
        _check(lib().blfls_server_stats(self._handle, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in Stats._fields_}

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _check(lib().blfls_server_destroy(self._handle))
            self._handle = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
