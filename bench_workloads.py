"""Secondary benchmark workloads of bench.py (each returns one JSON-able dict).

copy   a plain 1 GiB device copy (torch), the reference that scales the HBM
       byte counters rocprofv3 reports for the library's kernels
"""
from __future__ import annotations

import time


def run_copy(args, torch, blfls):
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        dst.copy_(src)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    return {"metric": "device copy GB/s (read + write)", "value": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
            "higher_is_better": True, "config": {"workload": "copy 1 GiB float32 with torch copy_",
                                                 "bytes_read": nbytes, "bytes_written": nbytes}}
