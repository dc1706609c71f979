"""Secondary benchmark workloads of bench.py (each returns one JSON-able dict).

copy   a plain 1 GiB device copy (torch), the reference that scales the HBM
       byte counters rocprofv3 reports for the library's kernels
uhd    3840x2160 RGB, sigma_s = 8 (r = 24), sigma_r = 0.05, lambda = 50: plain FP32
       against BF16 and FP16 field storage; each compared with the FP64 oracle
       over the whole image (oracle channels run in CPU worker processes started
       before the GPU is touched)
serve  requests of uneven sizes with Poisson arrivals through the continuous-
       batching server: saturation rate, then open loop at 0.7 of it; p50/p99
       latency; every result compared bitwise with the same request run alone
joint  64 guided 2048x2048 pairs, FP16 field storage, lambda = 30, sigma_s = 4,
       sigma_r = 0.08, through the server; 8 pairs checked against the oracle

Oracle worker processes start in ``prepare(args)``, before any GPU call; uhd, nc,
amf and grid hand them their jobs at once (the oracle runs beside the timed graph
replays), serve and joint only after their timed runs (the server's host thread
must not share the CPUs with them); ``run_*`` collects the results at the end.
"""
from __future__ import annotations

import math
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
SERVE_SIZES = [(320, 480), (480, 640), (720, 1280), (1080, 1920), (1536, 2048)]  # (H, W)


def _oracle_channel(job):
    """Worker: FP64 oracle on one channel (inputs already rounded to FP32)."""
    import oracle
    f, guide, lam, ss, sr = job[:5]
    kw = job[5] if len(job) > 5 else {}
    return oracle.smooth(f, lam, ss, sr, guide=guide, **kw)


# NC-LS workloads on the paper's timing shape (1024x1024 RGB, Table I): the HDR
# tone-mapping parameters of the NC-LS figure, and rolling-guidance NC-LS with the
# texture-removal settings (three iterations from a Gaussian-smoothed guide)
NC_CONFIGS = {
    "nc": dict(lam=20.0, sigma_s=12.0, sigma_r=0.05, filter="nc"),
    "nc_rolling": dict(lam=20.0, sigma_s=8.0, sigma_r=0.02, iterations=3, sigma_guide=2.5, filter="nc"),
}


# AMF-LS on the same shape: the detail-enhancement settings of the AMF-LS figures
# (sigma_s = 12, sigma_r = 0.02: a tree of height 2, three manifolds) and a deeper
# tree (height 3, seven manifolds) with the HDR settings (sigma_s = 16, sigma_r = 0.03)
AMF_CONFIGS = {
    "amf": dict(lam=20.0, sigma_s=12.0, sigma_r=0.02, filter="amf"),
    "amf_deep": dict(lam=20.0, sigma_s=16.0, sigma_r=0.03, filter="amf"),
}


def _pool(n):
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(processes=n)


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


# ---------------------------------------------------------------------------
# workload inputs (numpy, CPU) and oracle submissions, before any GPU call
# ---------------------------------------------------------------------------

def prepare(args):
    import synth
    state = {}
    if args.workload == "uhd":
        f = synth.voronoi_rgb(2160, 3840, 2)
        state["f"] = f.astype(np.float32)
        if not args.no_cpu_baseline:
            pool = _pool(3)
            jobs = [(state["f"][c].astype(np.float64), None, 50.0, 8.0, 0.05) for c in range(3)]
            state["t_oracle0"] = time.perf_counter()
            state["oracle"] = pool.map_async(_oracle_channel, jobs)
            state["pool"] = pool
    elif args.workload == "nc":
        f = synth.voronoi_rgb(1024, 1024, 1)
        state["f"] = f.astype(np.float32)
        if not args.no_cpu_baseline:
            pool = _pool(3)
            kw = {k: v for k, v in NC_CONFIGS["nc"].items() if k not in ("lam", "sigma_s", "sigma_r")}
            c = NC_CONFIGS["nc"]
            jobs = [(state["f"][ch].astype(np.float64), None, c["lam"], c["sigma_s"], c["sigma_r"], kw)
                    for ch in range(3)]
            state["t_oracle0"] = time.perf_counter()
            state["oracle"] = pool.map_async(_oracle_channel, jobs)
            state["pool"] = pool
    elif args.workload == "amf":
        f = synth.voronoi_rgb(1024, 1024, 1)
        state["f"] = f.astype(np.float32)
        if not args.no_cpu_baseline:
            pool = _pool(3)
            c = AMF_CONFIGS["amf"]
            kw = {k: v for k, v in c.items() if k not in ("lam", "sigma_s", "sigma_r")}
            jobs = [(state["f"][ch].astype(np.float64), None, c["lam"], c["sigma_s"], c["sigma_r"], kw)
                    for ch in range(3)]
            state["t_oracle0"] = time.perf_counter()
            state["oracle"] = pool.map_async(_oracle_channel, jobs)
            state["pool"] = pool
    elif args.workload == "grid":
        f = synth.voronoi_rgb(2160, 3840, 2)
        state["f"] = f.astype(np.float32)
        if not args.no_cpu_baseline:
            pool = _pool(1)
            c = GRID_CONFIG
            jobs = [(state["f"][0].astype(np.float64), None, c["lam"], c["sigma_s"], c["sigma_r"], {"filter": "grid"})]
            state["t_oracle0"] = time.perf_counter()
            state["oracle"] = pool.map_async(_oracle_channel, jobs)
            state["pool"] = pool
    elif args.workload == "joint":
        pairs = [synth.joint_pair(2048, 2048, i) for i in range(64 if args.requests >= 64 else args.requests)]
        state["pairs"] = [(t.astype(np.float32), g.astype(np.float32)) for t, g in pairs]
        if not args.no_cpu_baseline:
            # the workers start now (before the GPU is touched) but get their jobs only
            # after the timed runs: the server's host thread must not share the CPUs
            state["pool"] = _pool(8)
            state["oracle_jobs"] = [(t.astype(np.float64), g.astype(np.float64), 30.0, 4.0, 0.08)
                                    for t, g in state["pairs"][:8]]
    elif args.workload == "serve":
        rng = np.random.default_rng(3999)
        n = args.requests
        # a pool of 4 seeded images per size (seeds 3000 + 10 size + j), channels 1000-apart
        images = {}
        for si, (H, W) in enumerate(SERVE_SIZES):
            for j in range(4):
                base = 3000 + 10 * si + j
                images[(si, j)] = np.stack([synth.voronoi_image(H, W, base + 1000 * c) for c in range(3)]).astype(np.float32)
        reqs = []
        for i in range(n):
            r = np.random.default_rng(3000 + i)
            si = int(r.integers(0, len(SERVE_SIZES)))
            reqs.append(dict(img=(si, int(r.integers(0, 4))), lam=float(r.uniform(5, 100)),
                             sigma_s=float(r.choice([2.0, 4.0, 8.0])), sigma_r=float(r.uniform(0.03, 0.2))))
        state["images"] = images
        state["reqs"] = reqs
        state["gaps"] = rng.exponential(1.0, size=n)  # unit-rate inter-arrival times
        if not args.no_cpu_baseline:
            # oracle on a seeded sample of 8 requests of at most 1 MP (CPU minutes otherwise)
            small = [i for i, q in enumerate(reqs) if SERVE_SIZES[q["img"][0]][0] * SERVE_SIZES[q["img"][0]][1] <= 1_000_000]
            pick = sorted(np.random.default_rng(4242).choice(small, size=min(8, len(small)), replace=False).tolist())
            jobs = []
            for i in pick:
                q = reqs[i]
                jobs.append((images[q["img"]][0].astype(np.float64), None, q["lam"], q["sigma_s"], q["sigma_r"]))
            state["oracle_pick"] = pick
            state["pool"] = _pool(8)          # jobs submitted after the timed runs, as for joint
            state["oracle_jobs"] = jobs
    return state


def _submit(state):
    """Hand deferred oracle jobs to the workers started by prepare()."""
    if "oracle_jobs" in state and "oracle" not in state:
        state["t_oracle0"] = time.perf_counter()
        state["oracle"] = state["pool"].map_async(_oracle_channel, state.pop("oracle_jobs"))


def _collect(state):
    if "oracle" not in state:
        return None, None
    import sys
    t_wait = time.perf_counter()
    while not state["oracle"].ready():
        state["oracle"].wait(30.0)
        if not state["oracle"].ready():
            print(f"bench: waiting for the CPU oracle ({time.perf_counter() - t_wait:.0f} s)", file=sys.stderr,
                  flush=True)
    res = state["oracle"].get()
    t = time.perf_counter() - state.get("t_oracle0", time.perf_counter())
    state["pool"].close()
    state["pool"].join()
    return res, t


# ---------------------------------------------------------------------------

def run_copy(args, torch, blfls, state=None):
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


def run_uhd(args, torch, blfls, state):
    from bench import time_plan, fft_bytes, blf_roofline, filter_path
    H, W, C, r = 2160, 3840, 3, 24
    prm = dict(lam=50.0, sigma_s=8.0, sigma_r=0.05)
    f = torch.from_numpy(state["f"]).cuda()
    u = torch.empty_like(f)
    steps = max(1, min(args.steps, 10))
    results, outs = {}, {}
    for prec, fb in (("fp32", 4), ("bf16", 2), ("fp16", 2)):
        plan = blfls.Plan(H, W, C, prec)
        ms, stages = time_plan(plan, f, u, prm, steps, min(args.warmup, 2), torch, blfls)
        outs[prec] = plan.smooth(f, **prm).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        blf_ms = stages["blf"][0] / max(stages["blf"][1], 1)
        taps = C * H * W * 2 * (2 * r + 1) ** 2
        rf, cl, ri = fft_bytes(H, W, C, fb)
        fft_ms = sum(stages[k][0] / max(stages[k][1], 1) for k in ("rows_fwd", "cols", "rows_inv"))
        fft = {}
        for name, nbytes in (("rows_fwd", rf), ("cols", cl), ("rows_inv", ri)):
            t = stages[name][0] / max(stages[name][1], 1)
            fft[name] = {"ms": round(t, 4), "GB/s": round(nbytes / (t * 1e-3) / 1e9, 1),
                         "frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        ro = blf_roofline(filter_path(blfls, H, W, C, prm), H, W, C, r, blf_ms)
        results[prec] = {"MPix/s": round(H * W / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
                         "blf_ms": round(blf_ms, 4), "blf_roofline": ro,
                         "fft_ms": round(fft_ms, 4),
                         "fft_GB/s": round((rf + cl + ri) / (fft_ms * 1e-3) / 1e9, 1),
                         "fft_frac": round((rf + cl + ri) / (fft_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "fft_passes": fft}
        plan.close()
    for prec in ("bf16", "fp16"):
        results[prec]["max_abs_vs_fp32_gpu"] = float(np.max(np.abs(outs[prec] - outs["fp32"])))
    ref, t = _collect(state)
    out = {"metric": "MPix/s BLF-LS at 1 GPU (plain FP32 vs mixed)", "value": results["fp32"]["MPix/s"],
           "unit": "MPix/s", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 2),
           "ms_per_step": results["fp32"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "uhd: 3840x2160 RGB, lambda=50, sigma_s=8 (r=24), sigma_r=0.05, 1 iteration",
                      "H": H, "W": W, "C": C},
           "roofline": results["fp32"]["blf_roofline"],
           "precisions": results}
    if ref is not None:
        refs = np.stack(ref)
        for prec in results:
            results[prec]["max_abs_vs_oracle"] = float(np.max(np.abs(outs[prec] - refs)))
            results[prec]["psnr_vs_oracle_db"] = round(_psnr(outs[prec], refs), 2)
        out["cpu_baseline"] = {"value": round(H * W / t / 1e6, 5), "unit": "MPix/s", "cores": 3, "kind": "oracle",
                               "sample": f"whole image, 3 channels in 3 worker processes, {t:.0f} s wall "
                                         "(includes time overlapped with the GPU runs)"}
    return out


# the bilateral grid where it pays: the 3840x2160 RGB workload (sigma_s = 8, 2401 taps
# per pixel-field for the exact filter)
GRID_CONFIG = dict(lam=50.0, sigma_s=8.0, sigma_r=0.05)


def run_grid(args, torch, blfls, state):
    from bench import time_plan, time_graph
    H, W, C = 2160, 3840, 3
    f = torch.from_numpy(state["f"]).cuda()
    u = torch.empty_like(f)
    steps = max(1, min(args.steps, 20))
    res = {}
    outs = {}
    for name, prm in (("grid", dict(GRID_CONFIG, filter="grid")), ("exact", dict(GRID_CONFIG))):
        plan = blfls.Plan(H, W, C, "fp32")
        n = steps if name == "grid" else max(1, min(steps, 3))
        ms_eager, stages = time_plan(plan, f, u, prm, n, min(args.warmup, 2), torch, blfls)
        ug = torch.empty_like(f)
        ms, graph = time_graph(plan, f, ug, prm, n, min(args.warmup, 2), torch)
        outs[name] = plan.smooth(f, **prm).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        same = bool(np.array_equal(ug.cpu().numpy().astype(np.float64), outs[name]))
        del graph
        filt_ms = stages["blf"][0] / max(stages["blf"][1], 1)
        res[name] = {"MPix/s": round(H * W / (ms * 1e-3) / 1e6, 2), "ms_per_image": round(ms, 4),
                     "eager_MPix/s": round(H * W / (ms_eager * 1e-3) / 1e6, 2),
                     "graph_vs_eager_bitwise_equal": same,
                     "filter_ms": round(filt_ms, 4), "steps": n}
        plan.close()
    d = outs["grid"] - outs["exact"]
    res["grid"]["vs_exact_blf_ls"] = {"psnr_db": round(_psnr(outs["grid"], outs["exact"]), 2),
                                      "max_abs": float(np.max(np.abs(d))),
                                      "rms": float(np.sqrt(np.mean(d * d)))}
    out = {"metric": "MPix/s grid-approximated BLF-LS at 1 GPU", "value": res["grid"]["MPix/s"], "unit": "MPix/s",
           "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 2), "ms_per_step": res["grid"]["ms_per_image"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "grid: 3840x2160 RGB, lambda=50, sigma_s=8, sigma_r=0.05, bilateral-grid filter "
                                  "(cells of 8 pixels by one range cell) against the exact windowed filter (r=24)",
                      "H": H, "W": W, "C": C},
           "filters": res}
    ops = grid_ops(H, W, C, max(1, int(math.floor(GRID_CONFIG["sigma_s"] + 0.5))), grid_z_slots(state["f"], GRID_CONFIG["sigma_r"]))
    gfrac = ops / (res["grid"]["filter_ms"] * 1e-3) / 1e12
    out["roofline"] = {"kernel": "grid_filter_kernel", "bound": "alu", "achieved": round(gfrac, 3),
                       "peak": VALU_PEAK_T, "unit": "T lane-ops/s", "frac": round(gfrac / VALU_PEAK_T, 4),
                       "traffic": None, "launch_ms": res["grid"]["filter_ms"], "ops_per_launch": ops}
    ref, t = _collect(state)
    if ref is not None:
        out["max_abs_vs_oracle_ch0"] = float(np.max(np.abs(outs["grid"][0] - ref[0])))
        out["cpu_baseline"] = {"value": round(H * W / (3 * t) / 1e6, 5), "unit": "MPix/s", "cores": 1,
                               "kind": "oracle", "sample": f"channel 0 of the image ({t:.1f} s wall, overlapping the "
                                                           "GPU runs); rate scaled to RGB images"}
    return out


# single-issue VOP2 lane rate: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz
VALU_PEAK_T = 78.6432


def grid_ops(H, W, C, s, zslots):
    """Algorithmic VALU lane-operations of the bilateral-grid filter, per launch (both
    fields of every channel), each pixel and grid cell counted once: the splat of every
    pixel (two gradients, the bin, two read-add-writes: about 25 ops), the blur (3 axes x
    2 grids x 5 taps over the zslots range slots of every cell of the (W/s + 1) x (H/s + 1)
    grid), and the slice of every pixel (two gradients, the cell coordinates, 8 cells x 2
    grids trilinear, the division: about 60 ops).  The kernel's own halo work (each
    workgroup rebuilds the cells within 3 of its tile) is not counted."""
    cells = ((W - 1 + s // 2) // s + 1) * ((H - 1 + s // 2) // s + 1)
    per_field = H * W * 25 + cells * zslots * 2 * 5 * 3 + H * W * 60
    return int(2 * C * per_field)


def grid_z_slots(f, sigma_r, normalize=False):
    """Mean range slots per cell the grid blurs over the gradient fields of image f
    [C][H][W]: round(span / sigma_r) + 1 bins (round(1 / sigma_r) + 1 when the range
    axis is normalised), at most 32, plus two empty bins at each end."""
    slots = []
    for ch in np.asarray(f, dtype=np.float64):
        for ax in (1, 0):
            q = np.roll(ch, -1, axis=ax) - ch
            span = 1.0 if normalize else float(q.max() - q.min())
            slots.append(min(32, int(math.floor(span / sigma_r + 0.5)) + 1) + 4)
    return float(np.mean(slots))


def nc_bytes(H, W, C, field_bytes, rounds):
    """Algorithmic HBM bytes of the NC passes of one image: per field and pass, the field
    in (the first pass reads f instead), the range-source image in and the field out; the
    last pass also reads f and writes the residual in the field type."""
    per_field = 12 * 2 * rounds + field_bytes
    return 2 * C * H * W * per_field


def run_nc(args, torch, blfls, state):
    from bench import time_plan, time_graph, fft_bytes, traffic_from_profile
    H, W, C = 1024, 1024, 3
    f = torch.from_numpy(state["f"]).cuda()
    u = torch.empty_like(f)
    configs = {}
    outs = {}
    for name, prm in NC_CONFIGS.items():
        if args.only and name != args.only:
            continue
        iters = prm.get("iterations", 1)
        plan = blfls.Plan(H, W, C, "fp32")
        ms_eager, stages = time_plan(plan, f, u, prm, args.steps, args.warmup, torch, blfls)
        ug = torch.empty_like(f)
        ms, graph = time_graph(plan, f, ug, prm, args.steps, args.warmup, torch)
        outs[name] = plan.smooth(f, **prm).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        same = bool(np.array_equal(ug.cpu().numpy().astype(np.float64), outs[name]))
        del graph
        nc_ms = stages["blf"][0] / max(stages["blf"][1], 1)          # one iteration's NC passes
        nb = nc_bytes(H, W, C, 4, 3)
        rf, cl, ri = fft_bytes(H, W, C, 4)
        fft_ms = sum(stages[k][0] / max(stages[k][1], 1) for k in ("rows_fwd", "cols", "rows_inv"))
        configs[name] = {"params": {k: v for k, v in prm.items()}, "MPix/s": round(H * W / (ms * 1e-3) / 1e6, 2),
                         "ms_per_image": round(ms, 4), "iterations": iters,
                         "eager_MPix/s": round(H * W / (ms_eager * 1e-3) / 1e6, 2),
                         "graph_vs_eager_bitwise_equal": same,
                         "nc_passes_ms": round(nc_ms, 4),
                         "nc_passes": {"bound": "hbm", "bytes": nb, "GB/s": round(nb / (nc_ms * 1e-3) / 1e9, 1),
                                       "frac": round(nb / (nc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                         "fft_ms": round(fft_ms, 4),
                         "fft_GB/s": round((rf + cl + ri) / (fft_ms * 1e-3) / 1e9, 1)}
        plan.close()
    main = configs[args.only or "nc"]
    out = {"metric": "MPix/s NC-LS at 1 GPU", "value": main["MPix/s"], "unit": "MPix/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main["ms_per_image"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "nc: 1024x1024 RGB NC-LS, lambda=20, sigma_s=12, sigma_r=0.05, 3 NC rounds; "
                                  "nc_rolling: sigma_s=8, sigma_r=0.02, 3 iterations, Gaussian guide sigma=2.5",
                      "H": H, "W": W, "C": C},
           "roofline": {"kernel": "NC passes (nc_rows_kernel, nc_cols_kernel)", "bound": "hbm",
                        "achieved": main["nc_passes"]["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": main["nc_passes"]["frac"],
                        "traffic": traffic_from_profile("nc_kernels.hip", "nc_passes_rgb1024_pmc.md")},
           "configs": configs,
           "paper_context": {"value": 2.5, "unit": "MPix/s", "note": "Table I: NC-LS 0.42 s per 1024x1024 RGB image "
                             "(CPU Python with OpenCV's NC filter, hardware unstated)"}}
    ref, t = _collect(state)
    if ref is not None:
        refs = np.stack(ref)
        if "nc" in outs:
            out["max_abs_vs_oracle"] = float(np.max(np.abs(outs["nc"] - refs)))
        out["cpu_baseline"] = {"value": round(H * W / t / 1e6, 5), "unit": "MPix/s", "cores": 3, "kind": "oracle",
                               "sample": f"the nc configuration, whole image, 3 channels in 3 worker processes, "
                                         f"{t:.1f} s wall (overlapping the GPU runs)"}
    return out


def amf_tree_height(sigma_s, sigma_r):
    """The library's default tree height, max(2, ceil(H_s L)) capped at 6 (for the byte count)."""
    hs = max(0.0, math.floor(math.log2(float(np.float32(sigma_s)))) - 1.0)
    lr = 0.0 if math.isinf(sigma_r) else max(0.0, 1.0 - float(np.float32(sigma_r)))
    return int(min(6, max(2, math.ceil(hs * lr))))


def amf_bytes(H, W, C, field_bytes, height):
    """HBM bytes the AMF passes of one image move by design, per gradient field and pixel
    (FP32 values; an image read forms a gradient, its neighbour comes from cache):
      root low-pass  rows: image in, value out; columns: value in 3 times, manifold out;
      each manifold  rows: manifold, 2 images in, 2 values out; columns: 2 values and
                     the manifold in 3 times, range image in, the three running sums in
                     and out (the first slice only writes them, the last writes the
                     residual in the field type and reads f's image instead);
      inner ones     rows: manifold and image in, 4 values out; columns: 4 values in 3
                     times, 2 children out;
    plus the column scans' segment summaries and carries (16-row segments)."""
    def scan(n):   # per pixel: summaries, carry folds and carries of an n-channel column scan
        return (2 * (1 + n) + 2 * (1 + n) + 2 * n + 2 * n) / 16.0
    K = 2 ** height - 1
    inner = 2 ** (height - 1) - 1
    per = (2 + 4 + scan(1))                                    # root
    per += K * (5 + 9 + 1 + scan(2))                           # splat rows + columns (before the sums)
    if K == 1:                                                 # the only slice writes the residual
        per += 1 + field_bytes / 4.0
    else:                                                      # first writes, middle r+w, last r + out
        per += 3 + (K - 2) * 6 + (3 + 1 + field_bytes / 4.0)
    per += inner * (6 + 14 + scan(4))                          # split rows + columns
    return int(2 * C * H * W * 4 * per)


def run_amf(args, torch, blfls, state):
    from bench import time_plan, time_graph, fft_bytes, traffic_from_profile
    H, W, C = 1024, 1024, 3
    f = torch.from_numpy(state["f"]).cuda()
    u = torch.empty_like(f)
    configs = {}
    outs = {}
    for name, prm in AMF_CONFIGS.items():
        if args.only and name != args.only:
            continue
        plan = blfls.Plan(H, W, C, "fp32")
        ms_eager, stages = time_plan(plan, f, u, prm, args.steps, args.warmup, torch, blfls)
        ug = torch.empty_like(f)
        ms, graph = time_graph(plan, f, ug, prm, args.steps, args.warmup, torch)
        outs[name] = plan.smooth(f, **prm).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        same = bool(np.array_equal(ug.cpu().numpy().astype(np.float64), outs[name]))
        del graph
        amf_ms = stages["blf"][0] / max(stages["blf"][1], 1)
        height = amf_tree_height(prm["sigma_s"], prm["sigma_r"])
        nb = amf_bytes(H, W, C, 4, height)
        rf, cl, ri = fft_bytes(H, W, C, 4)
        fft_ms = sum(stages[k][0] / max(stages[k][1], 1) for k in ("rows_fwd", "cols", "rows_inv"))
        configs[name] = {"params": dict(prm), "tree_height": height, "manifolds": 2 ** height - 1,
                         "MPix/s": round(H * W / (ms * 1e-3) / 1e6, 2), "ms_per_image": round(ms, 4),
                         "eager_MPix/s": round(H * W / (ms_eager * 1e-3) / 1e6, 2),
                         "graph_vs_eager_bitwise_equal": same,
                         "amf_ms": round(amf_ms, 4),
                         "amf_passes": {"bound": "hbm", "bytes": nb, "GB/s": round(nb / (amf_ms * 1e-3) / 1e9, 1),
                                        "frac": round(nb / (amf_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                         "fft_ms": round(fft_ms, 4),
                         "fft_GB/s": round((rf + cl + ri) / (fft_ms * 1e-3) / 1e9, 1)}
        plan.close()
    main = configs[args.only or "amf"]
    out = {"metric": "MPix/s AMF-LS at 1 GPU", "value": main["MPix/s"], "unit": "MPix/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main["ms_per_image"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "amf: 1024x1024 RGB AMF-LS, lambda=20, sigma_s=12, sigma_r=0.02 (3 manifolds); "
                                  "amf_deep: sigma_s=16, sigma_r=0.03 (7 manifolds)",
                      "H": H, "W": W, "C": C},
           "roofline": {"kernel": "AMF passes (rows, column scans, carries)", "bound": "hbm",
                        "achieved": main["amf_passes"]["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": main["amf_passes"]["frac"],
                        "traffic": traffic_from_profile("amf_kernels.hip", "amf_passes_rgb1024_pmc.md")},
           "configs": configs,
           "paper_context": {"value": 1.87, "unit": "MPix/s", "note": "Table I: AMF-LS 0.56 s per 1024x1024 RGB "
                             "image (CPU Python with OpenCV's AMF, hardware unstated)"}}
    ref, t = _collect(state)
    if ref is not None:
        refs = np.stack(ref)
        if "amf" in outs:
            out["max_abs_vs_oracle"] = float(np.max(np.abs(outs["amf"] - refs)))
        out["cpu_baseline"] = {"value": round(H * W / t / 1e6, 5), "unit": "MPix/s", "cores": 3, "kind": "oracle",
                               "sample": f"the amf configuration, whole image, 3 channels in 3 worker processes, "
                                         f"{t:.1f} s wall (overlapping the GPU runs)"}
    return out


def _serve(server, blfls, torch, items, gaps_s=None, timeout_s=600.0):
    """Submit items (list of (f, guide, params, out)) with optional arrival gaps; wait for all."""
    pending = {}
    t0 = time.perf_counter()
    next_t = t0
    i = 0
    n = len(items)
    done = 0
    deadline = t0 + timeout_s
    while done < n:
        now = time.perf_counter()
        while i < n and (gaps_s is None or now >= next_t):
            f, g, prm, out = items[i]
            try:
                t, _ = server.submit(f, guide=g, out=out, **prm)
            except blfls.BlflsError as e:
                if e.status == -4:  # queue full: retry later
                    break
                raise
            pending[t] = i
            i += 1
            if gaps_s is not None:
                next_t += gaps_s[i - 1] if i - 1 < len(gaps_s) else 0.0
        for t in list(pending):
            state, status = server.poll(t)
            if state in (blfls.DONE, blfls.FAILED):
                if state == blfls.FAILED or status != 0:
                    raise RuntimeError(f"request {pending[t]} failed with status {status}")
                del pending[t]
                done += 1
        if time.perf_counter() > deadline:
            raise RuntimeError("serving run timed out")
        time.sleep(0.0002)
    return time.perf_counter() - t0


def run_serve(args, torch, blfls, state):
    images = {k: torch.from_numpy(v).cuda() for k, v in state["images"].items()}
    reqs = state["reqs"]
    n = len(reqs)
    outs = [torch.empty_like(images[q["img"]]) for q in reqs]
    items = [(images[q["img"]], None, dict(lam=q["lam"], sigma_s=q["sigma_s"], sigma_r=q["sigma_r"]), outs[i])
             for i, q in enumerate(reqs)]
    mpix = sum(images[q["img"]].shape[1] * images[q["img"]].shape[2] for q in reqs) / 1e6
    arena = 24 << 30
    # closed loop: everything queued at once -> saturation rate
    srv = blfls.Server(arena, max_slots=64, queue_capacity=n + 8, precision="fp32")
    _serve(srv, blfls, torch, items[: min(n, 64)])  # warm-up: plans and kernels
    srv.close()
    srv = blfls.Server(arena, max_slots=64, queue_capacity=n + 8, precision="fp32")
    t_sat = _serve(srv, blfls, torch, items)
    sat_stats = srv.stats()
    srv.close()
    r_sat = n / t_sat
    # open loop at 0.7 of saturation (Poisson arrivals)
    rate = 0.7 * r_sat
    gaps = state["gaps"] / rate
    srv = blfls.Server(arena, max_slots=64, queue_capacity=n + 8, precision="fp32")
    t_open = _serve(srv, blfls, torch, items, gaps_s=gaps)
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    # the plain synchronous FP32 path on the same requests, one after another on one stream
    plans = {}
    for q in reqs[:64]:
        img = images[q["img"]]
        key = tuple(img.shape)
        if key not in plans:
            plans[key] = blfls.Plan(key[1], key[2], key[0], "fp32")
        plans[key].smooth(img, out=outs[0].new_empty(img.shape), lam=q["lam"], sigma_s=q["sigma_s"], sigma_r=q["sigma_r"])
    scratch = {k: torch.empty(k, dtype=torch.float32, device="cuda") for k in plans}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in reqs:
        img = images[q["img"]]
        key = tuple(img.shape)
        plans[key].smooth(img, out=scratch[key], lam=q["lam"], sigma_s=q["sigma_s"], sigma_r=q["sigma_r"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    _submit(state)
    # every result equals the same request run alone
    mismatches = 0
    for i, q in enumerate(reqs):
        alone = blfls.smooth(images[q["img"]], lam=q["lam"], sigma_s=q["sigma_s"], sigma_r=q["sigma_r"])
        if not torch.equal(alone, outs[i]):
            mismatches += 1
    torch.cuda.synchronize()
    out = {"metric": "MPix/s BLF-LS served + p50/p99 latency", "value": round(mpix / t_open, 2), "unit": "MPix/s",
           "n_gpus": 1, "steps": n, "warmup": 64, "ms_per_step": round(1e3 * t_open / n, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"serve: {n} RGB requests, sizes uniform over {[(w, h) for h, w in SERVE_SIZES]} "
                                  "(WxH), lambda~U[5,100], sigma_s in {2,4,8}, sigma_r~U[0.03,0.2], Poisson arrivals "
                                  "at 0.7 x saturation", "requests": n},
           "saturation": {"req_per_s": round(r_sat, 2), "MPix/s": round(mpix / t_sat, 2),
                          "steps": sat_stats["steps"], "graph_steps": sat_stats["graph_steps"],
                          "direct_steps": sat_stats["direct_steps"], "p50_ms": round(sat_stats["latency_p50_ms"], 3),
                          "p99_ms": round(sat_stats["latency_p99_ms"], 3)},
           "open_loop": {"req_per_s_offered": round(rate, 2), "p50_ms": round(st["latency_p50_ms"], 3),
                         "p99_ms": round(st["latency_p99_ms"], 3), "max_ms": round(st["latency_max_ms"], 3),
                         "steps": st["steps"], "graph_steps": st["graph_steps"], "direct_steps": st["direct_steps"],
                         "mean_batch": round(n / max(st["steps"], 1), 2),
                         "arena_peak_GB": round(st["arena_peak"] / 1e9, 3)},
           "sequential_sync_MPix/s": round(mpix / t_seq, 2),
           "alone_vs_mix_bitwise_mismatches": mismatches}
    ref, t = _collect(state)
    if ref is not None:
        errs = []
        for k, i in enumerate(state["oracle_pick"]):
            errs.append(float(np.max(np.abs(outs[i][0].cpu().numpy().astype(np.float64) - ref[k]))))
        out["oracle_sample"] = {"requests": state["oracle_pick"], "channel": 0, "max_abs": max(errs)}
    return out


def run_joint(args, torch, blfls, state):
    pairs = state["pairs"]
    n = len(pairs)
    tg = [(torch.from_numpy(t).cuda(), torch.from_numpy(g).cuda()) for t, g in pairs]
    outs = [torch.empty_like(t) for t, _ in tg]
    prm = dict(lam=30.0, sigma_s=4.0, sigma_r=0.08)
    items = [(t, g, prm, outs[i]) for i, (t, g) in enumerate(tg)]
    arena = 16 << 30
    srv = blfls.Server(arena, max_slots=64, queue_capacity=n + 8, precision="fp16")
    _serve(srv, blfls, torch, items[:8])
    srv.close()
    srv = blfls.Server(arena, max_slots=64, queue_capacity=n + 8, precision="fp16")
    t_run = _serve(srv, blfls, torch, items)
    st = srv.stats()
    srv.close()
    # the same pairs through the synchronous FP16 path, one at a time
    plan = blfls.Plan(2048, 2048, 1, "fp16")
    u = torch.empty_like(tg[0][0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t, g in tg:
        plan.smooth(t, guide=g, out=u, **prm)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    _submit(state)
    mism = 0
    for i, (t, g) in enumerate(tg):
        alone = plan.smooth(t, guide=g, **prm)
        mism += 0 if torch.equal(alone, outs[i]) else 1
    plan.close()
    mpix = n * 2048 * 2048 / 1e6
    out = {"metric": "MPix/s joint BLF-LS served (FP16 fields)", "value": round(mpix / t_run, 2), "unit": "MPix/s",
           "n_gpus": 1, "steps": n, "warmup": 8, "ms_per_step": round(1e3 * t_run / n, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 (fp16 fields)", "data": "synthetic",
           "config": {"workload": f"joint: {n} pairs 2048x2048x1, target = guide + N(0,0.05^2), lambda=30, "
                                  "sigma_s=4 (r=12), sigma_r=0.08, FP16 field storage, served", "pairs": n},
           "served": {"p50_ms": round(st["latency_p50_ms"], 3), "p99_ms": round(st["latency_p99_ms"], 3),
                      "steps": st["steps"], "graph_steps": st["graph_steps"], "direct_steps": st["direct_steps"]},
           "sequential_sync_MPix/s": round(mpix / t_seq, 2),
           "alone_vs_mix_bitwise_mismatches": mism}
    ref, t = _collect(state)
    if ref is not None:
        errs, ps = [], []
        for k in range(len(ref)):
            o = outs[k].cpu().numpy().astype(np.float64)
            errs.append(float(np.max(np.abs(o - ref[k]))))
            ps.append(_psnr(o, ref[k]))
        out["oracle_sample"] = {"pairs": len(ref), "max_abs": max(errs), "min_psnr_db": round(min(ps), 2)}
    return out
