"""Benchmark of the MI355X scatterplot regulariser (one JSON line on stdout).

Headline workload (one step = one whole regularisation call):
  1,000,000 float32 points (8-component Gaussian mixture + 5% uniform
  outliers, seeded), 1024 x 1024 raster, Gaussian radius 8, 8 iterations;
  value = regularisation iterations per second.
Also reported:
  - per-stage times from HIP events recorded by the library on its stream,
    and the roofline of the dominant stage (algorithmic bytes / time);
  - the integral images alone on 8192 x 8192 rasters (uint32 Poisson(4) and
    float32 lognormal, all eight planes): Gpixel/s and GB/s;
  - the FP64 CPU oracle timed on the same workload (cpu_baseline).
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "InIm Gpixel/s (% HBM peak); regularize iters/s at 1M pts; surrogate vs plain speedup"
HBM_PEAK_GBS = 8000.0
PAPER_ITERS_PER_S = 8 / 12.63e-3  # Table 1: 8 iterations, 1M points, 1024^2, r = 8, RTX 2060


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes(n: int, res: int) -> dict:
    """Algorithmic bytes of one launch of each per-iteration stage (what the method must move)."""
    px = res * res
    return {
        "smooth_aggregate": 4 * px + 4 * px + 4 * px,  # read counts, write density, clear next counts
        "inim_deform": 4 * px + 8 * px,                # read the density, write the 2-channel field
        "advect_splat": 16 * n + 8 * px + 4 * px,      # read + write xy, read the field, next counts
    }


def bench_regularize(args, dev):
    import numpy as np
    import torch

    from paper_2408_06513_amd import capi, datagen

    n, res, iters, radius = args.n, args.res, args.iters, 8
    log(f"generating {n} points")
    xy0_np = datagen.plain_large(0, n=n)
    xy0 = torch.from_numpy(xy0_np).to(dev)
    xy = torch.empty_like(xy0)
    ws = capi.workspace(capi.workspace_size(res, n, radius), dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        xy.copy_(xy0)
        capi.regularize(xy, res, iters, radius=radius, ws=ws, check=False)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert capi.sync_status(ws) == capi.OK
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert capi.sync_status(ws) == capi.OK
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = iters * args.steps / (t1 - t0)

    # the same steps through a captured HIP graph of the whole call
    graph = capi.Graph()

    def gstep():
        xy.copy_(xy0)
        capi.regularize_graph(xy, res, iters, graph, ws)

    for _ in range(max(1, args.warmup)):
        gstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gstep()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert capi.sync_status(ws) == capi.OK
    graph_value = iters * args.steps / (t1 - t0)
    graph.close()

    # per-stage HIP events (same stream), separate pass so the headline is unperturbed
    log("stage timing")
    acc = {k: 0.0 for k in capi.STAGES}
    reps = max(3, min(args.steps, 10))
    for _ in range(reps):
        xy.copy_(xy0)
        ms = capi.regularize_timed(xy, res, iters, radius=radius, ws=ws)
        for k, v in ms.items():
            acc[k] += v
    stage_us = {k: 1e3 * v / (reps * iters) for k, v in acc.items() if k not in ("total", "sort_unsort")}
    stage_us["sort_unsort_per_call"] = 1e3 * acc["sort_unsort"] / reps
    stage_us["total_per_iter"] = 1e3 * acc["total"] / (reps * iters)
    sb = stage_bytes(n, res)
    dom = max(sb, key=lambda k: stage_us[k])
    t_dom = stage_us[dom] * 1e-6
    achieved = sb[dom] / t_dom / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "bytes_per_launch": sb[dom], "launch_us": round(stage_us[dom], 3)}
    return xy0_np, value, ms_per_step, stage_us, roofline, graph_value


def bench_inim(dev, res: int = 8192, reps: int = 20) -> dict:
    import numpy as np
    import torch

    from paper_2408_06513_amd import capi, datagen

    out = {}
    # evicting the 256 MB last-level cache between calls by reading 512 MB
    # (a read leaves no dirty lines whose write-back would land in the timing)
    flush = torch.ones(128 << 20, dtype=torch.float32, device=dev)
    for name, img_np in (("u32", datagen.poisson_raster(0, res)), ("f32", datagen.lognormal_raster(0, res))):
        log(f"inim {name} {res}^2")
        img = torch.from_numpy(img_np).to(dev)
        dt = capi.U32 if name == "u32" else capi.F32
        ws = capi.workspace(capi.inim_workspace_size(res, dt), dev)
        planes = torch.empty((8, res, res), dtype=img.dtype, device=dev)
        marg = torch.empty(6 * res - 1, dtype=torch.float64, device=dev)
        for _ in range(3):
            capi.inim(img, 0xFF, planes=planes, marg=marg, ws=ws)
        times = []
        for _ in range(reps):
            flush.sum()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            capi.inim(img, 0xFF, planes=planes, marg=marg, ws=ws)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) * 1e-3)
        t = float(np.median(times))
        alg = 36 * res * res
        out[name] = {"gpix_per_s": round(res * res / t / 1e9, 2), "ms": round(t * 1e3, 4),
                     "alg_GBps": round(alg / t / 1e9, 1), "frac_hbm": round(alg / t / 1e9 / HBM_PEAK_GBS, 4)}
        del img, ws, planes
    return out


def cpu_baseline(xy0_np, res: int, iters: int, budget_s: float) -> dict:
    import oracle
    log("cpu baseline (oracle)")
    done, t = 0, 0.0
    while t < budget_s:
        t0 = time.perf_counter()
        oracle.regularize(xy0_np, res, iters)
        t += time.perf_counter() - t0
        done += iters
    return {"value": round(done / t, 4), "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"full workload ({xy0_np.shape[0]} points, {res}^2, r=8), {done} iterations "
                      f"({done // iters} regularisations of {iters}), single thread, FP64",
            "host": os.uname().nodename}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=8)
    ap.add_argument("--no-inim", action="store_true", help="skip the 8192^2 integral-image measurement")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--only-inim", action="store_true",
                    help="print only the 8192^2 integral-image measurement (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding note in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    from paper_2408_06513_amd import capi
    capi.lib()

    if args.only_inim:
        print(json.dumps({"inim_8192_all_planes": bench_inim(dev)}), flush=True)
        return
    xy0_np, value, ms_per_step, stage_us, roofline, graph_value = bench_regularize(args, dev)
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / PAPER_ITERS_PER_S, 2),
        "baseline_note": "paper Table 1 (RTX 2060): 8 iterations of 1M points at 1024^2, r=8 in 12.63 ms",
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"regularize {args.n} points (8-component Gaussian mixture + 5% uniform "
                               f"outliers), {args.res}x{args.res} raster, r=8, {args.iters} iterations",
                   "n": args.n, "res": args.res, "iters": args.iters, "radius": 8},
        "roofline": roofline,
        "stages_us_per_iter": {k: round(v, 3) for k, v in stage_us.items()},
        "graph_replay_iters_per_s": round(graph_value, 2),
    }
    if not args.no_inim:
        rec["inim_8192_all_planes"] = bench_inim(dev)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(xy0_np, args.res, args.iters, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
