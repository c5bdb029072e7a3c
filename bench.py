"""Benchmark of the MI355X scatterplot regulariser (one JSON line on stdout).

Headline workload (one step = one whole regularisation call):
  1,000,000 float32 points (8-component Gaussian mixture + 5% uniform
  outliers, seeded), 1024 x 1024 raster, Gaussian radius 8, 8 iterations;
  value = regularisation iterations per second.
Also reported:
  - per-stage times from HIP events recorded by the library on its stream,
    and the roofline of the dominant stage (algorithmic bytes / time);
  - the same call through a captured HIP graph, and with the 1024 x 1024
    texel lattice moved along as probe points (composite map output);
  - a 45-plot scatterplot matrix (200,000 samples x 10 dims, rasters of
    256/512/1024, 6 iterations) in one batched call against 45 single calls;
  - the learned surrogate of the 256 x 256 method with its network at
    64 x 64, and with the network on the full 256 x 256 raster (both trained
    here by the project's kernels), against the method on held-out point
    sets, eager, as graph replays and batched;
  - the integral images alone on 8192 x 8192 rasters (uint32 Poisson(4) and
    float32 lognormal; all eight planes, and alpha + alpha_t with the
    marginals): Gpixel/s and GB/s, median with 10th and 90th percentiles;
  - parameter and quality sweeps: Table 1's grid (0.5-4M points x 1-8
    iterations), the radius r, the background d0 and the raster size with
    regularity, overplotting, folds, trustworthiness and orthogonal ordering,
    and the quality curves over the iterations;
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


# HBM traffic per launch of the per-iteration stages' kernels from two rocprofv3
# --pmc runs of `bench.py --profile-short` (FETCH_SIZE, then WRITE_SIZE; see
# profiles/pmc_traffic_regularize_1M_1024.md), each scaled by what the same
# counter reads for a plain 256 MiB device copy in that run (FETCH_SIZE
# counts half of the bytes read: factor 1.99982; WRITE_SIZE all: factor 1.000).
# Valid only for the sources they were taken with: SHA-256 over the files
# that hold the kernels (k_inim.hip, k_raster.hip) and every header;
# otherwise traffic is null.
TRAFFIC = {
    "src_sha256": "64c654500b4bb1210459632f574d9f3c7931fa8c2009f5394c13f32fe3f89fe4",
    # k_blur_aggregate: FETCH_SIZE 4129.1 KiB x 1.99982 + WRITE_SIZE 10112.0 KiB x 1.000
    "smooth_aggregate": 18810324,
    # k_inim_deform16x2: FETCH_SIZE 7840.1 KiB x 1.99982 + WRITE_SIZE 8192.0 KiB x 1.000
    "inim_deform": 24443688,
    # k_advect (1M samples): FETCH_SIZE 18650.1 KiB x 1.99982 + WRITE_SIZE 15536.7 KiB x 1.000
    "advect_splat": 54101548,
}


def kernel_sources_sha256() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2408_06513_amd", "csrc")
    files = [os.path.join(csrc, "k_inim.hip"), os.path.join(csrc, "k_raster.hip")] + glob.glob(os.path.join(csrc, "*.h"))
    for f in sorted(files):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stage: str):
    if TRAFFIC.get("src_sha256") != kernel_sources_sha256():
        return None
    return TRAFFIC.get(stage)


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes(n: int, res: int) -> dict:
    """Algorithmic bytes of one launch of each per-iteration stage (what the
    method must move).  The carry scans between the aggregate and the final
    pass move only scratch partial sums: no algorithmic bytes."""
    px = res * res
    return {
        "smooth_aggregate": 4 * px + 4 * px + 4 * px,  # read counts, write density, clear next counts
        "inim_scans": 0,                               # band carries (scratch only)
        "inim_deform": 4 * px + 8 * px,                # read the density, write the 2-channel field
        "advect_splat": 16 * n + 8 * px + 4 * px,      # read + write xy, read the field, next counts
    }


# The kernel the roofline field reports: the longest per-iteration kernel of
# the headline workload in the committed rocprofv3 kernel trace
# (profiles/regularize_1M_1024_kernels.md: k_advect).  Fixed rather than
# picked per run from event timings, where the stages lie within a few
# percent of each other and the pick would flip between runs.
ROOFLINE_STAGE = "advect_splat"


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

    # the same steps also moving the res x res texel lattice as probe points
    # (the composite map of all iterations on the lattice)
    lat0 = torch.from_numpy(datagen.lattice_points(res)).to(dev)
    lat = torch.empty_like(lat0)

    def pstep():
        xy.copy_(xy0)
        lat.copy_(lat0)
        capi.regularize_probes(xy, lat, res, iters, radius=radius, ws=ws, check=False)

    for _ in range(max(1, args.warmup)):
        pstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pstep()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert capi.sync_status(ws) == capi.OK
    probe_value = iters * args.steps / (t1 - t0)

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
    per_stage = {}
    for k, b in sb.items():
        t = stage_us[k] * 1e-6
        per_stage[k] = {"us": round(stage_us[k], 3), "bytes_per_launch": b,
                        "achieved_GBps": round(b / t / 1e9, 2), "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(k)}
    dom = ROOFLINE_STAGE
    achieved = per_stage[dom]["achieved_GBps"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom), "kernel": dom,
                "bytes_per_launch": sb[dom], "launch_us": round(stage_us[dom], 3), "stages": per_stage}

    # the small configuration (20,000 points, 256^2, 4 iterations) as a
    # graph replay, for the oracle's time on it
    c1 = datagen.plain_small(0)
    c1_0 = torch.from_numpy(c1).to(dev)
    c1_xy = torch.empty_like(c1_0)
    c1_ws = capi.workspace(capi.workspace_size(256, c1.shape[0], radius), dev)
    c1_graph = capi.Graph()
    c1_times = []
    for rep in range(21):
        c1_xy.copy_(c1_0)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        capi.regularize_graph(c1_xy, 256, 4, c1_graph, c1_ws)
        b.record()
        torch.cuda.synchronize()
        if rep:
            c1_times.append(a.elapsed_time(b))
    assert capi.sync_status(c1_ws) == capi.OK
    c1_graph.close()
    small = {"n": int(c1.shape[0]), "res": 256, "iters": 4, "ms_per_call": round(float(np.median(c1_times)), 4)}
    return xy0_np, value, ms_per_step, stage_us, roofline, graph_value, probe_value, small


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
        # all eight planes: 4 B read + 8 x 4 B written per texel; alpha and
        # alpha_t with the marginals: 4 + 2 x 4 (the marginals are 0.05 MB)
        for tag, mask, bpp in (("all", capi.MASK_ALL, 36), ("min", capi.MASK_MIN, 12)):
            for _ in range(3):
                capi.inim(img, mask, planes=planes, marg=marg, ws=ws)
            times = []
            for _ in range(reps):
                flush.sum()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                capi.inim(img, mask, planes=planes, marg=marg, ws=ws)
                b.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) * 1e-3)
            t = float(np.median(times))
            p10, p90 = (float(v) for v in np.percentile(times, [10, 90]))
            alg = bpp * res * res
            out[f"{name}_{tag}"] = {"gpix_per_s": round(res * res / t / 1e9, 2), "ms": round(t * 1e3, 4),
                                    "ms_p10": round(p10 * 1e3, 4), "ms_p90": round(p90 * 1e3, 4),
                                    "alg_GBps": round(alg / t / 1e9, 1),
                                    "frac_hbm": round(alg / t / 1e9 / HBM_PEAK_GBS, 4)}
        del img, ws, planes
    return out


def profile_short(args, dev):
    """A short run for rocprofv3 --pmc: each kernel of interest a few times
    (a 256 MiB device copy, the calibration of the byte counters; one
    regularisation of the headline workload; one 8192^2 integral-image call
    of each type with all planes and with alpha + alpha_t)."""
    import torch

    from paper_2408_06513_amd import capi, datagen
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)  # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    dst.copy_(src)  # the calibration copy: 256 MiB read, 256 MiB written
    torch.cuda.synchronize()
    del src, dst
    xy0 = torch.from_numpy(datagen.plain_large(0, n=args.n)).to(dev)
    ws = capi.workspace(capi.workspace_size(args.res, args.n, 8), dev)
    capi.regularize(xy0.clone(), args.res, args.iters, radius=8, ws=ws)
    torch.cuda.synchronize()
    res = 8192
    for dt, img_np in ((capi.U32, datagen.poisson_raster(0, res)), (capi.F32, datagen.lognormal_raster(0, res))):
        img = torch.from_numpy(img_np).to(dev)
        wsi = capi.workspace(capi.inim_workspace_size(res, dt), dev)
        planes = torch.empty((8, res, res), dtype=img.dtype, device=dev)
        capi.inim(img, 0xFF, planes=planes, ws=wsi)
        torch.cuda.synchronize()
        capi.inim(img, 0x11, planes=planes[:2], ws=wsi)  # alpha + alpha_t (float: summed in double)
        torch.cuda.synchronize()
        del img, wsi, planes
    print(json.dumps({"profile_short": "done", "n": args.n, "res": args.res, "iters": args.iters}), flush=True)


def bench_splom(dev, reps: int = 5) -> dict:
    """Scatterplot matrix: 200,000 samples x 10 dims, all 45 pairwise plots
    at raster sizes drawn from 256/512/1024, 6 iterations each; one batched
    call (plain launches, autotuned shape, captured graph) against 45
    inim_regularize calls.  Times from events around the calls only."""
    import numpy as np
    import torch

    from paper_2408_06513_amd import capi, datagen
    iters = 6
    log("splom: 45 plots")
    plots = datagen.splom_plots(0)
    src = [torch.from_numpy(xy).to(dev) for xy, _ in plots]
    res = [r for _, r in plots]
    xs = [torch.empty_like(s) for s in src]
    ws = capi.workspace(capi.batch_workspace_size(xs, res), dev)
    wss = [capi.workspace(capi.workspace_size(r, s.shape[0]), dev) for s, r in zip(src, res)]

    def timed(fn):
        out = []
        for rep in range(reps + 1):
            for x, s in zip(xs, src):
                x.copy_(s)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            if rep:
                out.append(a.elapsed_time(b))
        return float(np.median(out))

    def seq():
        for x, r, w in zip(xs, res, wss):
            capi.regularize(x, r, iters, ws=w, check=False)

    t_seq = timed(seq)
    t_def = timed(lambda: capi.regularize_batch(xs, res, iters, ws=ws, check=False))
    cfg, _ = capi.batch_autotune(xs, res, iters, ws=ws)
    t_tuned = timed(lambda: capi.regularize_batch(xs, res, iters, cfg=cfg, ws=ws, check=False))
    graph = capi.Graph()
    t_graph = timed(lambda: capi.regularize_batch(xs, res, iters, cfg=cfg, ws=ws, graph=graph, check=False))
    graph.close()
    assert capi.sync_status(ws) == capi.OK
    best = min(t_def, t_tuned, t_graph)
    return {"plots": len(plots), "samples_per_plot": int(src[0].shape[0]), "iters": iters,
            "sizes": {str(s): res.count(s) for s in sorted(set(res))},
            "sequential_ms": round(t_seq, 3), "batched_ms": round(t_def, 3), "batched_tuned_ms": round(t_tuned, 3),
            "batched_tuned_graph_ms": round(t_graph, 3), "tuned_config": repr(cfg),
            "speedup_vs_sequential": round(t_seq / best, 2)}


def bench_surrogate(dev, train_sets: int = 50000, steps: int = 10000, held_out: int = 16, batch: int = 16,
                    workers: int = 16, save_dir: str | None = None, full_field: bool = False,
                    train: bool = False) -> dict:
    """The learned surrogate of the 256 x 256, 8-iteration regularisation: a
    5-level U-Net (32-256 channels) reading the 256 x 256 density raster and
    the displacement of the method's first iteration on it (whose integral
    images carry the whole raster's mass, which 3 x 3 convolutions over five
    levels do not reach), predicting the displacement of all eight.
    Two output lattices are trained on the same sets with the same budget:
    the displacement on the 64 x 64 lattice (decoder up to level 2, the
    configuration in use) and on the full 256 x 256 lattice.  Training sets
    are point sets of 2-12 Gaussian components (10k-500k points) drawn by
    worker processes and labelled by the method itself (its composite map at
    the lattice's texel centres).  On held-out sets: uniformity, folds, gate
    decisions (the gate asks for no folded triangle and a 4 x 4-bin standard
    deviation at most the method's worst 8-to-1-iteration ratio (x 1.05)
    times the one after the method's own first step on the same set,
    calibrated on fresh training-distribution sets), and times per raster -- single and batched,
    ungated and gated -- against the method, also at equal final uniformity
    (the method's time at the fractional iteration count whose bin std equals
    the surrogate's).
    Without `train`, the 64 x 64 variant is the committed checkpoint
    (surrogate.C5_WEIGHTS, trained this way) and nothing is trained."""
    import numpy as np
    import torch

    from paper_2408_06513_amd import capi, datagen
    from paper_2408_06513_amd import surrogate as S
    res, iters, net_res = 256, 8, 256
    full_field = full_field and train
    sets, t_data = None, None
    if train:
        log(f"surrogate: {train_sets} training sets, labels on the 64^2 and 256^2 lattices")
        t0 = time.perf_counter()
        sets = S.dataset_compact(range(train_sets), res, iters, dev, net_res=net_res,
                                 out_levels=(2, 0) if full_field else (2,), workers=workers, log=log,
                                 first_step=True)
        t_data = time.perf_counter() - t0
    seeds = list(range(100_000, 100_000 + held_out))

    def ev_time(fn, reps=5):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # the method on the held-out sets: bin std after 0..8 iterations and the
    # graph-replayed time of 1..8 iterations, per raster
    xs0 = [torch.from_numpy(datagen.surrogate_mixture(s)).to(dev) for s in seeds]
    bs_k = np.zeros(iters + 1)
    t_k = np.zeros(iters + 1)
    for x0 in xs0:
        xy = x0.clone()
        bs_k[0] += S.bin_std(xy, res)
        ws = capi.workspace(capi.workspace_size(res, xy.shape[0]), dev)
        for k in range(1, iters + 1):
            graph = capi.Graph()
            t_k[k] += ev_time(lambda: (xy.copy_(x0), capi.regularize_graph(xy, res, k, graph, ws)))
            graph.close()
            xy.copy_(x0)
            capi.regularize(xy, res, k, ws=ws)
            bs_k[k] += S.bin_std(xy, res)
    bs_k /= len(xs0)
    t_k /= len(xs0)
    ratio = S.calibrate_gate(res, iters, dev)

    def at_equal_uniformity(bs):
        """The method's time per raster at the fractional iteration count
        where its mean bin std equals bs (capped at the full count)."""
        for k in range(1, iters + 1):
            if bs_k[k] <= bs:
                f = (bs_k[k - 1] - bs) / max(bs_k[k - 1] - bs_k[k], 1e-12)
                tk0 = t_k[k - 1] if k > 1 else 0.0
                return (k - 1) + f, tk0 + f * (t_k[k] - tk0)
        return float(iters), float(t_k[iters])

    def run_variant(out_level: int) -> dict:
        if not train:
            net = S.UNet.load(S.C5_WEIGHTS, dev)
            assert net.out_level == out_level and net.first_step
            log(f"surrogate (field {net_res >> out_level}^2): committed checkpoint, {net.t} steps")
            losses, t_train = None, None
        else:
            net = S.UNet(dev, seed=0, out_level=out_level, first_step=True)
            log(f"surrogate (field {net_res >> out_level}^2): {steps} steps x {batch}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            losses = S.train(net, sets[out_level], None, steps=steps, batch=batch, lr=1e-3)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
        if save_dir and train:
            os.makedirs(save_dir, exist_ok=True)
            net.save(os.path.join(save_dir, f"surrogate_256_field{net_res >> out_level}.npz"), optimizer=False)
        ev = S.evaluate(net, seeds, res, iters, dev, net_res=net_res, ratio=ratio)
        sur_bs = float(np.mean([r["surrogate"] for r in ev["rows"]]))
        # per raster, single: the method's graph, the surrogate's graph (ungated), the gated call
        plain, sur, gated, gated_eager = [], [], [], []
        for x0 in xs0:
            xy = x0.clone()
            ws = capi.workspace(capi.workspace_size(res, xy.shape[0]), dev)
            graph = capi.Graph()
            plain.append(ev_time(lambda: (xy.copy_(x0), capi.regularize_graph(xy, res, iters, graph, ws))))
            graph.close()
            sg = S.SurrogateGraph(net, xy.shape[0], res, net_res, xy=xy)
            sur.append(ev_time(lambda: (xy.copy_(x0), sg())))
            del sg
            gated_eager.append(ev_time(lambda: (xy.copy_(x0), S.regularize(net, xy, res, iters, net_res=net_res,
                                                                             ratio=ratio)), 3))
            gg = S.SurrogateGatedGraph(net, xy, res, iters, net_res=net_res, ratio=ratio)
            gated.append(ev_time(lambda: (xy.copy_(x0), gg()), 5))
            del gg
        # batched over the held-out sets
        xs = [x.clone() for x in xs0]

        def reset():
            for x, x0 in zip(xs, xs0):
                x.copy_(x0)
        sgm = S.SurrogateManyGraph(net, xs, res, net_res)
        t_b_sur = ev_time(lambda: (reset(), sgm()), 3) / len(xs)
        del sgm
        wsb = capi.workspace(capi.batch_workspace_size(xs, [res] * len(xs)), dev)
        cfg, _ = capi.batch_autotune(xs, [res] * len(xs), iters, ws=wsb)
        bgraph = capi.Graph()
        t_b_plain = ev_time(lambda: (reset(), capi.regularize_batch(xs, [res] * len(xs), iters, cfg=cfg, ws=wsb,
                                                                    graph=bgraph, check=False)), 3) / len(xs)
        bgraph.close()
        reset()
        dec = S.regularize_many_gated(net, xs, res, iters, net_res=net_res, ws_batch=wsb, ratio=ratio)
        bs_gated = float(np.mean([S.bin_std(x, res) for x in xs]))
        t_b_gated = ev_time(lambda: (reset(), S.regularize_many_gated(net, xs, res, iters, net_res=net_res,
                                                                      ws_batch=wsb, ratio=ratio)), 3) / len(xs)
        k_eq, t_eq = at_equal_uniformity(sur_bs)
        mean = lambda v: float(np.mean(v))
        rec = {"field_res": net_res >> out_level,
               "network": "trained in this run" if train else "committed checkpoint (weights/surrogate_256_field64.npz)",
               "train_steps": steps if train else net.t,
               "batch": batch if train else S.C5_TRAINING["batch"],
               "train_s": round(t_train, 1) if train else None,
               "loss_first10": round(mean(losses[:10]), 4) if train else None,
               "loss_last10": round(mean(losses[-10:]), 4) if train else None,
               "explained_variance": round(ev["explained"], 4),
               "bin_std_gain_plain": round(ev["plain_gain"], 4), "bin_std_gain_surrogate": round(ev["surrogate_gain"], 4),
               "folded_triangles": ev["folds"], "gate_ratio_to_first_step": round(ratio, 4),
               "gate_fallbacks": ev["fallbacks"], "gate_fallbacks_batched": dec.count("fallback"),
               "accepted_short_of_method": ev["accepted_short_of_method"],
               "bin_std_final_gated_batched": round(bs_gated, 3),
               "plain_graph_ms_per_raster": round(mean(plain), 4),
               "surrogate_graph_ms_per_raster": round(mean(sur), 4),
               "surrogate_gated_ms_per_raster": round(mean(gated), 4),
               "surrogate_gated_eager_ms_per_raster": round(mean(gated_eager), 4),
               f"plain_batched_graph_ms_per_raster_batch{held_out}": round(t_b_plain, 4),
               f"surrogate_batched_graph_ms_per_raster_batch{held_out}": round(t_b_sur, 4),
               f"surrogate_gated_batched_ms_per_raster_batch{held_out}": round(t_b_gated, 4),
               "equal_uniformity": {"surrogate_bin_std": round(sur_bs, 3), "method_iterations": round(k_eq, 2),
                                    "method_ms_per_raster": round(t_eq, 4)}}
        rec["speedup_vs_plain_gated"] = round(rec["plain_graph_ms_per_raster"] / rec["surrogate_gated_ms_per_raster"], 3)
        rec["speedup_vs_plain_ungated"] = round(rec["plain_graph_ms_per_raster"] / rec["surrogate_graph_ms_per_raster"], 3)
        rec[f"speedup_vs_plain_gated_batch{held_out}"] = round(t_b_plain / t_b_gated, 3)
        rec["speedup_at_equal_uniformity_ungated"] = round(t_eq / rec["surrogate_graph_ms_per_raster"], 3)
        del net
        return rec

    out = {"res": res, "net_input": net_res, "iters": iters,
           "train_sets": train_sets if train else S.C5_TRAINING["train_sets"], "held_out": held_out,
           "data_s": round(t_data, 1) if train else None, "workers": workers if train else None,
           "method_bin_std_by_iteration": [round(v, 3) for v in bs_k],
           "method_graph_ms_by_iteration": [round(v, 4) for v in t_k]}
    out["field64"] = run_variant(2)
    if full_field:
        out["field256"] = run_variant(0)
    del sets
    return out


def bench_convs(dev, imgs: int = 16, res: int = 256, reps: int = 10) -> dict:
    """Every convolution of the surrogate's network (256 x 256 input, decoder
    to level 2) at the training batch: forward, input gradient and weight
    gradient timed separately with events (median), in TFLOP/s of their
    2 P Cin Cout ks^2 multiply-adds and as a fraction of the 2.5 PFLOP/s
    dense BF16 matrix-core peak."""
    import numpy as np
    import torch

    from paper_2408_06513_amd import nn
    from paper_2408_06513_amd import surrogate as S
    g = torch.Generator(device="cpu").manual_seed(0)
    work = torch.empty(256, dtype=torch.uint8, device=dev)
    rows, tot = {}, {"fwd": [0.0, 0.0], "dgrad": [0.0, 0.0], "wgrad": [0.0, 0.0]}
    shapes = S.conv_shapes(out_level=2)
    lvl_of = lambda name: 2 if name == "head" else int(name[1])  # noqa: E731
    for name, cin, cout, ks in shapes:
        h = res >> lvl_of(name)
        x = (torch.rand((imgs, h, h, cin), generator=g) - 0.5).to(torch.bfloat16).to(dev)
        w = (torch.rand((cout, ks * ks, cin), generator=g) - 0.5).to(torch.bfloat16).to(dev)
        wT = torch.empty((cin, ks * ks, cout), dtype=torch.bfloat16, device=dev)
        nn.weight_transpose(w, wT)
        dy = (torch.rand((imgs, h, h, cout), generator=g) - 0.5).to(torch.bfloat16).to(dev)
        y16 = torch.empty((imgs, h, h, cout), dtype=torch.bfloat16, device=dev)
        dx = torch.empty((imgs, h, h, cin), dtype=torch.float32, device=dev)
        dw = torch.empty((cout, ks * ks, cin), dtype=torch.float32, device=dev)
        db = torch.empty(cout, dtype=torch.float32, device=dev)
        need = nn.conv_workspace(imgs, h, h, cin, cout, ks)
        if work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=dev)
        flop = 2.0 * imgs * h * h * cin * cout * ks * ks
        rec = {"h": h, "cin": cin, "cout": cout, "ks": ks, "gflop": round(flop / 1e9, 3)}
        for tag, fn in (("fwd", lambda: nn.conv_forward(x, w, None, True, y16=y16, work=work)),
                        ("dgrad", lambda: nn.conv_backward_data(dy, wT, dx, work=work)),
                        ("wgrad", lambda: nn.conv_backward_weight(dy, x, ks, dw, db, work=work))):
            fn()
            ts = []
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b) * 1e-3)
            t = float(np.median(ts))
            rec[f"{tag}_us"] = round(t * 1e6, 1)
            rec[f"{tag}_TFLOPs"] = round(flop / t / 1e12, 1)
            tot[tag][0] += flop
            tot[tag][1] += t
        rows[name] = rec
    out = {"imgs": imgs, "res": res, "layers": rows}
    for tag, (f, t) in tot.items():
        out[f"{tag}_total_TFLOPs"] = round(f / t / 1e12, 1)
        out[f"{tag}_frac_bf16_peak"] = round(f / t / 1e12 / 2500.0, 4)
        out[f"{tag}_total_ms"] = round(t * 1e3, 3)
    return out


def hbm_calibration(dev, mib: int = 1024, reps: int = 10) -> dict:
    """What the device sustains for plain streams (torch's own copy and fill
    kernels on buffers far larger than the 256 MB last-level cache): the
    context for the roofline fractions, which are taken against the 8 TB/s
    peak."""
    import numpy as np
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    flush = torch.empty(2 * n, dtype=torch.float32, device=dev)

    def timed(fn):
        out = []
        for rep in range(reps + 1):
            flush.fill_(1.0)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            if rep:
                out.append(a.elapsed_time(b) * 1e-3)
        return float(np.median(out))
    t_copy = timed(lambda: dst.copy_(src))
    t_fill = timed(lambda: dst.fill_(2.0))
    t_read = timed(lambda: src.sum())
    nb = n * 4
    out = {"buffer_MiB": mib, "copy_TBps": round(2 * nb / t_copy / 1e12, 3), "write_TBps": round(nb / t_fill / 1e12, 3),
           "read_TBps": round(nb / t_read / 1e12, 3)}
    out["copy_frac_of_peak"] = round(out["copy_TBps"] * 1000 / HBM_PEAK_GBS, 4)
    del src, dst, flush
    return out


def bench_sweeps(dev) -> dict:
    """Parameter and quality sweeps (Table 1's grid of sample counts x
    iterations; radius, background density and raster size with quality,
    fold and neighbourhood measures; the quality curves over iterations)."""
    from paper_2408_06513_amd import sweeps
    t0 = time.time()
    log("sweeps: Table 1 grid, r, d0, N, quality curves")
    sw = sweeps.run_all(dev)
    sw["summary"] = sweeps.summary(sw)
    sw["quality_kernels"] = sweeps.kernel_times(dev)
    sw["seconds"] = round(time.time() - t0, 1)
    log(f"sweeps: {sw['summary']}")
    return sw


def host_cpu() -> dict:
    """The host the oracle runs on: logical CPUs, the CPUs this process may
    use, and the model name."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model,
            "node": os.uname().nodename}


def oracle_threads_all() -> int:
    """All the threads this process should use: OMP_NUM_THREADS when set
    (the CPU share of the machine), else every CPU of its affinity mask."""
    aff = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(aff, int(env))) if env.isdigit() else aff


def cpu_baseline(xy0_np, res: int, iters: int, budget_s: float, gpu_ms: dict) -> dict:
    """The FP64 oracle timed on the host: the headline workload (bounded to
    about budget_s of work per thread count), the small configuration, and the
    8192^2 integral images, each on one thread and on all threads."""
    import numpy as np

    import oracle
    from paper_2408_06513_amd import datagen
    host = host_cpu()
    T = oracle_threads_all()
    log(f"cpu baseline (oracle), 1 and {T} threads, host {host}")

    def regularize_rate(k, budget):
        oracle.set_threads(k)
        done, t = 0, 0.0
        while t < budget:
            t0 = time.perf_counter()
            oracle.regularize(xy0_np, res, iters)
            t += time.perf_counter() - t0
            done += iters
        return done / t, done

    def once(k, fn, reps=1):
        oracle.set_threads(k)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    r1, n1 = regularize_rate(1, budget_s)
    rT, nT = regularize_rate(T, max(2.0, budget_s / 2))
    c1 = datagen.plain_small(0).astype(np.float64)
    c1_1 = once(1, lambda: oracle.regularize(c1, 256, 4), 3)
    c1_T = once(T, lambda: oracle.regularize(c1, 256, 4), 3)
    img = datagen.poisson_raster(0, 8192).astype(np.float64)
    c3 = {}
    for tag, mask in (("all", oracle.MASK_ALL), ("min", oracle.MASK_MIN)):
        t1 = once(1, lambda: oracle.planes(img, mask))
        tT = once(T, lambda: oracle.planes(img, mask))
        g = gpu_ms.get(f"inim_u32_{tag}")
        c3[tag] = {"s_1_thread": round(t1, 3), f"s_{T}_threads": round(tT, 3),
                   "gpu_ms": g, "gpu_speedup_vs_all_threads": round(tT * 1e3 / g, 1) if g else None}
    del img
    oracle.set_threads(1)
    g2 = gpu_ms.get("regularize_call")
    g1 = gpu_ms.get("small_call")
    return {"value": round(rT, 4), "unit": "iterations/s", "cores": T, "kind": "oracle",
            "sample": f"full workload ({xy0_np.shape[0]} points, {res}^2, r=8): {nT} iterations "
                      f"({nT // iters} regularisations of {iters}) on {T} threads; FP64",
            "single_thread": {"value": round(r1, 4), "unit": "iterations/s",
                              "sample": f"{n1} iterations ({n1 // iters} regularisations of {iters}), 1 thread"},
            "gpu_speedup_vs_all_threads": round(iters / (g2 * 1e-3) / rT, 1) if g2 else None,
            "small_config": {"n": int(c1.shape[0]), "res": 256, "iters": 4, "s_1_thread": round(c1_1, 4),
                             f"s_{T}_threads": round(c1_T, 4), "gpu_ms": g1,
                             "gpu_speedup_vs_all_threads": round(c1_T * 1e3 / g1, 1) if g1 else None},
            "inim_8192_u32": c3, "host": host}


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
    ap.add_argument("--no-splom", action="store_true", help="skip the 45-plot scatterplot-matrix measurement")
    ap.add_argument("--no-surrogate", action="store_true", help="skip training and timing the learned surrogate")
    ap.add_argument("--surrogate-train", action="store_true",
                    help="train the surrogate in the run (default: time the committed checkpoint)")
    ap.add_argument("--surrogate-sets", type=int, default=50000, help="training point sets of the surrogate")
    ap.add_argument("--surrogate-save", default=None, help="directory for the trained networks (.npz checkpoints)")
    ap.add_argument("--only-surrogate", action="store_true", help="print only the surrogate measurement")
    ap.add_argument("--surrogate-full-field", action="store_true",
                    help="also train and measure the network with the full 256 x 256 output lattice")
    ap.add_argument("--only-convs", action="store_true", help="print only the per-convolution matrix-core rates")
    ap.add_argument("--surrogate-steps", type=int, default=10000, help="training steps of the surrogate")
    ap.add_argument("--no-sweeps", action="store_true", help="skip the parameter and quality sweeps")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--only-sweeps", action="store_true",
                    help="print only the parameter and quality sweeps (for profiling)")
    ap.add_argument("--only-inim", action="store_true",
                    help="print only the 8192^2 integral-image measurement (for profiling)")
    ap.add_argument("--profile-short", action="store_true",
                    help="for counter collection: one 256 MiB device copy (the calibration of the byte "
                         "counters), one regularisation of the headline workload and one 8192^2 "
                         "integral-image call of each type; prints one line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    from paper_2408_06513_amd import capi
    capi.lib()

    if args.only_inim:
        print(json.dumps({"inim_8192": bench_inim(dev), "hbm_calibration": hbm_calibration(dev)}),
              flush=True)
        return
    if args.profile_short:
        profile_short(args, dev)
        return
    if args.only_convs:
        print(json.dumps({"surrogate_convs": bench_convs(dev)}), flush=True)
        return
    if args.only_surrogate:
        print(json.dumps({"surrogate_256": bench_surrogate(dev, args.surrogate_sets, args.surrogate_steps,
                                                           save_dir=args.surrogate_save,
                                                           full_field=args.surrogate_full_field,
                                                           train=args.surrogate_train)}), flush=True)
        return
    if args.only_sweeps:
        print(json.dumps({"sweeps": bench_sweeps(dev)}), flush=True)
        return
    xy0_np, value, ms_per_step, stage_us, roofline, graph_value, probe_value, small = bench_regularize(args, dev)
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
        "with_lattice_probes_iters_per_s": round(probe_value, 2),
        "small_config": small,
    }
    if not args.no_inim:
        rec["inim_8192"] = bench_inim(dev)
        rec["hbm_calibration"] = hbm_calibration(dev)
    if not args.no_splom:
        rec["splom_45_plots"] = bench_splom(dev)
    if not args.no_surrogate:
        rec["surrogate_256"] = bench_surrogate(dev, args.surrogate_sets, args.surrogate_steps,
                                               save_dir=args.surrogate_save, full_field=args.surrogate_full_field,
                                               train=args.surrogate_train)
        rec["surrogate_convs"] = bench_convs(dev)
    if not args.no_sweeps:
        rec["sweeps"] = bench_sweeps(dev)
    if not args.no_cpu:
        gpu_ms = {"regularize_call": ms_per_step, "small_call": small["ms_per_call"]}
        for tag in ("all", "min"):
            if "inim_8192" in rec:
                gpu_ms[f"inim_u32_{tag}"] = rec["inim_8192"][f"u32_{tag}"]["ms"]
        rec["cpu_baseline"] = cpu_baseline(xy0_np, args.res, args.iters, args.cpu_seconds, gpu_ms)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
