"""Parameter and quality sweeps of the regularisation (Sec. 6, numerical tests).

Everything here runs through the library's kernels; this module only sets
up inputs, times calls with HIP events and tabulates:

* ``table1``: call time over sample counts x iterations at 1024 x 1024,
  radius 8 (the grid of Table 1), with a per-n least-squares line
  ms = fixed + per_iter * iters;
* ``radius_sweep``: the smoothing radius r (the kernel size the paper
  discusses with its parameter choices): time, regularity, overplotting,
  folds of the composite map, trustworthiness and orthogonal ordering, and
  the folds with no background density at all (which larger r reduce);
* ``d0_sweep``: the background density d0 as a multiple of the paper's n/N^2
  (vanishing density is what the paper says makes mapped regions overlap;
  the paper's d0 removes the folds);
* ``res_sweep``: the raster size N (the paper's texture-size parameter k),
  measures taken on one common 1024 x 1024 display raster;
* ``quality_curves``: bin std and overplotting over the iterations, mean
  over random 1-8-cluster data sets at several sample counts (the paper's
  quality curves).

Folds are counted on the composite map of the whole call evaluated at the
texel centres (probe points, inim_regularize_probes): the lattice triangles
whose signed area is not positive.  The neighbourhood measures use the
first ``sample`` samples of the layout (the generators' order is random).
The quality sweeps use random 1-8 Gaussian-cluster data with no uniform
background (the paper's quality ensemble), so that regions of vanishing
density exist; the timings use the benchmark's mixture with outliers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi, datagen, nn, quality

# Table 1: milliseconds per call on a GeForce RTX 2060, 1024 x 1024, r = 8;
# rows 1..8 iterations, columns 0.5M, 1M, 2M, 4M samples (context only).
PAPER_TABLE1_MS = {
    500_000: [1.16, 2.33, 3.56, 4.78, 6.06, 7.34, 8.63, 9.92],
    1_000_000: [1.44, 2.95, 4.51, 6.06, 7.66, 9.30, 10.96, 12.63],
    2_000_000: [1.98, 4.12, 6.33, 8.53, 10.81, 13.16, 15.56, 17.97],
    4_000_000: [3.07, 6.40, 9.89, 13.33, 17.05, 20.81, 24.67, 28.55],
}


def _to(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _median_ms(fn, reset, reps: int) -> float:
    """Median of reps event-timed calls of fn, reset() before each (untimed);
    one extra untimed warm-up call first."""
    out = []
    for rep in range(reps + 1):
        reset()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        if rep:
            out.append(a.elapsed_time(b))
    return float(np.median(out))


def time_call(xy0: torch.Tensor, res: int, iters: int, radius: int = 8, d0=None, reps: int = 10) -> float:
    """Milliseconds of one regularisation call (graph replay), positions
    restored from xy0 before every call."""
    xy = torch.empty_like(xy0)
    ws = capi.workspace(capi.workspace_size(res, xy0.shape[0], radius, d0=d0), xy0.device)
    graph = capi.Graph()
    try:
        ms = _median_ms(lambda: capi.regularize_graph(xy, res, iters, graph, ws, radius=radius, d0=d0),
                        lambda: xy.copy_(xy0), reps)
        capi._check(capi.sync_status(ws))
    finally:
        graph.close()
    return ms


def layout_measures(xy0: torch.Tensor, res: int, iters: int, radius: int = 8, d0=None, display: int | None = None,
                    sample: int = 4096, k: int = 7) -> dict:
    """Regularises a copy of xy0 with texel-centre probes and measures the
    result: regularity and overplotting on the display raster, folds of the
    composite map, trustworthiness and orthogonal ordering of a sample."""
    dev = xy0.device
    display = display or res
    xy = xy0.clone()
    lattice = _to(datagen.lattice_points(res), dev)
    capi.regularize_probes(xy, lattice, res, iters, radius=radius, d0=d0)
    folds = torch.zeros(1, dtype=torch.uint32, device=dev)
    nn.count_folds(lattice, res, folds)
    m = quality.density_measures(xy, display)
    s = min(sample, xy.shape[0])
    a, b = xy0[:s].contiguous(), xy[:s].contiguous()
    return {"bin_std": round(m["bin_std"], 4), "overplotting": round(m["overplotting"], 5),
            "folds": int(folds.item()), "fold_frac": float(folds.item()) / (2 * (res - 1) ** 2),
            "trust": round(quality.trustworthiness(a, b, k), 6), "ordering": round(quality.orthogonal_ordering(a, b), 6)}


def table1(dev, ns=(500_000, 1_000_000, 2_000_000, 4_000_000), iters=range(1, 9), res: int = 1024,
           radius: int = 8, reps: int = 10, seed: int = 0) -> dict:
    iters = list(iters)
    rows = {}
    for n in ns:
        xy0 = _to(datagen.plain_large(seed, n=n), dev)
        ms = [time_call(xy0, res, it, radius, reps=reps) for it in iters]
        slope, fixed = np.polyfit(iters, ms, 1)
        entry = {"ms": [round(t, 4) for t in ms], "per_iter_ms": round(float(slope), 4),
                 "fixed_ms": round(float(fixed), 4)}
        if n in PAPER_TABLE1_MS and iters == list(range(1, 9)):
            entry["paper_rtx2060_ms"] = PAPER_TABLE1_MS[n]
            entry["speedup_vs_paper"] = [round(p / t, 1) for p, t in zip(PAPER_TABLE1_MS[n], ms)]
        rows[str(n)] = entry
        del xy0
    return {"res": res, "radius": radius, "iters": iters, "rows": rows}


def radius_sweep(dev, radii=(1, 2, 4, 8, 16), n: int = 1_000_000, res: int = 1024, iters: int = 8,
                 reps: int = 5, seed: int = 1) -> dict:
    xy0 = _to(datagen.random_clusters(seed, n), dev)
    out = {}
    for r in radii:
        e = layout_measures(xy0, res, iters, radius=r)
        e["folds_without_background"] = layout_measures(xy0, res, iters, radius=r, d0=0.0)["folds"]
        e["ms"] = round(time_call(xy0, res, iters, r, reps=reps), 4)
        out[str(r)] = e
    return {"n": n, "res": res, "iters": iters, "by_radius": out}


def d0_sweep(dev, scales=(0.0, 1e-3, 1e-2, 0.1, 0.5, 1.0, 2.0, 4.0), n: int = 1_000_000, res: int = 1024,
             iters: int = 8, seed: int = 1) -> dict:
    xy0 = _to(datagen.random_clusters(seed, n), dev)
    base = n / (res * res)
    return {"n": n, "res": res, "iters": iters, "d0_unit": base,
            "by_scale": {str(s): layout_measures(xy0, res, iters, d0=s * base) for s in scales}}


def res_sweep(dev, sizes=(256, 512, 1024, 2048, 4096), n: int = 1_000_000, iters: int = 8, radius: int = 8,
              display: int = 1024, reps: int = 5, seed: int = 1) -> dict:
    xy0 = _to(datagen.random_clusters(seed, n), dev)
    out = {}
    for N in sizes:
        e = layout_measures(xy0, N, iters, radius=radius, display=display)
        e["ms"] = round(time_call(xy0, N, iters, radius, reps=reps), 4)
        out[str(N)] = e
    return {"n": n, "iters": iters, "radius": radius, "display": display, "by_res": out}


def quality_curves(dev, ns=(250_000, 1_000_000, 3_000_000), datasets: int = 4, res: int = 1024, iters: int = 8,
                   radius: int = 8) -> dict:
    out = {}
    for n in ns:
        s = np.zeros(iters + 1)
        o = np.zeros(iters + 1)
        ws = capi.workspace(capi.workspace_size(res, n, radius), dev)
        for d in range(datasets):
            xy = _to(datagen.random_clusters(d, n), dev)
            for it in range(iters + 1):
                m = quality.density_measures(xy, res)
                s[it] += m["bin_std"]
                o[it] += m["overplotting"]
                if it < iters:
                    capi.regularize(xy, res, 1, radius=radius, ws=ws)
        out[str(n)] = {"bin_std": [round(v / datasets, 4) for v in s],
                       "overplotting": [round(v / datasets, 5) for v in o]}
    return {"res": res, "datasets": datasets, "by_n": out}


FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X, vector (non-matrix) FP64


def kernel_times(dev, sizes=(4096, 16384), k: int = 7, res: int = 1024, reps: int = 10) -> dict:
    """Event times of the quality kernels on samples of a regularised 1M-sample
    layout.  The neighbourhood kernels are bound by FP64 vector arithmetic:
    trustworthiness needs every sample's squared distance to every other in
    both layouts, 2 n (n - 1) distances of 5 FP64 operations each (2
    differences, 2 products, 1 sum); orthogonal ordering compares
    n (n - 1) / 2 pairs."""
    xy0 = _to(datagen.random_clusters(1, 1_000_000), dev)
    xy = xy0.clone()
    capi.regularize(xy, res, 8)
    counts = quality.texel_counts(xy, res)
    c3 = torch.zeros(3, dtype=torch.int64, device=dev)
    c1 = torch.zeros(1, dtype=torch.int64, device=dev)
    ms = _median_ms(lambda: quality.bin_stats(counts, 4, c3), c3.zero_, reps)
    out = {"bins_1024": {"ms": round(ms, 4), "GBps": round(4 * res * res / ms / 1e6, 1)}}
    for n in sizes:
        a, b = xy0[:n].contiguous(), xy[:n].contiguous()
        t_ord = _median_ms(lambda: quality.ordering_counts(a, b, c3), c3.zero_, reps)
        t_tr = _median_ms(lambda: quality.trust_penalty(a, b, k, c1), c1.zero_, reps)
        flops = 5.0 * n * (n - 1) * 2
        tf = flops / t_tr / 1e9
        out[f"n{n}"] = {"ordering_ms": round(t_ord, 4), "ordering_Gpairs_per_s": round(n * (n - 1) / 2 / t_ord / 1e6, 1),
                        "trust_ms": round(t_tr, 4), "trust_fp64_TFLOPs": round(tf, 2),
                        "trust_frac_fp64_peak": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4)}
    return out


def monotone_decreasing(v) -> bool:
    return all(a > b for a, b in zip(v, v[1:]))


def run_all(dev, quick: bool = False) -> dict:
    """Every sweep; quick=True shrinks them for a test run."""
    if quick:
        return {"table1": table1(dev, ns=(500_000, 1_000_000), iters=(1, 2, 4), reps=3),
                "radius": radius_sweep(dev, radii=(2, 8), n=200_000, res=512, iters=4, reps=2),
                "d0": d0_sweep(dev, scales=(0.0, 0.01, 1.0), n=200_000, res=512, iters=4),
                "res": res_sweep(dev, sizes=(256, 1024), n=200_000, iters=4, reps=2),
                "quality_curves": quality_curves(dev, ns=(250_000,), datasets=2, iters=4)}
    return {"table1": table1(dev), "radius": radius_sweep(dev), "d0": d0_sweep(dev), "res": res_sweep(dev),
            "quality_curves": quality_curves(dev)}


def summary(sw: dict) -> dict:
    """The few numbers worth a line of their own."""
    t = sw["table1"]["rows"]
    out = {"table1_per_iter_ms": {n: r["per_iter_ms"] for n, r in t.items()},
           "table1_ms_8iters": {n: r["ms"][-1] for n, r in t.items()}}
    if "1000000" in t and "speedup_vs_paper" in t["1000000"]:
        out["speedup_vs_paper_1M_8iters"] = t["1000000"]["speedup_vs_paper"][-1]
    curves = sw["quality_curves"]["by_n"]
    out["quality_monotone"] = all(monotone_decreasing(c["bin_std"]) and monotone_decreasing(c["overplotting"])
                                  for c in curves.values())
    out["folds_by_d0_scale"] = {s: e["folds"] for s, e in sw["d0"]["by_scale"].items()}
    out["trust_by_radius"] = {r: e["trust"] for r, e in sw["radius"]["by_radius"].items()}
    return out


__all__ = ["PAPER_TABLE1_MS", "FP64_VECTOR_PEAK_TFLOPS", "kernel_times", "time_call", "layout_measures", "table1", "radius_sweep", "d0_sweep", "res_sweep",
           "quality_curves", "run_all", "summary", "monotone_decreasing"]
