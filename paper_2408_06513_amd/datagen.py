"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random inputs; it holds none of the regularisation's
arithmetic (no splat, blur, integral image, map or interpolation).  Every value
is drawn in float64 from ``numpy.random.Generator(PCG64(seed))`` and cast to
its storage type once, so the oracle and the HIP path read identical bytes.

The workloads stand in for the paper's synthetic experiments (Sec. 6, the
clustered test sets of the quality measures and Table 1's 1024x1024 setting);
the paper's real data sets (MNIST embeddings, COIL, UCI) are not used.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "gaussian_mixture",
    "plain_small",
    "plain_large",
    "random_clusters",
    "four_clusters",
    "diagonal_line",
    "poisson_raster",
    "lognormal_raster",
    "lattice_points",
    "splom_table",
    "splom_plots",
    "surrogate_mixture",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _rotated_gaussian(g: np.random.Generator, n: int, mean, stds, theta) -> np.ndarray:
    """n draws of an anisotropic 2D Gaussian rotated by theta, rejection-resampled
    until every point lies in the closed unit square."""
    c, s = np.cos(theta), np.sin(theta)
    rot = np.array([[c, -s], [s, c]])
    out = np.empty((0, 2))
    while out.shape[0] < n:
        m = n - out.shape[0]
        z = g.standard_normal((max(m * 2, 16), 2)) * np.asarray(stds)[None, :]
        p = z @ rot.T + np.asarray(mean)[None, :]
        keep = np.all((p >= 0.0) & (p <= 1.0), axis=1)
        out = np.concatenate([out, p[keep][:m]], axis=0)
    return out


def gaussian_mixture(seed: int, counts, mean_lo: float, mean_hi: float,
                     std_lo: float, std_hi: float, outliers: int = 0) -> np.ndarray:
    """Mixture with exact per-component counts, random means, axis stds and
    rotations, plus ``outliers`` uniform points; rows are shuffled."""
    g = rng(seed)
    parts = []
    for cnt in counts:
        mean = g.uniform(mean_lo, mean_hi, size=2)
        stds = g.uniform(std_lo, std_hi, size=2)
        theta = g.uniform(0.0, np.pi)
        parts.append(_rotated_gaussian(g, int(cnt), mean, stds, theta))
    if outliers:
        parts.append(g.uniform(0.0, 1.0, size=(outliers, 2)))
    pts = np.concatenate(parts, axis=0)
    pts = pts[g.permutation(pts.shape[0])]
    return np.ascontiguousarray(pts.astype(np.float32))


def plain_small(seed: int = 0) -> np.ndarray:
    """20,000 points: 3 components with 10k/6k/4k points (weights .5/.3/.2),
    means U[.25,.75]^2, axis stds U[.02,.15], random rotation."""
    return gaussian_mixture(seed, [10_000, 6_000, 4_000], 0.25, 0.75, 0.02, 0.15)


def _dirichlet_counts(g: np.random.Generator, total: int, k: int) -> list[int]:
    w = g.dirichlet(np.ones(k))
    cnt = np.floor(w * total).astype(np.int64)
    cnt[np.argmax(w)] += total - int(cnt.sum())
    return [int(c) for c in cnt]


def plain_large(seed: int = 0, n: int = 1_000_000) -> np.ndarray:
    """n points: 95% from 8 components (Dirichlet(1) weights, means U[.15,.85]^2,
    stds U[.01,.1], random rotation) plus 5% uniform outliers."""
    g = rng(10_000 + seed)
    n_out = n // 20
    counts = _dirichlet_counts(g, n - n_out, 8)
    return gaussian_mixture(20_000 + seed, counts, 0.15, 0.85, 0.01, 0.10, outliers=n_out)


def random_clusters(seed: int, n: int, k: int | None = None) -> np.ndarray:
    """1..8 variable-sized Gaussian clusters at random locations (the ensemble
    behind the paper's bin-std / overplotting curves)."""
    g = rng(30_000 + seed)
    if k is None:
        k = int(g.integers(1, 9))
    counts = _dirichlet_counts(g, n, k)
    return gaussian_mixture(40_000 + seed, counts, 0.15, 0.85, 0.01, 0.12)


def four_clusters(seed: int = 0, scale: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Four clusters with 4:3:2:1 sizes (400k/300k/200k/100k at scale=1000);
    returns points and their cluster labels (unshuffled label order)."""
    g = rng(50_000 + seed)
    sizes = [400 * scale, 300 * scale, 200 * scale, 100 * scale]
    pts, lab = [], []
    for c, m in enumerate(sizes):
        mean = g.uniform(0.2, 0.8, size=2)
        stds = g.uniform(0.02, 0.08, size=2)
        theta = g.uniform(0.0, np.pi)
        pts.append(_rotated_gaussian(g, m, mean, stds, theta))
        lab.append(np.full(m, c, dtype=np.int32))
    return (np.ascontiguousarray(np.concatenate(pts).astype(np.float32)),
            np.concatenate(lab))


def diagonal_line(seed: int, n: int, jitter: float = 0.002) -> np.ndarray:
    """Points along the main diagonal with a small perpendicular jitter."""
    g = rng(60_000 + seed)
    t = g.uniform(0.05, 0.95, size=n)
    e = g.normal(0.0, jitter, size=n)
    p = np.stack([t + e, t - e], axis=1)
    return np.ascontiguousarray(np.clip(p, 0.0, 1.0).astype(np.float32))


def poisson_raster(seed: int, res: int, lam: float = 4.0) -> np.ndarray:
    """res x res uint32 counts, i.i.d. Poisson(lam)."""
    return np.ascontiguousarray(rng(70_000 + seed).poisson(lam, size=(res, res)).astype(np.uint32))


def lognormal_raster(seed: int, res: int, sigma: float = 1.0) -> np.ndarray:
    """res x res float32 values, i.i.d. lognormal(0, sigma)."""
    return np.ascontiguousarray(rng(80_000 + seed).lognormal(0.0, sigma, size=(res, res)).astype(np.float32))


def lattice_points(res: int, repeat: int = 1) -> np.ndarray:
    """One point (or ``repeat`` points) at every texel centre of a res x res raster."""
    c = (np.arange(res, dtype=np.float64) + 0.5) / res
    xx, yy = np.meshgrid(c, c, indexing="xy")
    p = np.stack([xx.ravel(), yy.ravel()], axis=1)
    if repeat > 1:
        p = np.repeat(p, repeat, axis=0)
    return np.ascontiguousarray(p.astype(np.float32))


def splom_table(seed: int = 0, n: int = 200_000, dims: int = 10) -> np.ndarray:
    """n x dims table: dims 0..6 correlated Gaussian, the rest a 4-cluster
    mixture with shared labels; each column min-max normalised to [0, 1]."""
    g = rng(90_000 + seed)
    k = min(7, dims)
    a = g.standard_normal((k, k))
    cov = a @ a.T + 0.1 * np.eye(k)
    dsd = np.sqrt(np.diag(cov))
    corr = cov / dsd[:, None] / dsd[None, :]
    cols = [g.multivariate_normal(np.zeros(k), corr, size=n)]
    if dims > k:
        lab = g.integers(0, 4, size=n)
        centres = g.uniform(-3, 3, size=(4, dims - k))
        cols.append(centres[lab] + 0.4 * g.standard_normal((n, dims - k)))
    t = np.concatenate(cols, axis=1)
    lo, hi = t.min(axis=0), t.max(axis=0)
    t = (t - lo) / (hi - lo)
    return np.ascontiguousarray(np.clip(t, 0.0, 1.0).astype(np.float32))


def splom_plots(seed: int = 0, n: int = 200_000, dims: int = 10, sizes=(256, 512, 1024)):
    """All dims*(dims-1)/2 pairwise plots of splom_table: a list of
    (xy float32 [n, 2] = columns (a, b), raster size drawn from `sizes`)."""
    t = splom_table(seed, n, dims)
    g = rng(91_000 + seed)
    out = []
    for a in range(dims):
        for b in range(a + 1, dims):
            res = int(g.choice(np.asarray(sizes)))
            out.append((np.ascontiguousarray(t[:, [a, b]]), res))
    return out


def surrogate_mixture(seed: int, n_lo: int = 10_000, n_hi: int = 500_000) -> np.ndarray:
    """A training or held-out input of the learned surrogate: K ~ U{2..12}
    Gaussian components (the small-configuration shapes: means U[.15,.85]^2,
    axis stds U[.02,.15], random rotations, Dirichlet(1) sizes) and
    n ~ log-uniform[n_lo, n_hi] points."""
    g = rng(100_000 + seed)
    k = int(g.integers(2, 13))
    n = int(np.exp(g.uniform(np.log(n_lo), np.log(n_hi))))
    counts = _dirichlet_counts(g, n, k)
    return gaussian_mixture(110_000 + seed, [c for c in counts if c > 0], 0.15, 0.85, 0.02, 0.15)
