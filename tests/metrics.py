"""Quality measures used as test and benchmark instruments (Sec. 6 of the paper).

bin_std      standard deviation of per-bin sample counts, 4x4-pixel bins.
overplotting (n - number of occupied pixels) / n.
grid_folds   orientation and monotonicity checks of a deformed texel lattice.
"""
from __future__ import annotations

import numpy as np


def _pixels(xy: np.ndarray, res: int) -> tuple[np.ndarray, np.ndarray]:
    xy = np.asarray(xy, dtype=np.float64)
    i = np.minimum(np.floor(xy[:, 0] * res).astype(np.int64), res - 1)
    j = np.minimum(np.floor(xy[:, 1] * res).astype(np.int64), res - 1)
    return i, j


def bin_std(xy: np.ndarray, res: int, bin_px: int = 4) -> float:
    i, j = _pixels(xy, res)
    nb = res // bin_px
    h = np.bincount((j // bin_px) * nb + (i // bin_px), minlength=nb * nb)
    return float(np.std(h.astype(np.float64)))


def overplotting(xy: np.ndarray, res: int) -> float:
    i, j = _pixels(xy, res)
    occ = np.unique(j * res + i).size
    n = xy.shape[0]
    return float((n - occ) / n)


def grid_folds(grid: np.ndarray) -> dict:
    """grid: [N, N, 2] positions of the texel lattice (row j, column i).
    Counts cells with non-positive orientation and lattice edges that break
    x-monotonicity along rows or y-monotonicity along columns."""
    g = np.asarray(grid, dtype=np.float64)
    a = g[:-1, :-1]
    b = g[:-1, 1:]
    c = g[1:, :-1]
    e1 = b - a
    e2 = c - a
    cross = e1[..., 0] * e2[..., 1] - e1[..., 1] * e2[..., 0]
    # second triangle of each cell
    d = g[1:, 1:]
    f1 = c - d
    f2 = b - d
    cross2 = f1[..., 0] * f2[..., 1] - f1[..., 1] * f2[..., 0]
    return {
        "nonpos_cells": int(np.sum(cross <= 0) + np.sum(cross2 <= 0)),
        "x_nonmono": int(np.sum(np.diff(g[..., 0], axis=1) <= 0)),
        "y_nonmono": int(np.sum(np.diff(g[..., 1], axis=0) <= 0)),
    }
