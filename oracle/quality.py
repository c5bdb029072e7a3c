"""FP64 CPU oracle of the layout quality measures of Sec. 6 (numerical tests).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this; the library's product path never does.

Positions are ``[n, 2]`` arrays (x, y) in the unit square, FLOAT32 VALUES
(the precision the regularisation produces); every measure is written out
from its definition:

* the sample counts per texel of an N x N display raster, a sample going to
  texel min(floor(x N), N - 1) with x N rounded in float32 (the splat of
  Sec. 4.1);
* the regularity measure: the standard deviation of the per-bin sample
  counts over bin x bin texel blocks (4 x 4 in the paper) about their mean;
* overplotting: (samples - occupied texels) / samples;
* trustworthiness (Venna and Kaski) with k output-space neighbours;
* orthogonal ordering (Misue et al.): the share of sample pairs whose
  left/right and above/below relation is the same before and after.

Readings where the paper names a measure without defining it:
* the bin standard deviation is the population one (divided by the number of
  bins, not one less);
* the neighbour order of a sample i sorts the others by squared Euclidean
  distance in float64, ``dx*dx + dy*dy`` with every operation rounded
  (dx = x_j - x_i of the float32 values taken as float64), ties by index, so
  ranks are unique;
* orthogonal ordering compares the signs (-1, 0, +1) of x_j - x_i and of
  y_j - y_i; a pair counts as kept along an axis when the sign is unchanged,
  and the measure is the share of unordered pairs kept along both axes.
"""
from __future__ import annotations

import numpy as np


def texel_counts(xy, res: int) -> np.ndarray:
    """[res, res] int64 counts, indexed [row (y), column (x)]."""
    p = np.asarray(xy, dtype=np.float32)
    t = np.minimum(np.floor(p * np.float32(res)), np.float32(res - 1)).astype(np.int64)
    counts = np.zeros((res, res), dtype=np.int64)
    np.add.at(counts, (t[:, 1], t[:, 0]), 1)
    return counts


def bin_stats(counts: np.ndarray, bin_px: int) -> tuple[int, int, int]:
    """(occupied texels, sum of bin counts, sum of squared bin counts)."""
    res = counts.shape[0]
    nb = res // bin_px
    bins = counts.reshape(nb, bin_px, nb, bin_px).sum(axis=(1, 3))
    return int((counts > 0).sum()), int(bins.sum()), int((bins * bins).sum())


def bin_std(xy, res: int, bin_px: int = 4) -> float:
    """Standard deviation of the per-bin sample counts about their mean."""
    _, s1, s2 = bin_stats(texel_counts(xy, res), bin_px)
    nbins = (res // bin_px) ** 2
    mean = s1 / nbins
    return float(np.sqrt(max(s2 / nbins - mean * mean, 0.0)))


def overplotting(xy, res: int) -> float:
    """(samples - occupied texels) / samples."""
    n = len(xy)
    occupied = int((texel_counts(xy, res) > 0).sum())
    return (n - occupied) / n


def _sq_dist_from(p: np.ndarray, i: int) -> np.ndarray:
    d = p - p[i]
    return d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]


def _neighbour_order(p: np.ndarray, i: int) -> np.ndarray:
    """The other samples sorted by squared distance to sample i, ties by index."""
    others = np.delete(np.arange(len(p)), i)
    d = _sq_dist_from(p, i)[others]
    return others[np.lexsort((others, d))]


def trust_penalty(a, b, k: int) -> int:
    """Sum over samples i of (r(i, j) - k) over the j that are among the k
    nearest neighbours of i after the mapping (b) but not before (a), with
    r(i, j) the rank of j in the order before (1 = nearest)."""
    A = np.asarray(a, dtype=np.float32).astype(np.float64)
    B = np.asarray(b, dtype=np.float32).astype(np.float64)
    n = len(A)
    total = 0
    for i in range(n):
        rank_a = np.empty(n, dtype=np.int64)
        rank_a[_neighbour_order(A, i)] = np.arange(1, n)
        for j in _neighbour_order(B, i)[:k]:
            if rank_a[j] > k:
                total += int(rank_a[j]) - k
    return total


def trustworthiness(a, b, k: int) -> float:
    """1 - 2 / (n k (2n - 3k - 1)) * trust_penalty; 1 when every output
    neighbourhood was already a neighbourhood of the input."""
    n = len(a)
    return 1.0 - 2.0 * trust_penalty(a, b, k) / (n * k * (2 * n - 3 * k - 1))


def ordering_counts(a, b) -> tuple[int, int, int]:
    """Unordered pairs kept along x, along y, along both."""
    A = np.asarray(a, dtype=np.float32)
    B = np.asarray(b, dtype=np.float32)
    n = len(A)
    upper = np.triu(np.ones((n, n), dtype=bool), 1)

    def sign(v):
        return (v[None, :] > v[:, None]).astype(np.int8) - (v[None, :] < v[:, None]).astype(np.int8)

    kx = (sign(A[:, 0]) == sign(B[:, 0])) & upper
    ky = (sign(A[:, 1]) == sign(B[:, 1])) & upper
    return int(kx.sum()), int(ky.sum()), int((kx & ky).sum())


def orthogonal_ordering(a, b) -> float:
    n = len(a)
    return ordering_counts(a, b)[2] / (n * (n - 1) // 2)
