"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each check is independent of the oracle's own code path: brute force over the
printed inequalities (Sec. 3.1), a hand-worked example of eq. (map) and
eq. (map_res) (tests/golden/map_2x2.txt), closed forms for the constant raster,
textbook summed-area tables, a library convolution with the same border rule,
and the paper's stated properties (identity on a constant density, Sec. 4.2;
convex combination, Sec. 5; monotone, fold-free deformation; decreasing
bin-std and overplotting, Sec. 6).
"""
from __future__ import annotations

import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2408_06513_amd import datagen as dg
from tests import metrics

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- brute force
def brute_planes(d: np.ndarray) -> np.ndarray:
    """All eight planes by evaluating the printed inequalities of Sec. 3.1 for
    every (pixel, pixel') pair: O(N^4)."""
    N = d.shape[0]
    r = np.arange(N)
    # axes: [j, i, j', i']
    J, I, Jp, Ip = np.meshgrid(r, r, r, r, indexing="ij")
    D = d[Jp, Ip]
    conds = [
        (Ip <= I) & (Jp <= J),
        (Ip <= I) & (Jp > J),
        (Ip > I) & (Jp > J),
        (Ip > I) & (Jp <= J),
        (Ip + Jp <= I + J) & (Ip - Jp >= I - J),
        (Ip + Jp <= I + J) & (Ip - Jp < I - J),
        (Ip + Jp > I + J) & (Ip - Jp < I - J),
        (Ip + Jp > I + J) & (Ip - Jp >= I - J),
    ]
    return np.stack([np.where(c, D, 0.0).sum(axis=(2, 3)) for c in conds])


def brute_marg(d: np.ndarray) -> dict:
    N = d.shape[0]
    J, I = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    X = np.array([d[I <= i].sum() for i in range(N)])
    Y = np.array([d[J <= j].sum() for j in range(N)])
    U = np.array([d[I + J <= u].sum() for u in range(2 * N - 1)])
    V = np.array([d[I - J >= v].sum() for v in range(-(N - 1), N)])
    return {"X": X, "Y": Y, "U": U, "V": V, "C": d.sum()}


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_planes_match_brute_force_integers(N):
    d = dg.rng(N).integers(0, 9, size=(N, N)).astype(np.float64)
    P, m = oracle.planes(d)
    B = brute_planes(d)
    assert np.array_equal(P, B)
    bm = brute_marg(d)
    for k in "XYUV":
        assert np.array_equal(m[k], bm[k]), k
    assert m["C"] == bm["C"]


@pytest.mark.parametrize("N", [2, 4, 16])
def test_planes_match_brute_force_floats(N):
    d = dg.rng(100 + N).lognormal(0.0, 1.0, size=(N, N))
    P, _ = oracle.planes(d)
    B = brute_planes(d)
    np.testing.assert_allclose(P, B, rtol=1e-12, atol=0)


def test_mask_selects_planes_in_bit_order():
    d = dg.rng(5).integers(0, 5, size=(8, 8)).astype(np.float64)
    full, _ = oracle.planes(d, oracle.MASK_ALL)
    sub, _ = oracle.planes(d, 0b10100110)
    assert np.array_equal(sub, full[[1, 2, 5, 7]])


@pytest.mark.parametrize("N", [4, 64, 256])
def test_partitions_and_corner(N):
    """alpha+beta+gamma+delta = C and alpha_t+...+delta_t = C at every pixel
    (Sec. 3.1); alpha at the last pixel is C; exact for integer data."""
    d = dg.poisson_raster(1, N).astype(np.float64)
    P, m = oracle.planes(d)
    C = m["C"]
    assert np.all(P[0] + P[1] + P[2] + P[3] == C)
    assert np.all(P[4] + P[5] + P[6] + P[7] == C)
    assert P[0][-1, -1] == C == d.sum()
    assert np.array_equal(P[0][-1, :], m["X"]) and np.array_equal(P[0][:, -1], m["Y"])


@pytest.mark.parametrize("N", [8, 128])
def test_alpha_is_summed_area_table(N):
    d = dg.poisson_raster(2, N).astype(np.float64)
    P, _ = oracle.planes(d, 0x01)
    assert np.array_equal(P[0], np.cumsum(np.cumsum(d, axis=0), axis=1))


def lienhart_rotated_sat(d: np.ndarray) -> np.ndarray:
    """Rotated summed-area table by Lienhart's recurrence
    RSAT(i,j) = RSAT(i-1,j-1) + RSAT(i+1,j-1) - RSAT(i,j-2) + d(i,j) + d(i,j-1)
    on a zero-padded grid widened by N+1 columns on each side (integer data)."""
    N = d.shape[0]
    pad = N + 1
    W = N + 2 * pad
    dd = np.zeros((N, W), dtype=np.int64)
    dd[:, pad:pad + N] = d
    R = np.zeros((N + 2, W), dtype=np.int64)  # row index j+2
    for j in range(N):
        for i in range(W):
            left = R[j + 1, i - 1] if i >= 1 else 0
            right = R[j + 1, i + 1] if i + 1 < W else 0
            v = left + right - R[j, i] + dd[j, i] + (dd[j - 1, i] if j >= 1 else 0)
            R[j + 2, i] = v
    return R[2:, pad:pad + N]


@pytest.mark.parametrize("N", [4, 32])
def test_alpha_t_matches_lienhart_recurrence(N):
    d = dg.poisson_raster(3, N).astype(np.int64)
    P, _ = oracle.planes(d.astype(np.float64), 0x10)
    assert np.array_equal(P[0].astype(np.int64), lienhart_rotated_sat(d))


def ones_closed_forms(N: int) -> np.ndarray:
    """Planes of the all-ones raster, counted combinatorially."""
    J, I = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    alpha = (I + 1) * (J + 1)
    beta = (I + 1) * (N - 1 - J)
    gamma = (N - 1 - I) * (N - 1 - J)
    delta = (N - 1 - I) * (J + 1)
    m = J + 1

    def F(K):
        return K * m - K * (K + 1) // 2

    alpha_t = m + F(np.minimum(I, m)) + F(np.minimum(N - 1 - I, m))
    u = I + J
    v = I - J
    U = np.where(u <= N - 1, (u + 1) * (u + 2) // 2, N * N - (2 * N - 2 - u) * (2 * N - 1 - u) // 2)
    V = np.where(v >= 0, (N - v) * (N - v + 1) // 2, N * N - (N + v - 1) * (N + v) // 2)
    beta_t = U - alpha_t
    delta_t = V - alpha_t
    gamma_t = N * N - U - V + alpha_t
    return np.stack([alpha, beta, gamma, delta, alpha_t, beta_t, gamma_t, delta_t]).astype(np.float64)


@pytest.mark.parametrize("N", [2, 4, 16, 128, 512])
def test_constant_raster_closed_forms(N):
    P, m = oracle.planes(np.ones((N, N)))
    assert np.array_equal(P, ones_closed_forms(N))
    assert m["C"] == N * N


# ---------------------------------------------------------------- golden map
def load_golden():
    rows = []
    d = None
    with open(os.path.join(HERE, "golden", "map_2x2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("d "):
                d = np.array([float(t) for t in line.split()[1:]]).reshape(2, 2)
                continue
            rows.append([float(t) for t in line.split()])
    return d, np.array(rows)


def test_golden_hand_worked_planes_and_map():
    d, rows = load_golden()
    P, _ = oracle.planes(d)
    t = oracle.tmap(d)
    t1 = oracle.tmap(np.ones((2, 2)))
    T = oracle.deform(d, 0.0)
    for r in rows:
        i, j = int(r[0]), int(r[1])
        assert np.array_equal(P[:, j, i], r[2:10])
        np.testing.assert_allclose(t[j, i], r[10:12], rtol=0, atol=1e-15)
        np.testing.assert_allclose(t1[j, i], r[12:14], rtol=0, atol=1e-15)
        np.testing.assert_allclose(T[j, i], r[14:16], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- map properties
@pytest.mark.parametrize("N", [2, 16, 64])
def test_constant_density_is_identity(N):
    """eq. (map_res) is the identity for a constant density (Sec. 4.2)."""
    for d0 in (0.25, 3.0):
        T = oracle.deform(np.zeros((N, N)), d0)
        c = (np.arange(N) + 0.5) / N
        np.testing.assert_allclose(T[..., 0], np.broadcast_to(c[None, :], (N, N)), rtol=0, atol=1e-13)
        np.testing.assert_allclose(T[..., 1], np.broadcast_to(c[:, None], (N, N)), rtol=0, atol=1e-13)


def test_map_is_convex_combination_and_scale_invariant():
    """t(p;d) lies in the unit square (non-negative weights on boundary points,
    Sec. 5) and scaling d by a power of two leaves it bit-identical."""
    d = dg.rng(9).lognormal(0.0, 1.5, size=(32, 32))
    t = oracle.tmap(d)
    assert t.min() >= 0.0 and t.max() <= 1.0
    assert np.array_equal(t, oracle.tmap(d * 8.0))
    assert np.array_equal(oracle.deform(d, 0.5), oracle.deform(d * 4.0, 2.0))


def test_background_density_damps_displacement():
    """eq. (map) is a ratio of functionals linear in d, so with d = d_r + d0
    (eq. (d0)) the displacement of eq. (map_res) is that of d_r alone scaled
    by C_r / (C_r + N^2 d0): doubling the background shrinks it by a known
    factor, and a huge background makes the map the identity."""
    N = 16
    dr = dg.rng(3).lognormal(0.0, 1.0, size=(N, N))
    Cr = dr.sum()
    c = (np.arange(N) + 0.5) / N
    P = np.stack(np.broadcast_arrays(c[None, :], c[:, None]), axis=-1)
    d1 = oracle.deform(dr, 0.5) - P
    d2 = oracle.deform(dr, 1.0) - P
    np.testing.assert_allclose(d2, d1 * (Cr + N * N * 0.5) / (Cr + N * N * 1.0), rtol=1e-10, atol=1e-15)
    assert np.abs(oracle.deform(dr, 1e12) - P).max() < 1e-9


def test_map_of_spike_pushes_neighbourhood_away():
    """A single heavy pixel expands its surroundings: texels left of it are
    displaced to the left and texels right of it to the right (Sec. 3.2)."""
    N = 32
    d = np.zeros((N, N))
    d[16, 16] = 1000.0
    T = oracle.deform(d, 1.0)
    c = (np.arange(N) + 0.5) / N
    disp = T[..., 0] - c[None, :]
    assert disp[16, 8] < 0 < disp[16, 24]


# ---------------------------------------------------------------- splat, blur
def test_counts_brute_force_and_edges():
    xy = np.array([[0.0, 0.0], [1.0, 1.0], [0.5, 0.5], [0.49999, 0.5], [0.25, 1.0]])
    c = oracle.counts(xy, 4)
    exp = np.zeros((4, 4))
    for x, y in xy:
        exp[min(int(np.floor(y * 4)), 3), min(int(np.floor(x * 4)), 3)] += 1
    assert np.array_equal(c, exp)
    assert c[0, 0] == 1 and c[3, 3] == 1 and c[2, 2] == 1 and c[2, 1] == 1 and c[3, 1] == 1
    xy = dg.plain_small(0)
    c = oracle.counts(xy, 256)
    assert c.sum() == xy.shape[0]
    h, _, _ = np.histogram2d(xy[:, 1].astype(np.float64), xy[:, 0].astype(np.float64),
                             bins=256, range=[[0, 1], [0, 1]])
    assert np.array_equal(c, h)


def gaussian_taps(r: int, sigma: float) -> np.ndarray:
    m = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-m * m / (2 * sigma * sigma))
    return g / g.sum()


@pytest.mark.parametrize("N,r", [(64, 8), (32, 3), (16, 1)])
def test_blur_matches_library_reflect_convolution(N, r):
    c = dg.poisson_raster(4, N).astype(np.float64)
    g = gaussian_taps(r, r / 2)
    ref = ndimage.correlate1d(ndimage.correlate1d(c, g, axis=1, mode="reflect"), g, axis=0, mode="reflect")
    np.testing.assert_allclose(oracle.blur(c, r), ref, rtol=1e-13, atol=1e-12)


def test_blur_wide_kernel_on_small_raster():
    """r larger than N: the half-sample symmetric extension repeats (numpy's
    'symmetric' padding)."""
    N, r = 4, 8
    c = dg.poisson_raster(5, N).astype(np.float64)
    g = gaussian_taps(r, 2.5)
    p = np.pad(c, r, mode="symmetric")
    tmp = sum(g[k] * p[:, k:k + N] for k in range(2 * r + 1))
    ref = sum(g[k] * tmp[k:k + N, :] for k in range(2 * r + 1))
    np.testing.assert_allclose(oracle.blur(c, r, 2.5), ref, rtol=1e-13, atol=1e-12)


def test_blur_conserves_mass_and_constants():
    c = dg.poisson_raster(6, 128).astype(np.float64)
    assert abs(oracle.blur(c, 8).sum() - c.sum()) < 1e-8 * c.sum()
    np.testing.assert_allclose(oracle.blur(np.full((32, 32), 3.0), 8), 3.0, rtol=1e-14)
    assert np.array_equal(oracle.blur(c, 0), c)


# ---------------------------------------------------------------- advect
def test_advect_reproduces_affine_field_exactly():
    """Bilinear interpolation with linear extrapolation at the border reproduces
    an affine field, so samples move by exactly the affine map."""
    N = 16
    c = (np.arange(N) + 0.5) / N
    X, Y = np.meshgrid(c, c, indexing="xy")
    A = np.array([[0.75, 0.125], [-0.0625, 0.5]])
    b = np.array([0.125, 0.25])
    field = np.stack([A[0, 0] * X + A[0, 1] * Y + b[0], A[1, 0] * X + A[1, 1] * Y + b[1]], axis=-1)
    xy = dg.rng(7).uniform(0, 1, size=(1000, 2))
    out = oracle.advect(field, xy)
    np.testing.assert_allclose(out, np.clip(xy @ A.T + b, 0, 1), rtol=0, atol=1e-14)


def test_advect_identity_field_and_clamp():
    N = 8
    c = (np.arange(N) + 0.5) / N
    X, Y = np.meshgrid(c, c, indexing="xy")
    ident = np.stack([X, Y], axis=-1)
    xy = np.array([[0.0, 0.0], [1.0, 1.0], [0.3, 0.9]])
    np.testing.assert_allclose(oracle.advect(ident, xy), xy, rtol=0, atol=1e-15)
    out = oracle.advect(ident * 2.0, xy)
    assert out.max() == 1.0 and out.min() >= 0.0


# ---------------------------------------------------------------- errors
def test_errors():
    xy = np.array([[0.5, 0.5]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.regularize(xy, 3, 1)
    assert e.value.status == oracle.EINVAL
    bad = np.array([[0.5, 0.5], [np.nan, 0.1]])
    st, out = oracle.regularize_status(bad, 8, 2)
    assert st == oracle.EDOMAIN
    assert np.array_equal(out[0], bad[0]) and np.isnan(out[1, 0])
    st, _ = oracle.regularize_status(np.array([[1.5, 0.5]]), 8, 2)
    assert st == oracle.EDOMAIN
    assert oracle.regularize(np.zeros((0, 2)), 8, 3).shape == (0, 2)


# ---------------------------------------------------------------- whole iteration
def test_duplicated_samples_give_identical_positions():
    """Doubling every sample doubles counts, d_r and d0 = n/N^2, so d doubles
    and t is unchanged (scale invariance): positions are bit-identical."""
    xy = dg.plain_small(0)[:5000]
    a = oracle.regularize(xy, 128, 3)
    b = oracle.regularize(np.repeat(xy, 2, axis=0), 128, 3)
    assert np.array_equal(np.repeat(a, 2, axis=0), b)


def test_permutation_equivariance():
    xy = dg.plain_small(1)[:4000]
    perm = dg.rng(11).permutation(xy.shape[0])
    a = oracle.regularize(xy, 64, 3)
    b = oracle.regularize(xy[perm], 64, 3)
    assert np.array_equal(a[perm], b)


@pytest.mark.parametrize("N", [16, 64])
def test_uniform_lattice_is_fixed_point(N):
    xy = dg.lattice_points(N)
    out = oracle.regularize(xy, N, 3)
    np.testing.assert_allclose(out, xy.astype(np.float64), rtol=0, atol=1e-12)


def iterate_with_grid(xy, N, iters, r=8):
    """Runs the oracle step by step, carrying the texel lattice along (it adds
    no density); returns positions, grids and quality after each iteration."""
    xy = np.asarray(xy, np.float64).copy()
    n = xy.shape[0]
    d0 = n / N / N
    grid = dg.lattice_points(N).astype(np.float64)
    out = []
    for _ in range(iters):
        dr = oracle.blur(oracle.counts(xy, N), r)
        T = oracle.deform(dr, d0)
        xy = oracle.advect(T, xy)
        grid = oracle.advect(T, grid)
        out.append((xy.copy(), grid.reshape(N, N, 2).copy()))
    return out


def test_probes_are_passive_and_follow_the_map():
    """Probe points take no part in the density (the samples end exactly as
    without them), a probe placed on a sample moves exactly like it, and the
    probes on the texel lattice give the step-by-step composite of the
    per-iteration deformations (Sec. 4.3)."""
    xy = dg.plain_small(0)[:3000]
    N = 64
    probe = np.concatenate([xy[:50], dg.lattice_points(N)])
    a = oracle.regularize(xy, N, 3)
    s, p = oracle.regularize_probes(xy, probe, N, 3)
    assert np.array_equal(s, a)
    assert np.array_equal(p[:50], a[:50])
    steps = iterate_with_grid(xy, N, 3)
    assert np.array_equal(p[50:].reshape(N, N, 2), steps[-1][1])


def test_composite_map_is_identity_for_uniform_samples():
    """Samples on the texel lattice are a fixed point, so the composite map is
    the identity at any probe (the field is affine and reproduced exactly)."""
    N = 32
    xy = dg.lattice_points(N)
    probe = dg.rng(5).uniform(0, 1, size=(500, 2))
    s, p = oracle.regularize_probes(xy, probe, N, 3)
    np.testing.assert_allclose(p, probe, rtol=0, atol=1e-12)


def test_probe_errors_and_noop():
    xy = dg.plain_small(0)[:100]
    bad = np.array([[0.5, 1.5]])
    with pytest.raises(oracle.OracleError):
        oracle.regularize_probes(xy, bad, 16, 2)
    # no samples: nothing moves, whatever the probes hold
    s, p = oracle.regularize_probes(np.zeros((0, 2)), bad, 16, 2)
    assert np.array_equal(p, bad)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_no_folds_and_decreasing_measures_small(seed):
    """Sec. 5 and Sec. 6: the deformation keeps the lattice fold-free and
    monotone; bin-std and overplotting decrease at every iteration."""
    xy = dg.plain_small(seed)
    N = 256
    steps = iterate_with_grid(xy, N, 4)
    bs = [metrics.bin_std(xy, N)] + [metrics.bin_std(p, N) for p, _ in steps]
    op = [metrics.overplotting(xy, N)] + [metrics.overplotting(p, N) for p, _ in steps]
    assert all(b1 < b0 for b0, b1 in zip(bs, bs[1:])), bs
    assert all(o1 < o0 for o0, o1 in zip(op, op[1:])), op
    for _, g in steps:
        f = metrics.grid_folds(g)
        assert f == {"nonpos_cells": 0, "x_nonmono": 0, "y_nonmono": 0}, f


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_random_cluster_ensemble_improves(seed):
    xy = dg.random_clusters(seed, 30_000)
    N = 128
    out = oracle.regularize(xy, N, 4)
    assert metrics.bin_std(out, N) < 0.5 * metrics.bin_std(xy, N)
    assert metrics.overplotting(out, N) < metrics.overplotting(xy, N)


def test_selections_do_not_mix():
    """Sec. 6 (manual selections keep sharp boundaries): after regularisation
    nearly every sample's nearest neighbours carry its own label."""
    from scipy.spatial import cKDTree
    pts, lab = dg.four_clusters(0, scale=10)
    out = oracle.regularize(pts, 256, 8)
    tree = cKDTree(out)
    _, nn = tree.query(out, k=9)
    purity_after = np.mean(lab[nn[:, 1:]] == lab[:, None])
    _, nn0 = cKDTree(pts.astype(np.float64)).query(pts, k=9)
    purity_before = np.mean(lab[nn0[:, 1:]] == lab[:, None])
    assert purity_after >= purity_before - 0.01


def test_diagonal_line_spreads():
    """Samples on the diagonal spread over the plot (the paper's first synthetic
    example): occupied 16x16 bins increase and overplotting falls."""
    xy = dg.diagonal_line(0, 20_000)
    N = 256
    out = oracle.regularize(xy, N, 8)

    def occupied(p):
        i = np.minimum((p[:, 0] * 16).astype(int), 15)
        j = np.minimum((p[:, 1] * 16).astype(int), 15)
        return np.unique(j * 16 + i).size

    assert occupied(out) > 2 * occupied(xy.astype(np.float64))
    assert metrics.overplotting(out, N) < metrics.overplotting(xy, N)
