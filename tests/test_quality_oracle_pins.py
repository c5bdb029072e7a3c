"""CPU pins of the quality-measure oracle (oracle/quality.py) against library
routines, brute-force loops, closed forms, and the paper's own claim that
the regularity measure and overplotting fall monotonically over the
iterations (Sec. 6, numerical tests)."""
from __future__ import annotations

import itertools

import numpy as np
import pytest
import scipy.stats
import sklearn.manifold

import oracle
from oracle import quality as Q
from paper_2408_06513_amd import datagen


def rnd_points(seed, n):
    return np.random.Generator(np.random.PCG64(seed)).random((n, 2)).astype(np.float32)


def warp(p):
    """A smooth nonlinear map of the unit square into itself (changes neighbourhoods)."""
    x, y = p[:, 0].astype(np.float64), p[:, 1].astype(np.float64)
    u = x + 0.08 * np.sin(7 * y) * x * (1 - x)
    v = y + 0.08 * np.sin(9 * x) * y * (1 - y)
    return np.stack([u, v], 1).astype(np.float32)


@pytest.mark.parametrize("res", [8, 64])
def test_texel_counts_match_histogram2d(res):
    p = rnd_points(1, 5000)
    p[:4] = [[0, 0], [1, 1], [1, 0], [0.5, 1]]  # the edges: x = 1 belongs to the last texel
    h, _, _ = np.histogram2d(p[:, 1].astype(np.float64), p[:, 0].astype(np.float64),
                             bins=np.linspace(0, 1, res + 1))
    assert np.array_equal(Q.texel_counts(p, res), h.astype(np.int64))


def test_lattice_has_no_overplotting_and_uniform_bins():
    res = 32
    p = datagen.lattice_points(res).astype(np.float32)
    occ, s1, s2 = Q.bin_stats(Q.texel_counts(p, res), 4)
    assert (occ, s1, s2) == (res * res, res * res, (res // 4) ** 2 * 16 ** 2)
    assert Q.overplotting(p, res) == 0.0 and Q.bin_std(p, res) == 0.0


def test_one_texel_closed_forms():
    res, n = 16, 1000
    p = np.full((n, 2), 0.3, dtype=np.float32)
    bins = (res // 4) ** 2
    assert Q.overplotting(p, res) == (n - 1) / n
    # one bin holds n samples, the others none
    assert Q.bin_std(p, res) == pytest.approx(n * np.sqrt(bins - 1) / bins, rel=1e-14)


@pytest.mark.parametrize("k", [5, 7])
def test_trustworthiness_matches_sklearn(k):
    a = rnd_points(2, 240)
    b = warp(a)
    want = sklearn.manifold.trustworthiness(a.astype(np.float64), b.astype(np.float64), n_neighbors=k)
    got = Q.trustworthiness(a, b, k)
    assert got < 1.0  # the warp changes some neighbourhoods
    assert got == pytest.approx(want, abs=1e-12)


def brute_trust_penalty(a, b, k):
    A = [(float(x), float(y)) for x, y in a]
    B = [(float(x), float(y)) for x, y in b]
    n = len(A)

    def order(P, i):
        def key(j):
            dx, dy = P[j][0] - P[i][0], P[j][1] - P[i][1]
            return (dx * dx + dy * dy, j)
        return sorted((j for j in range(n) if j != i), key=key)

    total = 0
    for i in range(n):
        oa = order(A, i)
        for j in order(B, i)[:k]:
            r = oa.index(j) + 1
            total += max(0, r - k)
    return total


def test_trust_penalty_brute_force_with_ties():
    # a lattice has many equal distances: the index tie rule decides the order
    a = (datagen.lattice_points(4)[:14]).astype(np.float32)
    b = warp(rnd_points(3, 14))
    for k in (1, 3, 6):
        assert Q.trust_penalty(a, b, k) == brute_trust_penalty(a, b, k)
    c = rnd_points(4, 20)
    assert Q.trust_penalty(c, warp(c), 4) == brute_trust_penalty(c, warp(c), 4)


def test_trustworthiness_of_isometries_is_one():
    a = rnd_points(5, 150)
    assert Q.trust_penalty(a, a, 7) == 0
    assert Q.trust_penalty(a, a[:, ::-1].copy(), 7) == 0  # the reflection x <-> y keeps every distance
    assert Q.trustworthiness(a, a, 7) == 1.0


def brute_ordering(a, b):
    kx = ky = kb = 0
    sgn = lambda v: (v > 0) - (v < 0)
    for i, j in itertools.combinations(range(len(a)), 2):
        sx = sgn(float(a[j, 0]) - float(a[i, 0])) == sgn(float(b[j, 0]) - float(b[i, 0]))
        sy = sgn(float(a[j, 1]) - float(a[i, 1])) == sgn(float(b[j, 1]) - float(b[i, 1]))
        kx += sx
        ky += sy
        kb += sx and sy
    return kx, ky, kb


def test_ordering_brute_force_and_kendall_tau():
    a = rnd_points(6, 60)
    b = warp(a)
    b[::7] = rnd_points(7, len(b[::7]))  # some samples jump
    assert Q.ordering_counts(a, b) == brute_ordering(a, b)
    # ties: equal coordinates keep their pairs only when they stay equal
    t = np.round(a * 4) / 4
    assert Q.ordering_counts(t, b) == brute_ordering(t, b)
    # along one axis, kept pairs are the concordant pairs of Kendall's tau
    n = len(a)
    pairs = n * (n - 1) // 2
    for ax in (0, 1):
        tau = scipy.stats.kendalltau(a[:, ax], b[:, ax]).statistic
        assert Q.ordering_counts(a, b)[ax] == round(pairs * (1 + tau) / 2)


def test_ordering_closed_forms():
    a = rnd_points(8, 100)
    n = len(a)
    pairs = n * (n - 1) // 2
    assert Q.ordering_counts(a, a) == (pairs, pairs, pairs)
    mirror = a.copy()
    mirror[:, 0] = 1 - mirror[:, 0]
    assert Q.ordering_counts(a, mirror) == (0, pairs, 0)
    assert Q.orthogonal_ordering(a, a) == 1.0


def test_regularisation_lowers_bin_std_and_overplotting_every_iteration():
    """The paper reports both measures falling monotonically over the
    iterations on random 1-8 Gaussian-cluster data; the oracle's method
    reproduces that on every data set here (128 x 128, about one sample per
    texel like 1M samples on 1024 x 1024)."""
    res, n = 128, 16000
    for seed in range(3):
        xy = datagen.random_clusters(seed, n).astype(np.float64)
        s = [Q.bin_std(xy, res)]
        o = [Q.overplotting(xy, res)]
        p = xy
        for _ in range(6):
            p = oracle.regularize(p, res, 1, radius=8)
            s.append(Q.bin_std(p, res))
            o.append(Q.overplotting(p, res))
        assert all(x > y for x, y in zip(s, s[1:])), (seed, s)
        assert all(x > y for x, y in zip(o, o[1:])), (seed, o)
        assert s[-1] < 0.4 * s[0]
