"""Layout quality measures through the C ABI (marked gpu): every integer sum
bit-identical to the oracle (oracle/quality.py), at small ragged sizes and
at the sizes the sweeps use (1M samples on 1024 x 1024, 4096-sample
neighbourhood measures)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import quality as Q
from paper_2408_06513_amd import datagen as dg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(msg: str):
    print(f"[quality] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def q():
    from paper_2408_06513_amd import quality
    quality.lib()
    return quality


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def rnd_points(seed, n):
    return np.random.Generator(np.random.PCG64(seed)).random((n, 2)).astype(np.float32)


def warp(p, seed):
    """Smooth warp plus a few jumps: neighbourhoods and orders change."""
    x, y = p[:, 0].astype(np.float64), p[:, 1].astype(np.float64)
    u = x + 0.08 * np.sin(7 * y) * x * (1 - x)
    v = y + 0.08 * np.sin(9 * x) * y * (1 - y)
    out = np.stack([u, v], 1).astype(np.float32)
    out[::11] = rnd_points(seed, len(out[::11]))
    return out


@pytest.mark.parametrize("res,bin_px", [(64, 4), (256, 8), (100, 5), (4, 4), (1024, 4)])
def test_bins_match_oracle(q, dev, res, bin_px):
    note(f"bins res={res} bin={bin_px}")
    g = np.random.Generator(np.random.PCG64(res))
    c = (g.poisson(0.7, (res, res)) * (g.random((res, res)) < 0.6)).astype(np.uint32)
    c[0, 0] = 4_000_000  # large counts: squares beyond 32 bits
    got = q.bin_stats(torch.from_numpy(c).to(dev), bin_px).tolist()
    assert tuple(got) == Q.bin_stats(c.astype(np.int64), bin_px)


def test_density_measures_end_to_end(q, dev):
    xy = dg.random_clusters(3, 200_000).astype(np.float32)
    note("density measures 200k at 1024")
    m = q.density_measures(to_dev(xy, dev), 1024)
    assert m["bin_std"] == pytest.approx(Q.bin_std(xy, 1024), rel=1e-12)
    assert m["overplotting"] == pytest.approx(Q.overplotting(xy, 1024), rel=1e-12)


@pytest.mark.parametrize("n", [2, 3, 257, 1000, 2049])
def test_ordering_matches_oracle(q, dev, n):
    note(f"ordering n={n}")
    a = rnd_points(n, n)
    a[: n // 3] = np.round(a[: n // 3] * 8) / 8  # equal coordinates
    b = warp(a, n + 1)
    got = tuple(q.ordering_counts(to_dev(a, dev), to_dev(b, dev)).tolist())
    assert got == Q.ordering_counts(a, b)


def test_ordering_of_nothing_and_of_the_identity(q, dev):
    e = torch.empty((0, 2), dtype=torch.float32, device=dev)
    assert q.ordering_counts(e, e).tolist() == [0, 0, 0]
    a = to_dev(rnd_points(9, 700), dev)
    pairs = 700 * 699 // 2
    assert q.ordering_counts(a, a).tolist() == [pairs] * 3


@pytest.mark.parametrize("n,k", [(3, 1), (64, 5), (300, 7), (1025, 20), (1025, 1)])
def test_trust_matches_oracle(q, dev, n, k):
    note(f"trust n={n} k={k}")
    a = rnd_points(2 * n, n)
    a[: n // 4] = dg.lattice_points(16)[: n // 4]  # equal distances: the index decides
    b = warp(a, 2 * n + 1)
    assert q.trust_penalty(to_dev(a, dev), to_dev(b, dev), k).item() == Q.trust_penalty(a, b, k)


def test_trust_rejects_too_many_neighbours(q, dev):
    a = to_dev(rnd_points(1, 10), dev)
    with pytest.raises(ValueError, match="2k < n"):
        q.trust_penalty(a, a, 5)


@pytest.fixture(scope="module")
def regularised_1m(dev):
    from paper_2408_06513_amd import capi
    xy = dg.random_clusters(0, 1_000_000).astype(np.float32)
    d = to_dev(xy, dev)
    capi.regularize(d, 1024, 4)
    torch.cuda.synchronize()
    return xy, d.cpu().numpy()


def test_neighbourhood_measures_at_sweep_size(q, dev, regularised_1m):
    """The first 4096 samples of a 1M-sample layout regularised on 1024 x 1024
    (the sample the sweeps measure): exact penalty and pair counts."""
    xy, out = regularised_1m
    a, b = xy[:4096], out[:4096]
    note("trust + ordering at 4096 of 1M")
    assert q.trust_penalty(to_dev(a, dev), to_dev(b, dev), 7).item() == Q.trust_penalty(a, b, 7)
    assert tuple(q.ordering_counts(to_dev(a, dev), to_dev(b, dev)).tolist()) == Q.ordering_counts(a, b)


def test_regularisation_lowers_bin_std_and_overplotting_every_iteration(q, dev):
    """The paper's quality curves: both measures fall monotonically over the
    iterations, here for 1M samples of three cluster data sets on 1024 x 1024."""
    from paper_2408_06513_amd import capi
    for seed in range(3):
        xy = to_dev(dg.random_clusters(seed, 1_000_000), dev)
        s, o = [], []
        for it in range(9):
            m = q.density_measures(xy, 1024)
            s.append(m["bin_std"])
            o.append(m["overplotting"])
            if it < 8:
                capi.regularize(xy, 1024, 1)
        note(f"seed {seed}: bin std {np.round(s, 2)} overplotting {np.round(o, 3)}")
        assert all(x > y for x, y in zip(s, s[1:])), s
        assert all(x > y for x, y in zip(o, o[1:])), o


def test_neighbourhood_measures_at_the_timed_size_keep_their_invariants(q, dev):
    """16384 samples, the largest size the benchmark times, in its launch
    configuration: isometries (identity, the x <-> y reflection) keep every
    neighbourhood, the identity keeps every pair's order and a mirror in x
    inverts every x-order while keeping the y-orders."""
    n = 16384
    a_np = dg.random_clusters(5, n).astype(np.float32)
    a = to_dev(a_np, dev)
    note(f"invariants at n={n}")
    assert q.trust_penalty(a, a, 7).item() == 0
    assert q.trust_penalty(a, to_dev(a_np[:, ::-1], dev), 7).item() == 0
    pairs = n * (n - 1) // 2
    assert q.ordering_counts(a, a).tolist() == [pairs] * 3
    mirror = a_np.copy()
    mirror[:, 0] = 1.0 - mirror[:, 0]
    # x -> 1 - x reverses every strict x-order (or rounds it to a tie); only
    # pairs with equal x keep their (zero) sign
    _, cnt = np.unique(a_np[:, 0], return_counts=True)
    equal_x = int((cnt * (cnt - 1) // 2).sum())
    kept = q.ordering_counts(a, to_dev(mirror, dev)).tolist()
    assert kept == [equal_x, pairs, equal_x]
