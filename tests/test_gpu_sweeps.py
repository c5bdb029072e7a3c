"""The parameter sweeps (marked gpu): the configurations they visit that the
other parity tests do not (4096 x 4096 rasters, r = 16, a background d0
far below n/N^2) against the oracle, then a shortened run of every sweep
with the trends the paper reports."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2408_06513_amd import datagen as dg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(msg: str):
    print(f"[sweeps] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    from paper_2408_06513_amd import capi
    capi.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("res,radius,d0_scale", [(4096, 8, 1.0), (2048, 16, 1e-3), (1024, 1, 1e-2), (512, 8, 0.0)])
def test_sweep_configurations_match_oracle(dev, res, radius, d0_scale):
    from paper_2408_06513_amd import capi
    n, iters = 50_000, 2
    xy = dg.plain_large(0, n=n) if d0_scale == 1.0 else dg.random_clusters(1, n)
    d0 = d0_scale * n / (res * res)
    note(f"regularize res={res} r={radius} d0={d0:.3g} (oracle takes seconds)")
    t = torch.from_numpy(xy.astype(np.float32)).to(dev)
    capi.regularize(t, res, iters, radius=radius, d0=d0)
    got = t.cpu().numpy().astype(np.float64)
    ref = oracle.regularize(xy.astype(np.float32).astype(np.float64), res, iters, radius=radius, d0=d0)
    err = np.abs(got - ref).max()
    note(f"max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-5


def test_quick_sweeps_and_their_trends(dev):
    from paper_2408_06513_amd import sweeps
    note("quick sweeps")
    sw = sweeps.run_all(dev, quick=True)
    t = sw["table1"]["rows"]
    for row in t.values():
        ms = row["ms"]
        assert all(a < b for a, b in zip(ms, ms[1:])), ms  # more iterations take longer
        assert row["per_iter_ms"] > 0
    assert t["1000000"]["ms"][-1] > t["500000"]["ms"][-1] * 0.9
    for c in sw["quality_curves"]["by_n"].values():
        assert sweeps.monotone_decreasing(c["bin_std"]) and sweeps.monotone_decreasing(c["overplotting"])
    for e in list(sw["radius"]["by_radius"].values()) + list(sw["d0"]["by_scale"].values()):
        assert 0.5 < e["trust"] <= 1.0 and 0.5 < e["ordering"] <= 1.0 and e["folds"] >= 0
    # the paper: vanishing density lets mapped regions overlap, its d0 prevents
    # that, and larger kernels soften it
    d = sw["d0"]["by_scale"]
    assert d["1.0"]["folds"] == 0 < d["0.0"]["folds"]
    by_r = sw["radius"]["by_radius"]
    assert by_r["8"]["folds"] == by_r["2"]["folds"] == 0
    assert by_r["8"]["folds_without_background"] <= by_r["2"]["folds_without_background"]
    s = sweeps.summary(sw)
    assert s["quality_monotone"]
    kt = sweeps.kernel_times(dev, sizes=(1024,), reps=2)
    assert kt["n1024"]["trust_ms"] > 0 and kt["bins_1024"]["ms"] > 0
    note(f"summary {s}")
