"""Probe points through the C ABI (marked gpu): the composite map of all
iterations at passive points, against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2408_06513_amd import datagen as dg
from tests import metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(msg: str):
    print(f"[probes] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def capi():
    from paper_2408_06513_amd import capi as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def test_probes_small_config(capi, dev):
    """20k points at 256^2, 4 iterations, probes on the texel lattice plus on
    100 samples: probes within 1e-5 of the oracle, samples bit-identical to a
    run without probes, probes on samples bit-identical to those samples."""
    xy = dg.plain_small(0)
    res, iters = 256, 4
    probe = np.concatenate([xy[:100], dg.lattice_points(res)])
    note("probes C1")
    g, p = to_dev(xy, dev), to_dev(probe, dev)
    capi.regularize_probes(g, p, res, iters)
    plain = to_dev(xy, dev)
    capi.regularize(plain, res, iters)
    got_xy, got_p = g.cpu().numpy(), p.cpu().numpy()
    assert np.array_equal(got_xy, plain.cpu().numpy())
    assert np.array_equal(got_p[:100], got_xy[:100])
    ref_xy, ref_p = oracle.regularize_probes(xy, probe, res, iters)
    err = np.abs(got_p.astype(np.float64) - ref_p).max()
    note(f"C1 probes max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-5
    assert np.abs(got_xy.astype(np.float64) - ref_xy).max() <= 1e-5


def test_probes_large_config_lattice(capi, dev):
    """1M points at 1024^2, 8 iterations, the whole 1024^2 lattice as probes:
    within 1e-5 of the oracle, and the deformed grid is fold-free."""
    xy = dg.plain_large(0)
    res, iters = 1024, 8
    lat = dg.lattice_points(res)
    note("probes C2 (oracle takes a few seconds)")
    g, p = to_dev(xy, dev), to_dev(lat, dev)
    capi.regularize_probes(g, p, res, iters)
    got = p.cpu().numpy()
    _, ref = oracle.regularize_probes(xy, lat, res, iters)
    err = np.abs(got.astype(np.float64) - ref).max()
    note(f"C2 probes max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-5
    f = metrics.grid_folds(got.reshape(res, res, 2))
    assert f == {"nonpos_cells": 0, "x_nonmono": 0, "y_nonmono": 0}, f


def test_probes_uniform_samples_identity(capi, dev):
    res = 64
    xy = dg.lattice_points(res)
    probe = dg.rng(5).uniform(0, 1, size=(5000, 2)).astype(np.float32)
    g, p = to_dev(xy, dev), to_dev(probe, dev)
    capi.regularize_probes(g, p, res, 3)
    assert np.abs(p.cpu().numpy() - probe).max() <= 1e-6


def test_probe_errors_and_noop(capi, dev):
    xy = dg.plain_small(6)[:1000].copy()
    probe = dg.lattice_points(32)
    for bad in (np.nan, 1.5, -0.25):
        pb = probe.copy()
        pb[77, 0] = bad
        g, p = to_dev(xy, dev), to_dev(pb, dev)
        with pytest.raises(capi.DomainError):
            capi.regularize_probes(g, p, 64, 3)
        assert np.array_equal(g.cpu().numpy(), xy)
        assert np.array_equal(p.cpu().numpy(), pb, equal_nan=True)
    # no probes: the plain result; no samples or no iterations: nothing moves
    g = to_dev(xy, dev)
    capi.regularize_probes(g, torch.empty((0, 2), dtype=torch.float32, device=dev), 64, 2)
    assert np.abs(g.cpu().numpy() - oracle.regularize(xy, 64, 2)).max() <= 1e-5
    p = to_dev(probe, dev)
    capi.regularize_probes(torch.empty((0, 2), dtype=torch.float32, device=dev), p, 64, 2)
    assert np.array_equal(p.cpu().numpy(), probe)
    g = to_dev(xy, dev)
    capi.regularize_probes(g, p, 64, 0)
    assert np.array_equal(p.cpu().numpy(), probe) and np.array_equal(g.cpu().numpy(), xy)
