"""The oracle's OpenMP loops change nothing: every result is bit-identical
for 1, 2, 3 and 8 threads (each value is computed by the same operations in
the same order whatever the thread count)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2408_06513_amd import datagen as dg


@pytest.fixture
def threads():
    yield oracle.set_threads
    oracle.set_threads(1)


def _all_results():
    xy = dg.plain_small(0)[:6000].astype(np.float64)
    res = 128
    c = oracle.counts(xy, res)
    d = oracle.blur(c, 8)
    pl, marg = oracle.planes(d, oracle.MASK_ALL)
    field = oracle.deform(d, 6000 / res**2)
    moved = oracle.advect(field, xy)
    reg = oracle.regularize(xy, res, 2, radius=4)
    pr_xy, pr = oracle.regularize_probes(xy, dg.lattice_points(32), 64, 2, radius=2)
    return [c, d, pl, marg["X"], marg["U"], marg["V"], field, moved, reg, pr_xy, pr]


def test_results_do_not_depend_on_thread_count(threads):
    assert threads(1) == 1
    ref = _all_results()
    for k in (2, 3, 8):
        assert threads(k) == k
        got = _all_results()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), k


def test_thread_count_floor(threads):
    assert threads(0) == 1
    assert threads(-3) == 1
