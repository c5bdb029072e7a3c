"""Batched plots (a scatterplot matrix) through the C ABI (marked gpu): every
plot equal bit for bit to its own inim_regularize call, in every launch shape
and through a graph; two plots against the oracle; errors."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2408_06513_amd import datagen as dg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(msg: str):
    print(f"[batch] {msg}", file=sys.stderr, flush=True)


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


def sequential(capi, dev, plots, iters):
    out = []
    for xy, res in plots:
        g = to_dev(xy, dev)
        capi.regularize(g, res, iters)
        out.append(g.cpu().numpy())
    return out


@pytest.fixture(scope="module")
def small_splom():
    return dg.splom_plots(seed=1, n=20_000, dims=6, sizes=(64, 128, 256))


def test_batch_equals_sequential_every_shape(capi, dev, small_splom):
    iters = 3
    ref = sequential(capi, dev, small_splom, iters)
    res = [r for _, r in small_splom]
    for wpb in (1, 2, 4, 8):
        for order in (0, 1):
            note(f"15 plots, waves_per_block={wpb}, order={order}")
            xs = [to_dev(xy, dev) for xy, _ in small_splom]
            capi.regularize_batch(xs, res, iters, cfg=capi.BatchConfig(wpb, order))
            for k, x in enumerate(xs):
                assert np.array_equal(x.cpu().numpy(), ref[k]), (wpb, order, k)


def test_batch_graph_replays(capi, dev, small_splom):
    iters = 2
    ref = sequential(capi, dev, small_splom, iters)
    res = [r for _, r in small_splom]
    xs = [to_dev(xy, dev) for xy, _ in small_splom]
    ws = capi.workspace(capi.batch_workspace_size(xs, res), dev)
    graph = capi.Graph()
    try:
        for rep in range(3):
            for x, (xy, _) in zip(xs, small_splom):
                x.copy_(to_dev(xy, dev))
            capi.regularize_batch(xs, res, iters, ws=ws, graph=graph)
            torch.cuda.synchronize()
            for k, x in enumerate(xs):
                assert np.array_equal(x.cpu().numpy(), ref[k]), (rep, k)
            _ = torch.ones(1000, device=dev).sum().item()  # eager work between replays
    finally:
        graph.close()


def test_batch_oracle_parity(capi, dev):
    plots = dg.splom_plots(seed=2, n=20_000, dims=3, sizes=(256,))
    xs = [to_dev(xy, dev) for xy, _ in plots]
    capi.regularize_batch(xs, [r for _, r in plots], 4)
    for x, (xy, res) in zip(xs, plots):
        err = np.abs(x.cpu().numpy().astype(np.float64) - oracle.regularize(xy, res, 4)).max()
        note(f"plot at {res}^2: max|gpu-oracle| = {err:.3e}")
        assert err <= 1e-5


def test_batch_full_splom_equals_sequential(capi, dev):
    """The benchmark's matrix: 200,000 samples x 10 dims, 45 plots at
    256/512/1024, 6 iterations."""
    plots = dg.splom_plots(seed=0)
    iters = 6
    note("45-plot matrix: sequential reference")
    ref = sequential(capi, dev, plots, iters)
    xs = [to_dev(xy, dev) for xy, _ in plots]
    note("45-plot matrix: batched")
    capi.regularize_batch(xs, [r for _, r in plots], iters)
    for k, x in enumerate(xs):
        assert np.array_equal(x.cpu().numpy(), ref[k]), k


def test_batch_grouped_rows_and_both_sorts(capi, dev):
    """Plots whose per-row sort takes groups of rows (few samples on 2048^2
    and 512^2), one with dense rows, and 128^2 plots sorted by global ranks,
    in one batched call: bit-identical to one call per plot."""
    g = np.random.Generator(np.random.PCG64(11))
    dense = np.stack([g.random(30_000), 0.5 + g.random(30_000) / 700], 1).astype(np.float32)
    plots = [(dg.plain_small(1)[:3_000], 2048), (dg.plain_small(2)[:9], 512), (dense, 512),
             (dg.plain_small(3)[:5_000], 128), (dg.plain_small(4), 2048)]
    iters = 2
    ref = sequential(capi, dev, plots, iters)
    xs = [to_dev(xy, dev) for xy, _ in plots]
    note("grouped rows, dense rows and both sorts in one batch")
    capi.regularize_batch(xs, [r for _, r in plots], iters)
    for k, x in enumerate(xs):
        assert np.array_equal(x.cpu().numpy(), ref[k]), k


def test_batch_autotune_leaves_samples(capi, dev, small_splom):
    res = [r for _, r in small_splom]
    xs = [to_dev(xy, dev) for xy, _ in small_splom]
    cfg, ms = capi.batch_autotune(xs, res, 2)
    assert cfg.waves_per_block in (1, 2, 4, 8) and cfg.order in (0, 1) and ms > 0
    for x, (xy, _) in zip(xs, small_splom):
        assert np.array_equal(x.cpu().numpy(), xy)


def test_batch_errors_and_empty_plots(capi, dev):
    plots = dg.splom_plots(seed=3, n=5_000, dims=3, sizes=(64,))
    res = [r for _, r in plots]
    # an invalid sample anywhere: nothing moves
    bad = [xy.copy() for xy, _ in plots]
    bad[1][10, 0] = np.nan
    xs = [to_dev(b, dev) for b in bad]
    with pytest.raises(capi.DomainError):
        capi.regularize_batch(xs, res, 2)
    for x, b in zip(xs, bad):
        assert np.array_equal(x.cpu().numpy(), b, equal_nan=True)
    # a plot without samples is left alone and the others are unaffected
    xs = [to_dev(xy, dev) for xy, _ in plots]
    xs[0] = torch.empty((0, 2), dtype=torch.float32, device=dev)
    capi.regularize_batch(xs, res, 2)
    ref = sequential(capi, dev, plots[1:], 2)
    for x, r in zip(xs[1:], ref):
        assert np.array_equal(x.cpu().numpy(), r)
    with pytest.raises(capi.InvalidArgument):
        capi.regularize_batch([to_dev(plots[0][0], dev)], [32], 2)
    with pytest.raises(capi.InvalidArgument):
        capi.regularize_batch([to_dev(plots[0][0], dev)], [64], 2, radius=0)
    with pytest.raises(capi.InvalidArgument):
        capi.regularize_batch([to_dev(plots[0][0], dev)], [64], 2, cfg=capi.BatchConfig(3, 0))
