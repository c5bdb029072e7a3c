"""Bindings and status reporting (marked gpu): the C defaults, and the
wrappers that must not leave samples silently unmoved.

- inim_default_params leaves sigma unset, so a C caller who only raises the
  radius gets sigma = radius / 2, as the Python bindings do.
- rasterize, advect, their many-set forms, the surrogate's batched move and
  its graphs read the status word on request and raise DomainError for a
  NaN sample; the samples are then unmoved.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

from paper_2408_06513_amd import datagen as dg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(msg: str):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def capi():
    from paper_2408_06513_amd import capi as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def test_c_default_sigma_follows_radius(capi, dev):
    note("inim_rasterize with C defaults and radius 16")
    xy = torch.from_numpy(dg.plain_small(0)).to(dev)
    res = 256
    p = capi.Params()
    capi.lib().inim_default_params(ctypes.byref(p))
    p.radius = 16
    counts = torch.empty((res, res), dtype=torch.uint32, device=dev)
    dens = torch.empty((res, res), dtype=torch.float32, device=dev)
    ws = capi.workspace(256, dev)
    st = capi.lib().inim_rasterize(ctypes.c_void_p(xy.data_ptr()), xy.shape[0], res, ctypes.byref(p),
                                   ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(dens.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert st == capi.OK
    assert capi.sync_status(ws) == capi.OK
    _, ref8, _ = capi.rasterize(xy, res, radius=16, sigma=8.0)
    _, ref4, _ = capi.rasterize(xy, res, radius=16, sigma=4.0)
    assert torch.equal(dens, ref8)
    assert not torch.equal(dens, ref4)


def test_rasterize_and_advect_raise_on_nan(capi, dev):
    note("rasterize / advect with a NaN sample")
    xy = torch.from_numpy(dg.plain_small(1)[:4096]).to(dev)
    xy[17, 1] = float("nan")
    with pytest.raises(capi.DomainError):
        capi.rasterize(xy, 64, radius=2)
    field = torch.from_numpy(dg.lattice_points(64).reshape(64, 64, 2)).to(dev)
    before = xy.clone()
    with pytest.raises(capi.DomainError):
        capi.advect(field, xy)
    assert np.array_equal(xy.cpu().numpy(), before.cpu().numpy(), equal_nan=True)
    xs = [torch.from_numpy(dg.plain_small(s)[:2048]).to(dev) for s in range(3)]
    xs[2][5, 0] = 1.5
    with pytest.raises(capi.DomainError):
        capi.rasterize_many(xs, 64, radius=2)


def _small_net(dev):
    from paper_2408_06513_amd import surrogate as S
    return S.UNet(dev, seed=3, chans=(8, 16, 16))


def test_surrogate_batched_move_raises_on_nan(capi, dev):
    from paper_2408_06513_amd import surrogate as S
    note("surrogate regularize_many / graphs with a NaN sample")
    net = _small_net(dev)
    xs = [torch.from_numpy(dg.surrogate_mixture(s, n_hi=20_000)).to(dev) for s in range(4)]
    xs[1][3, 0] = float("nan")
    before = [x.clone() for x in xs]
    with pytest.raises(capi.DomainError):
        S.regularize_many(net, xs, 256, net_res=64)
    for x, b in zip(xs, before):  # no set of the group moved
        assert np.array_equal(x.cpu().numpy(), b.cpu().numpy(), equal_nan=True)
    g = S.SurrogateManyGraph(net, xs, 256, net_res=64)
    with pytest.raises(capi.DomainError):
        g(check=True)
    for x, b in zip(xs, before):
        assert np.array_equal(x.cpu().numpy(), b.cpu().numpy(), equal_nan=True)
    del g
    one = xs[1]
    sg = S.SurrogateGraph(net, one.shape[0], 256, net_res=64, xy=one)
    with pytest.raises(capi.DomainError):
        sg(check=True)
    assert np.array_equal(one.cpu().numpy(), before[1].cpu().numpy(), equal_nan=True)
    # a clean set through the same graph class passes the check
    good = torch.from_numpy(dg.surrogate_mixture(7, n_hi=20_000)).to(dev)
    sg2 = S.SurrogateGraph(net, good.shape[0], 256, net_res=64, xy=good)
    sg2(check=True)
