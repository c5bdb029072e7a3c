"""Several sample sets in shared launches (marked gpu): rasterize_many,
advect_many, pack_density_many and field_many give, for every set, exactly
what the single-set calls give, and the surrogate's batched move is the
single-set steps around the same batched forward pass, bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2408_06513_amd import datagen as dg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(msg):
    print(f"[many] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def sets(dev, sizes, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k, n in enumerate(sizes):
        xy = dg.plain_small(k % 7)[: min(n, 20_000)] if n <= 20_000 else g.random((n, 2))
        xy = np.ascontiguousarray(xy, dtype=np.float32)
        xy[: len(xy) // 5] = xy[: len(xy) // 5] * np.float32(0.01) + np.float32(0.3)  # crowded texels
        out.append(torch.from_numpy(xy).to(dev))
    return out


@pytest.mark.parametrize("res,radius", [(64, 2), (256, 8), (128, 0)])
def test_rasterize_many_equals_single(dev, res, radius):
    from paper_2408_06513_amd import capi
    xs = sets(dev, [5000, 0, 1, 20_000, 70_001, 333], seed=res)
    note(f"rasterize_many res={res} r={radius}")
    counts, dens, _ = capi.rasterize_many(xs, res, radius=radius)
    for q, x in enumerate(xs):
        c1, d1, _ = capi.rasterize(x, res, radius=radius)
        assert torch.equal(counts[q], c1), q
        assert torch.equal(dens[q], d1), q


def test_advect_many_equals_single_and_rejects_any_bad_set(dev):
    from paper_2408_06513_amd import capi
    res = 128
    g = np.random.Generator(np.random.PCG64(3))
    xs = sets(dev, [4000, 17, 0, 30_000], seed=3)
    centres = (np.arange(res) + 0.5) / res
    base = np.stack(np.meshgrid(centres, centres), -1)
    field = torch.from_numpy((base[None] + 0.01 * g.standard_normal((len(xs), res, res, 2))).astype(np.float32))
    field = field.to(dev).contiguous()
    ref = [x.clone() for x in xs]
    for q, x in enumerate(ref):
        capi.advect(field[q].contiguous(), x)
    note("advect_many 4 sets")
    capi.advect_many(field, xs)
    for q in range(len(xs)):
        assert torch.equal(xs[q], ref[q]), q
    bad = [x.clone() for x in ref]
    bad[3][100, 0] = float("nan")
    before = [b.clone() for b in bad]
    ws = capi.workspace(256, dev)
    capi.advect_many(field, bad, ws=ws, check=False)
    assert capi.sync_status(ws) == capi.EDOMAIN
    with pytest.raises(capi.DomainError):
        capi.advect_many(field, bad, ws=ws)
    for q in range(len(bad)):  # no set moved, the bad sample's NaN included
        assert np.array_equal(bad[q].cpu().numpy(), before[q].cpu().numpy(), equal_nan=True), q


def test_pack_and_field_many_equal_single(dev):
    from paper_2408_06513_amd import nn
    g = torch.Generator(device="cpu").manual_seed(5)
    k, res, c = 5, 64, 8
    dens = torch.rand((k, res, res), generator=g).to(dev)
    scales = [0.5, 1.0, 3.25, 1e-3, 7.0]
    x = torch.empty((k, res, res, c), dtype=torch.bfloat16, device=dev)
    nn.pack_density_many(dens, scales, x)
    y = (torch.randn((k, res, res, c), generator=g) * 3).to(dev)
    f = torch.empty((k, res, res, 2), dtype=torch.float32, device=dev)
    nn.field_many(y, res, f, 2)
    for q in range(k):
        x1 = torch.empty((res, res, c), dtype=torch.bfloat16, device=dev)
        nn.pack_density(dens[q].contiguous(), scales[q], x1)
        assert torch.equal(x[q], x1), q
        f1 = torch.empty((res, res, 2), dtype=torch.float32, device=dev)
        nn.field(y[q].contiguous(), res, f1, 2)
        assert torch.equal(f[q], f1), q


def test_surrogate_batched_move_equals_single_steps(dev):
    """regularize_many = per-set density, pack, field and advect around the
    same batched forward pass (an untrained network: the equality is exact
    whatever the weights)."""
    from paper_2408_06513_amd import capi, nn
    from paper_2408_06513_amd import surrogate as S
    res, net_res = 256, 64
    net = S.UNet(dev, seed=3)
    xs0 = [torch.from_numpy(dg.surrogate_mixture(s, n_hi=60_000)).to(dev) for s in range(7)]
    got = [x.clone() for x in xs0]
    note("regularize_many, 7 sets")
    S.regularize_many(net, got, res, net_res=net_res)
    ref = [x.clone() for x in xs0]
    r = S.net_radius(8, res, net_res)
    x16 = torch.empty((len(ref), net_res, net_res, S.CIN), dtype=torch.bfloat16, device=dev)
    for q, xy in enumerate(ref):
        S.density_input(xy, net_res, r, x16[q])
    y = net.forward(x16)
    for q, xy in enumerate(ref):
        field = torch.empty((net_res, net_res, 2), dtype=torch.float32, device=dev)
        nn.field(y[q], net_res, field, S.field_radius(net_res))
        capi.advect(field, xy)
    for q in range(len(ref)):
        assert torch.equal(got[q], ref[q]), q


def test_surrogate_batched_graph_replays_equal_eager(dev):
    """The captured batched move equals the eager one on every replay, with
    other GPU work between the replays."""
    from paper_2408_06513_amd import capi
    from paper_2408_06513_amd import surrogate as S
    net = S.UNet(dev, seed=4)
    xs0 = [torch.from_numpy(dg.surrogate_mixture(s, n_hi=40_000)).to(dev) for s in range(10, 15)]
    eager = [x.clone() for x in xs0]
    S.regularize_many(net, eager, 256, net_res=64)
    xs = [x.clone() for x in xs0]
    g = S.SurrogateManyGraph(net, xs, 256, 64)
    for x, x0 in zip(xs, xs0):
        assert torch.equal(x, x0)  # capture leaves the sets as they were
    other = torch.from_numpy(dg.plain_small(0)).to(dev)
    for rep in range(3):
        for x, x0 in zip(xs, xs0):
            x.copy_(x0)
        g()
        torch.cuda.synchronize()
        for q in range(len(xs)):
            assert torch.equal(xs[q], eager[q]), (rep, q)
        capi.regularize(other.clone(), 256, 2)
        torch.cuda.synchronize()


def test_pack_input_many_channels(dev):
    """The first-step input: channel 0 the scaled density (bit for bit),
    channels 1-2 the field's displacement from the texel centres times 64
    (within one bfloat16 unit: the device may fuse the centre's product into
    the difference), the other channels exactly 0."""
    from paper_2408_06513_amd import nn
    g = torch.Generator(device="cpu").manual_seed(9)
    k, res, c = 3, 32, 8
    dens = torch.rand((k, res, res), generator=g)
    centre = (torch.arange(res, dtype=torch.float32) + 0.5) * np.float32(1.0 / res)
    field = torch.stack(torch.broadcast_tensors(centre[None, None, :], centre[None, :, None]), dim=-1).expand(k, res, res, 2)
    field = (field + (torch.rand((k, res, res, 2), generator=g) - 0.5) * 0.05).contiguous()
    scales = [1.5, 2.0, 0.25]
    x = torch.empty((k, res, res, c), dtype=torch.bfloat16, device=dev)
    nn.pack_input_many(dens.to(dev), field.to(dev), scales, x)
    got = x.float().cpu()
    for q in range(k):
        assert torch.equal(got[q, ..., 0], (dens[q] * np.float32(scales[q])).to(torch.bfloat16).float())
    disp = (field - torch.stack(torch.broadcast_tensors(centre[None, None, :], centre[None, :, None]), dim=-1)) * 64
    ref = disp.to(torch.bfloat16).float()
    ulp = ref.abs().clamp(min=1e-30) * 2.0 ** -7
    assert ((got[..., 1:3] - ref).abs() <= ulp).all()
    assert torch.equal(got[..., 3:], torch.zeros_like(got[..., 3:]))


def test_first_step_batched_move_equals_single_steps(dev):
    """A network that also reads the method's first step: its batched move
    (regularize_many) gives every set exactly the single-set result."""
    from paper_2408_06513_amd import capi
    from paper_2408_06513_amd import surrogate as S
    net = S.UNet(dev, seed=11, chans=(8, 16, 16), out_level=1, first_step=True)
    xs0 = [torch.from_numpy(dg.surrogate_mixture(s, n_hi=30_000)).to(dev) for s in range(5)]
    ref = []
    for x0 in xs0:
        x = x0.clone()
        capi.advect(S.predict_field(net, x, 128, net_res=64), x)
        ref.append(x)
    xs = [x.clone() for x in xs0]
    S.regularize_many(net, xs, 128, net_res=64)
    for q in range(len(xs)):
        assert torch.equal(xs[q], ref[q]), q

