"""The surrogate's layers through the C ABI (marked gpu), against the FP64
oracle (oracle/nn_oracle.py).  Convolutions of small integers are exact in
FP32, so those comparisons are bit for bit (they pin the matrix-core lane
layout and every index); random operands are held to the FP32 accumulation
bound |err| <= 1e-3 * sum |x| |w|."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import nn_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
D, BF = torch.float64, torch.bfloat16

CONV_SHAPES = [(2, 16, 16, 8, 8, 3), (1, 20, 13, 16, 40, 3), (2, 8, 8, 24, 136, 3), (1, 32, 32, 64, 8, 1),
               (3, 5, 7, 8, 16, 3), (1, 64, 64, 32, 32, 3), (2, 16, 16, 256, 256, 3), (2, 32, 32, 32, 64, 3),
               (1, 16, 16, 96, 48, 3)]


def note(msg):
    print(f"[nn] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def nn():
    from paper_2408_06513_amd import nn as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def ints(seed, shape, lo=-3, hi=3):
    return torch.tensor(np.random.Generator(np.random.PCG64(seed)).integers(lo, hi + 1, size=shape), dtype=D)


def normal(seed, shape, scale=1.0):
    return O.bf16_round(torch.tensor(np.random.Generator(np.random.PCG64(seed)).standard_normal(shape) * scale, dtype=D))


def g16(t, dev):
    return t.to(torch.float32).to(BF).to(dev).contiguous()


def g32(t, dev):
    return t.to(torch.float32).to(dev).contiguous()


@pytest.mark.parametrize("shape", CONV_SHAPES)
def test_conv_forward_exact(nn, dev, shape):
    n, h, w, cin, cout, ks = shape
    note(f"conv forward {shape}")
    x, wt, b = ints(1, (n, h, w, cin)), ints(2, (cout, ks * ks, cin)), ints(3, (cout,), -20, 20)
    y32 = torch.empty((n, h, w, cout), dtype=torch.float32, device=dev)
    y16 = torch.empty((n, h, w, cout), dtype=BF, device=dev)
    nn.conv_forward(g16(x, dev), g16(wt, dev), g32(b, dev), relu=True, y16=y16, y32=y32)
    ref = O.conv(x, wt, b, relu=True)
    assert torch.equal(y32.cpu().double(), ref)
    assert torch.equal(y16.cpu().double(), O.bf16_round(ref))


@pytest.mark.parametrize("imgs,h,w,ca,cb", [(1, 4, 4, 256, 256), (2, 8, 5, 64, 32), (3, 1, 1, 8, 16)])
def test_concat_up2_equals_upsample_and_copy(nn, dev, imgs, h, w, ca, cb):
    a = g16(normal(50, (imgs, h, w, ca)), dev)
    b = g16(normal(51, (imgs, 2 * h, 2 * w, cb)), dev)
    y = torch.empty((imgs, 2 * h, 2 * w, ca + cb), dtype=BF, device=dev)
    nn.concat_up2(a, b, y)
    ref = torch.empty_like(y)
    nn.upsample2_into(a, ref, 0)
    nn.copy_channels_into(b, ref, ca)
    assert torch.equal(y, ref)


def test_split_forward_passes_share_one_work_buffer(nn, dev):
    """Split forward passes of several shapes, repeated on one work buffer:
    every repeat is exact."""
    shapes = [(1, 4, 4, 256, 256, 3), (1, 8, 8, 128, 256, 3), (2, 16, 16, 256, 256, 3), (1, 32, 32, 64, 128, 3)]
    work = torch.empty(max(nn.conv_workspace(*sh) for sh in shapes), dtype=torch.uint8, device=dev)
    cases = []
    for k, (n, h, w, cin, cout, ks) in enumerate(shapes):
        x, wt, b = ints(20 + k, (n, h, w, cin)), ints(30 + k, (cout, ks * ks, cin)), ints(40 + k, (cout,), -20, 20)
        cases.append((g16(x, dev), g16(wt, dev), g32(b, dev), (n, h, w, cout), O.conv(x, wt, b, relu=True)))
    for rep in range(3):
        for k, (x, wt, b, oshape, ref) in enumerate(cases):
            note(f"split forward {shapes[k]} repeat {rep}")
            y32 = torch.empty(oshape, dtype=torch.float32, device=dev)
            nn.conv_forward(x, wt, b, relu=True, y32=y32, work=work)
            assert torch.equal(y32.cpu().double(), ref), (rep, k)


@pytest.mark.parametrize("shape", CONV_SHAPES)
def test_conv_backward_exact(nn, dev, shape):
    n, h, w, cin, cout, ks = shape
    note(f"conv backward {shape}")
    x, wt, dy = ints(4, (n, h, w, cin)), ints(5, (cout, ks * ks, cin)), ints(6, (n, h, w, cout))
    xr, wr = x.clone().requires_grad_(True), wt.clone().requires_grad_(True)
    br = torch.zeros(cout, dtype=D, requires_grad=True)
    (O.conv(xr, wr, br) * dy).sum().backward()
    w16 = g16(wt, dev)
    wT = torch.empty((cin, ks * ks, cout), dtype=BF, device=dev)
    nn.weight_transpose(w16, wT)
    assert torch.equal(wT.cpu(), w16.cpu().permute(2, 1, 0).contiguous())
    dx = torch.empty((n, h, w, cin), dtype=torch.float32, device=dev)
    nn.conv_backward_data(g16(dy, dev), wT, dx)
    assert torch.equal(dx.cpu().double(), xr.grad)
    dw = torch.empty((cout, ks * ks, cin), dtype=torch.float32, device=dev)
    db = torch.empty(cout, dtype=torch.float32, device=dev)
    nn.conv_backward_weight(g16(dy, dev), g16(x, dev), ks, dw, db)
    assert torch.equal(dw.cpu().double(), wr.grad)
    assert torch.equal(db.cpu().double(), br.grad)


def test_conv_random_operands_within_fp32_bound(nn, dev):
    n, h, w, cin, cout, ks = 2, 32, 32, 256, 128, 3
    x, wt = normal(7, (n, h, w, cin)), normal(8, (cout, ks * ks, cin), 0.05)
    y = torch.empty((n, h, w, cout), dtype=torch.float32, device=dev)
    nn.conv_forward(g16(x, dev), g16(wt, dev), None, y32=y)
    ref = O.conv(x, wt)
    bound = O.conv(x.abs(), wt.abs())
    assert ((y.cpu().double() - ref).abs() <= 1e-3 * bound + 1e-6).all()


def test_elementwise_layers(nn, dev):
    n, h, w, c = 2, 8, 12, 16
    x = normal(9, (n, h, w, c))
    p = torch.empty((n, h // 2, w // 2, c), dtype=BF, device=dev)
    nn.pool2(g16(x, dev), p)
    assert torch.allclose(p.cpu().double(), O.bf16_round(O.pool2(x)), rtol=0, atol=0)
    dy = normal(10, (n, h // 2, w // 2, c))
    dx = g32(normal(11, (n, h, w, c)), dev)
    base = dx.cpu().double()
    nn.pool2_backward(g32(dy, dev), dx, accumulate=True)
    ref = base + torch.repeat_interleave(torch.repeat_interleave(dy, 2, 1), 2, 2) / 4
    assert torch.allclose(dx.cpu().double(), ref, rtol=1e-6, atol=1e-6)
    # concatenation [up(a) | b] and its gradient
    a, b = normal(12, (n, h // 2, w // 2, 8)), normal(13, (n, h, w, 24))
    cat = torch.empty((n, h, w, 32), dtype=BF, device=dev)
    nn.upsample2_into(g16(a, dev), cat, 0)
    nn.copy_channels_into(g16(b, dev), cat, 8)
    assert torch.equal(cat.cpu().double(), torch.cat([O.up2(a), b], dim=-1))
    gcat = normal(14, (n, h, w, 32))
    da = torch.empty((n, h // 2, w // 2, 8), dtype=torch.float32, device=dev)
    nn.upsample2_backward(g32(gcat, dev), da)
    assert torch.allclose(da.cpu().double(), gcat[..., :8].reshape(n, h // 2, 2, w // 2, 2, 8).sum(dim=(2, 4)),
                          rtol=1e-6, atol=1e-6)
    db = torch.empty((n, h, w, 24), dtype=torch.float32, device=dev)
    nn.take_channels(g32(gcat, dev), 8, db)
    assert torch.equal(db.cpu().double(), gcat[..., 8:].float().double())
    # ReLU gradient with the mask of the layer's output, BF16 cast
    g = normal(15, (n, h, w, c))
    act = normal(16, (n, h, w, c)).clamp(min=0)
    out = torch.empty((n, h, w, c), dtype=BF, device=dev)
    nn.relu_backward(g32(g, dev), g16(act, dev), out)
    assert torch.equal(out.cpu().double(), O.bf16_round(g * (act > 0)))
    f = torch.tensor([1.0, 1.00390625, 1.01171875, -3.3e-5, 65504.0, 1e-40], dtype=torch.float32)
    b16 = torch.empty(6, dtype=BF, device=dev)
    nn.to_bf16(f.to(dev), b16)
    assert torch.equal(b16.cpu(), f.to(BF))


def test_mse_and_adam(nn, dev):
    pred, tgt = normal(17, (2, 8, 8, 8)), normal(18, (2, 8, 8, 2))
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = torch.empty((2, 8, 8, 8), dtype=BF, device=dev)
    nn.mse(g32(pred, dev), g32(tgt, dev), loss, grad)
    assert abs(float(loss.item()) - float(O.mse(pred, tgt))) <= 1e-5 * float(O.mse(pred, tgt))
    gref = torch.zeros_like(pred)
    gref[..., :2] = 2 * (pred[..., :2] - tgt) / tgt.numel()
    assert torch.allclose(grad.cpu().double(), O.bf16_round(gref), rtol=1e-2, atol=1e-7)
    w0, gr = normal(19, (1000,)), normal(20, (1000,))
    w, m, v = g32(w0, dev), torch.zeros(1000, device=dev), torch.zeros(1000, device=dev)
    wr, mr, vr = w0.clone(), torch.zeros(1000, dtype=D), torch.zeros(1000, dtype=D)
    for step in (1, 2, 3):
        nn.adam(w, g32(gr, dev), m, v, step, lr=0.01)
        wr, mr, vr = O.adam_step(wr, gr, mr, vr, step, lr=0.01)
    assert torch.allclose(w.cpu().double(), wr, rtol=0, atol=1e-5)


def test_unet_forward_and_gradients_match_oracle(dev):
    from paper_2408_06513_amd import surrogate as S
    chans = (8, 16, 16)
    net = S.UNet(dev, seed=3, chans=chans)
    x = normal(21, (2, 16, 16, 8))
    t = normal(22, (2, 16, 16, 2))
    y = net.forward(g16(x, dev))
    p = net.params_f64()
    loss, grads, yref = O.unet_loss_grads(p, x, t, levels=3, bf16=True)
    yg = y.cpu().double()
    assert (yg - yref).abs().max() <= 2e-2 * yref.abs().max()
    lo = torch.zeros(1, dtype=torch.float32, device=dev)
    gy = torch.empty(y.shape, dtype=BF, device=dev)
    from paper_2408_06513_amd import nn as m
    m.mse(y, g32(t, dev), lo, gy)
    net.backward(gy)
    for name, c in net.convs.items():
        for key, gpu in ((name + ".w", c.gw), (name + ".b", c.gb)):
            a, b = gpu.cpu().double().reshape(-1), grads[key].reshape(-1)
            cos = float((a @ b) / (a.norm() * b.norm() + 1e-300))
            assert cos >= 0.995, (key, cos)
            assert abs(float(a.norm() / b.norm()) - 1.0) <= 0.03, (key, float(a.norm() / b.norm()))


# ------------------------------------------------------------------ 5-level network, element by element
U = 2.0 ** -24  # unit roundoff of FP32


def gamma(k: int) -> float:
    """Worst-case relative bound of a sum of k FP32 roundings (any order)."""
    return k * U / (1.0 - k * U)


def check_close(name, got, ref, bound):
    """Element-wise |got - ref| <= bound, reporting the worst ratio."""
    err = (got - ref).abs()
    ratio = float((err / bound.clamp(min=1e-300)).max())
    note(f"{name}: max|err| {float(err.max()):.3e}, worst err/bound {ratio:.3f}")
    assert (err <= bound).all(), (name, ratio)


def test_unet5_lockstep_elementwise(dev):
    """The 5-level 32-256 network (the surrogate's configuration) at 32 x 32,
    two images, compared element by element with the FP64 oracle, one layer at
    a time: each layer's output is recomputed by the oracle from the inputs the
    layer received, so no rounding difference of an earlier layer is carried
    along.  (Run end to end, FP32 and FP64 accumulation under the same BF16
    storage already differ by up to half the scale of the deepest layer's
    weight gradient on the CPU: ReLU masks and BF16 roundings flip and the
    flips compound, so no element-wise tolerance would mean anything there.)

    Bounds, from the arithmetic: a product of two BF16 values is exact in
    FP32, a sum of K of them carries at most gamma(K) = K u / (1 - K u) of the
    sum of their magnitudes (u = 2^-24, any order, split sums included), taken
    twice for margin; a value stored in BF16 (round to nearest even) is
    within 2^-8 of its magnitude of what was rounded; the ReLU-masked cast is
    the same rounding on both sides and must match bit for bit."""
    from paper_2408_06513_amd import nn as m
    from paper_2408_06513_amd import surrogate as S

    net = S.UNet(dev, seed=3)  # channels 32, 64, 128, 256, 256
    assert net.levels == 5
    n, hw = 2, 32
    x = normal(21, (n, hw, hw, 8))
    t = normal(22, (n, hw, hw, 2))
    y = net.forward(g16(x, dev))
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    gy = torch.empty(y.shape, dtype=BF, device=dev)
    m.mse(y, g32(t, dev), loss, gy)
    rec = {}
    net.backward(gy, record=rec)
    torch.cuda.synchronize()
    unet_lockstep_checks(net, y, gy, t, rec)


def test_unet5_coarse_output_lockstep_elementwise(dev):
    """The same element-wise checks for the network whose decoder stops at
    level 2 (the field on a quarter-resolution lattice, the surrogate's
    configuration on the 256 x 256 raster): 32 x 32 in, 8 x 8 out; the two
    top encoder levels then feed only the deeper path (no skip gradient)."""
    from paper_2408_06513_amd import nn as m
    from paper_2408_06513_amd import surrogate as S

    net = S.UNet(dev, seed=4, out_level=2)
    assert net.levels == 5 and "d0a" not in net.convs and "d1a" not in net.convs
    n, hw = 2, 32
    x = normal(23, (n, hw, hw, 8))
    t = normal(24, (n, hw // 4, hw // 4, 2))
    y = net.forward(g16(x, dev))
    assert tuple(y.shape) == (n, hw // 4, hw // 4, 8)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    gy = torch.empty(y.shape, dtype=BF, device=dev)
    m.mse(y, g32(t, dev), loss, gy)
    rec = {}
    net.backward(gy, record=rec)
    torch.cuda.synchronize()
    unet_lockstep_checks(net, y, gy, t, rec)


def unet_lockstep_checks(net, y, gy, t, rec):
    """The element-wise checks of test_unet5_lockstep_elementwise on a network
    after one forward and backward pass (tensors on any device)."""
    n, hw = y.shape[0], y.shape[1]
    lo, L = net.out_level, net.levels
    h64 = lambda a: a.detach().cpu().double()  # noqa: E731
    bf = O.bf16_round
    W = {k: h64(c.w16) for k, c in net.convs.items()}
    for k, c in net.convs.items():
        assert torch.equal(W[k], bf(h64(c.w))), k  # the BF16 weight copies
    hin = net.inp["e0"].shape[1]
    pixels = n * hin * hin  # the most terms a weight gradient sums (the top level)

    def conv_inputs(name):
        if name == "head":
            return h64(net.inp["head"])
        lvl = name[:2]
        return h64(net.inp[lvl]) if name.endswith("a") else h64(net.mid[lvl])

    def conv_output(name):
        lvl = name[:2]
        return h64(net.mid[lvl]) if name.endswith("a") else h64(net.out[lvl])

    # forward, every convolution: output = bf16(relu(conv(input) + bias))
    for name, c in net.convs.items():
        xin = conv_inputs(name)
        k = c.cin * c.ks * c.ks + 1
        ref = O.conv(xin, W[name], h64(c.b))
        mag = O.conv(xin.abs(), W[name].abs(), h64(c.b).abs())
        acc = 2 * gamma(k) * mag
        if name == "head":
            check_close("forward head", h64(y), ref, acc)
            continue
        ref = torch.relu(ref)
        check_close(f"forward {name}", conv_output(name), ref, 2.0 ** -8 * (ref + acc) + acc)

    # forward glue: pooling (BF16 mean of four BF16 values) and concatenation
    for lvl in range(1, L):
        ref = O.pool2(h64(net.out[f"e{lvl - 1}"]))
        check_close(f"pool into e{lvl}", h64(net.inp[f"e{lvl}"]), ref, 2.0 ** -8 * ref.abs() + 1e-30)
    for lvl in range(lo, L - 1):
        below = h64(net.out[f"d{lvl + 1}"] if lvl < L - 2 else net.out[f"e{L - 1}"])
        ref = torch.cat([O.up2(below), h64(net.out[f"e{lvl}"])], dim=-1)
        assert torch.equal(h64(net.inp[f"d{lvl}"]), ref), lvl

    # the squared-error gradient: bf16(2 (y - t) / (pixels * 2)) on the first two channels
    ref = torch.zeros_like(h64(y))
    ref[..., :2] = 2 * (h64(y)[..., :2] - t.float().double()) / t.numel()
    check_close("mse gradient", h64(gy), ref, 2.0 ** -8 * ref.abs() + 1e-30)

    # backward, every convolution
    for name, c in net.convs.items():
        r = rec[name]
        xin, gz = conv_inputs(name), h64(r["gz"])
        if "g" in r:  # the ReLU mask and BF16 cast, the same rounding on both sides
            mask = conv_output(name) > 0
            assert torch.equal(gz, bf(h64(r["g"]) * mask)), name
        kw = pixels
        ref = O._conv_dw(xin, gz, c.ks)
        check_close(f"weight gradient {name}", h64(c.gw), ref, 2 * gamma(kw) * O._conv_dw(xin.abs(), gz.abs(), c.ks))
        check_close(f"bias gradient {name}", h64(c.gb), gz.sum(dim=(0, 1, 2)),
                    2 * gamma(kw) * gz.abs().sum(dim=(0, 1, 2)) + 1e-30)
        if "dx" in r:
            ref = O._conv_dx(gz, W[name], xin.shape)
            bound = 2 * gamma(c.cout * c.ks * c.ks) * O._conv_dx(gz.abs(), W[name].abs(), xin.shape)
            check_close(f"data gradient {name}", h64(r["dx"]), ref, bound + 1e-30)

    # backward glue: the upsampling adjoint feeds the level below, the pooling
    # adjoint plus the skip gradient feed each encoder level but the deepest
    # (levels above the output level feed only the deeper path: no skip term)
    for lvl in range(lo, L - 1):
        gcat = h64(rec[f"d{lvl}a"]["dx"])
        cu = gcat.shape[-1] - net.out[f"e{lvl}"].shape[3]
        ref = O._up2_adjoint(gcat[..., :cu])
        below = f"d{lvl + 1}b" if lvl < L - 2 else f"e{L - 1}b"
        check_close(f"upsampling adjoint into {below}", h64(rec[below]["g"]), ref,
                    2 * gamma(4) * O._up2_adjoint(gcat[..., :cu].abs()) + 1e-30)
    for lvl in range(L - 1):
        ref = O._pool2_adjoint(h64(rec[f"e{lvl + 1}a"]["dx"]))
        mag = O._pool2_adjoint(h64(rec[f"e{lvl + 1}a"]["dx"]).abs())
        if lvl >= lo:
            gcat = h64(rec[f"d{lvl}a"]["dx"])
            cu = gcat.shape[-1] - net.out[f"e{lvl}"].shape[3]
            ref, mag = ref + gcat[..., cu:], mag + gcat[..., cu:].abs()
        check_close(f"pooling adjoint (+ skip) into e{lvl}b", h64(rec[f"e{lvl}b"]["g"]), ref,
                    2 * gamma(1) * mag + 1e-30)


def test_adam_two_step_closed_form(nn, dev):
    """The GPU's Adam on gradients (1, 0): the second move is
    -lr (b1 / (1 + b1)) / (sqrt(b2 / (1 + b2)) + eps), which tells b1 from b2."""
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    w = torch.zeros(256, device=dev)
    mo, v = torch.zeros_like(w), torch.zeros_like(w)
    nn.adam(w, torch.ones_like(w), mo, v, 1, lr=lr, b1=b1, b2=b2, eps=eps)
    w1 = w.clone()
    nn.adam(w, torch.zeros_like(w), mo, v, 2, lr=lr, b1=b1, b2=b2, eps=eps)
    step2 = -lr * (b1 / (1 + b1)) / (np.sqrt(b2 / (1 + b2)) + eps)
    assert torch.allclose(w1.cpu().double(), torch.full((256,), -lr / (1 + eps), dtype=D), rtol=1e-6, atol=0)
    assert torch.allclose((w - w1).cpu().double(), torch.full((256,), step2, dtype=D), rtol=1e-5, atol=0)
