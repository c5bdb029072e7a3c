"""CPU pins of the surrogate's oracle (oracle/nn_oracle.py): each layer
against its definition written as loops or an identity, the network's
gradients against finite differences."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import nn_oracle as O

D = torch.float64


def rnd(seed, *shape):
    return torch.tensor(np.random.Generator(np.random.PCG64(seed)).standard_normal(shape), dtype=D)


@pytest.mark.parametrize("ks", [1, 3])
def test_conv_matches_direct_loops(ks):
    n, h, w, cin, cout = 2, 4, 5, 3, 2
    x, wt, b = rnd(1, n, h, w, cin), rnd(2, cout, ks * ks, cin), rnd(3, cout)
    y = O.conv(x, wt, b)
    r = ks // 2
    ref = np.zeros((n, h, w, cout))
    for i in range(n):
        for yy in range(h):
            for xx in range(w):
                for co in range(cout):
                    s = float(b[co])
                    for ky in range(ks):
                        for kx in range(ks):
                            sy, sx = yy + ky - r, xx + kx - r
                            if 0 <= sy < h and 0 <= sx < w:
                                s += float((x[i, sy, sx, :] * wt[co, ky * ks + kx, :]).sum())
                    ref[i, yy, xx, co] = s
    np.testing.assert_allclose(y.numpy(), ref, rtol=1e-12, atol=1e-12)
    assert torch.equal(O.conv(x, wt, b, relu=True), torch.relu(y))


def test_pool_and_upsample_definitions_and_adjoints():
    x = rnd(4, 2, 6, 8, 3)
    p = O.pool2(x)
    assert torch.allclose(p[1, 2, 3, 1], x[1, 4:6, 6:8, 1].mean())
    u = O.up2(p)
    assert torch.equal(u[0, 5, 7], p[0, 2, 3])
    # adjoints: the pooling gradient spreads a quarter, the upsampling gradient sums the 2x2 block
    y = rnd(5, 2, 3, 4, 3)
    back_pool = torch.repeat_interleave(torch.repeat_interleave(y, 2, 1), 2, 2) / 4
    assert torch.allclose((O.pool2(x) * y).sum(), (x * back_pool).sum())
    z = rnd(6, 2, 6, 8, 3)
    back_up = z.reshape(2, 3, 2, 4, 2, 3).sum(dim=(2, 4))
    assert torch.allclose((O.up2(y) * z).sum(), (y * back_up).sum())


def test_adam_first_step_moves_by_lr_against_the_gradient():
    g = torch.tensor([3.0, -0.5, 1e-3], dtype=D)
    w, m, v = O.adam_step(torch.zeros(3, dtype=D), g, torch.zeros(3, dtype=D), torch.zeros(3, dtype=D), 1, lr=0.01)
    np.testing.assert_allclose(w.numpy(), -0.01 * np.sign(g.numpy()), rtol=1e-4)


def test_unet_gradients_match_finite_differences():
    chans = (8, 16, 16)
    p = O.init_params(0, cin=8, cout=8, chans=chans)
    x = rnd(7, 1, 8, 8, 8)
    t = rnd(8, 1, 8, 8, 2)
    loss, grads, _ = O.unet_loss_grads(p, x, t, levels=3)
    g = np.random.Generator(np.random.PCG64(9))
    for name in ("e0a.w", "e2b.w", "d0a.w", "d1b.b", "head.w"):
        flat = p[name].reshape(-1)
        for k in g.choice(flat.numel(), size=3, replace=False):
            h = 1e-6
            up = {a: b.clone() for a, b in p.items()}
            dn = {a: b.clone() for a, b in p.items()}
            up[name].reshape(-1)[k] += h
            dn[name].reshape(-1)[k] -= h
            lu = O.mse(O.unet_forward(up, x, 3), t) / t.numel()
            ld = O.mse(O.unet_forward(dn, x, 3), t) / t.numel()
            fd = float((lu - ld) / (2 * h))
            an = float(grads[name].reshape(-1)[k])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, k, fd, an)


def test_unet_shapes_are_the_five_level_network():
    s = O.unet_shapes()
    assert [c[2] for c in s[:10]] == [32, 32, 64, 64, 128, 128, 256, 256, 256, 256]
    assert [(c[1], c[2]) for c in s[10:18:2]] == [(512, 256), (384, 128), (192, 64), (96, 32)]
    assert s[-1] == ("head", 32, 8, 1)
    flops = sum(2 * 9 * ci * co * (256 >> (int(n[1]) if n[0] in "ed" else 0)) ** 2 for n, ci, co, ks in s if ks == 3)
    assert 24e9 < flops < 27e9  # about 25 GFLOP per 256 x 256 raster
