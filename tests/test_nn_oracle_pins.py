"""CPU pins of the surrogate's oracle (oracle/nn_oracle.py): each layer
against its definition written as loops or an identity, Adam against closed
forms of its update, the network's gradients against finite differences, and
the written-out backward against autograd.

Every check takes the oracle module as its argument, so that
tests/test_nn_oracle_mutants.py can run the same checks on copies of the
oracle with planted mistakes."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import nn_oracle

D = torch.float64


def rnd(seed, *shape):
    return torch.tensor(np.random.Generator(np.random.PCG64(seed)).standard_normal(shape), dtype=D)


def check_conv_direct_loops(O, ks):
    """The convolution against its definition as loops (cross-correlation,
    zero padding, taps (ky, kx) row-major)."""
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


def check_pool_and_upsample(O):
    """Pooling is the 2x2 mean, upsampling repeats, and their adjoints spread a
    quarter / sum the 2x2 block."""
    x = rnd(4, 2, 6, 8, 3)
    p = O.pool2(x)
    assert torch.allclose(p[1, 2, 3, 1], x[1, 4:6, 6:8, 1].mean())
    u = O.up2(p)
    assert torch.equal(u[0, 5, 7], p[0, 2, 3])
    y = rnd(5, 2, 3, 4, 3)
    back_pool = torch.repeat_interleave(torch.repeat_interleave(y, 2, 1), 2, 2) / 4
    assert torch.allclose((O.pool2(x) * y).sum(), (x * back_pool).sum())
    z = rnd(6, 2, 6, 8, 3)
    back_up = z.reshape(2, 3, 2, 4, 2, 3).sum(dim=(2, 4))
    assert torch.allclose((O.up2(y) * z).sum(), (y * back_up).sum())


# Adam (Kingma and Ba, Algorithm 1) pinned by closed forms of its definition.
def pin_adam_first_step(O):
    """Step 1 from zero moments: m_hat = g and v_hat = g^2 exactly, so the
    weight moves by lr g / (|g| + eps)."""
    g = torch.tensor([3.0, -0.5, 1e-3], dtype=D)
    z = torch.zeros(3, dtype=D)
    w, m, v = O.adam_step(z.clone(), g, z.clone(), z.clone(), 1, lr=0.01)
    np.testing.assert_allclose(w.numpy(), -0.01 * g.numpy() / (np.abs(g.numpy()) + 1e-8), rtol=1e-12)


def pin_adam_second_step_separates_the_decay_rates(O):
    """Gradient 1 at step 1, then 0: m_2 = b1 (1 - b1) and v_2 = b2 (1 - b2),
    so the bias-corrected moments are b1 / (1 + b1) and b2 / (1 + b2) and the
    second move is -lr (b1 / (1 + b1)) / (sqrt(b2 / (1 + b2)) + eps).  With
    b1 and b2 exchanged it would be 0.7261 lr instead of 0.6701 lr."""
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    one, z = torch.ones(1, dtype=D), torch.zeros(1, dtype=D)
    w1, m, v = O.adam_step(z.clone(), one, z.clone(), z.clone(), 1, lr=lr, b1=b1, b2=b2, eps=eps)
    w2, m, v = O.adam_step(w1, z.clone(), m, v, 2, lr=lr, b1=b1, b2=b2, eps=eps)
    step2 = -lr * (b1 / (1 + b1)) / (np.sqrt(b2 / (1 + b2)) + eps)
    np.testing.assert_allclose(float(w1), -lr / (1 + eps), rtol=1e-12)
    np.testing.assert_allclose(float(w2 - w1), step2, rtol=1e-12)
    np.testing.assert_allclose(float(m), b1 * (1 - b1), rtol=1e-12)
    np.testing.assert_allclose(float(v), b2 * (1 - b2), rtol=1e-12)


def pin_adam_constant_gradient(O):
    """A constant gradient keeps m_hat = g and v_hat = g^2 at every step (the
    bias corrections use the step's own power), so each of 5 steps moves by
    lr g / (|g| + eps); with b1 = 0.5, b2 = 0.25 a wrong power is far off."""
    g = torch.tensor([2.0, -0.25], dtype=D)
    w, m, v = torch.zeros(2, dtype=D), torch.zeros(2, dtype=D), torch.zeros(2, dtype=D)
    for step in range(1, 6):
        w0 = w.clone()
        w, m, v = O.adam_step(w, g, m, v, step, lr=0.1, b1=0.5, b2=0.25, eps=1e-8)
        np.testing.assert_allclose((w - w0).numpy(), -0.1 * g.numpy() / (np.abs(g.numpy()) + 1e-8), rtol=1e-12)


ADAM_PINS = (pin_adam_first_step, pin_adam_second_step_separates_the_decay_rates, pin_adam_constant_gradient)


def check_unet_finite_differences(O):
    """Autograd gradients of the 3-level network against central differences."""
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


def check_stored_backward_identity(O):
    """The written-out backward of unet_grads_stored equals autograd of the
    forward definition when nothing is rounded, and its loss and output are
    the definition's."""
    chans = (8, 16, 16)
    p = O.init_params(0, cin=8, cout=8, chans=chans)
    x, t = rnd(7, 2, 8, 8, 8), rnd(8, 2, 8, 8, 2)
    loss, grads, y = O.unet_loss_grads(p, x, t, levels=3)
    loss2, grads2, y2 = O.unet_grads_stored(p, x, t, levels=3, store=lambda v: v)
    assert abs(float(loss - loss2)) <= 1e-14 * float(loss)
    assert torch.allclose(y, y2, rtol=0, atol=1e-13)
    for k in grads:
        assert torch.allclose(grads[k], grads2[k], rtol=1e-11, atol=1e-13 * float(grads[k].abs().max())), k


# ------------------------------------------------------------------ the tests
@pytest.mark.parametrize("ks", [1, 3])
def test_conv_matches_direct_loops(ks):
    check_conv_direct_loops(nn_oracle, ks)


def test_pool_and_upsample_definitions_and_adjoints():
    check_pool_and_upsample(nn_oracle)


@pytest.mark.parametrize("pin", ADAM_PINS, ids=lambda f: f.__name__)
def test_adam_pins(pin):
    pin(nn_oracle)


def test_unet_gradients_match_finite_differences():
    check_unet_finite_differences(nn_oracle)


def test_stored_backward_with_identity_storage_is_the_exact_gradient():
    check_stored_backward_identity(nn_oracle)


def test_stored_backward_rounds_where_the_gpu_stores_bf16():
    """With bfloat16 storage the forward equals the autograd oracle's bf16
    forward (the same values are rounded) and the gradients stay close to the
    exact ones."""
    O = nn_oracle
    chans = (8, 16, 16)
    p = O.init_params(1, cin=8, cout=8, chans=chans)
    x, t = O.bf16_round(rnd(9, 1, 8, 8, 8)), rnd(10, 1, 8, 8, 2)
    _, _, yb = O.unet_loss_grads(p, x, t, levels=3, bf16=True)
    _, g, ys = O.unet_grads_stored(p, x, t, levels=3)
    assert torch.equal(yb, ys)
    _, g_exact, _ = O.unet_loss_grads(p, x, t, levels=3)
    for k in g:
        a, b = g[k].reshape(-1), g_exact[k].reshape(-1)
        assert float((a @ b) / (a.norm() * b.norm())) > 0.95, k


def test_unet_shapes_are_the_five_level_network():
    s = nn_oracle.unet_shapes()
    assert [c[2] for c in s[:10]] == [32, 32, 64, 64, 128, 128, 256, 256, 256, 256]
    assert [(c[1], c[2]) for c in s[10:18:2]] == [(512, 256), (384, 128), (192, 64), (96, 32)]
    assert s[-1] == ("head", 32, 8, 1)
    flops = sum(2 * 9 * ci * co * (256 >> (int(n[1]) if n[0] in "ed" else 0)) ** 2 for n, ci, co, ks in s if ks == 3)
    assert 24e9 < flops < 27e9  # about 25 GFLOP per 256 x 256 raster
