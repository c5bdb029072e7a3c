"""TEST INFRASTRUCTURE ONLY -- CPU oracle of the learned surrogate's layers.

Plain FP64 PyTorch CPU operations written from the definitions of each layer
(library convolution, pooling and autograd serve as steps); NHWC tensors as in
the HIP path.  Only tests, the package's smoke check and the benchmark's CPU
baseline may use it; the product path never does.

The network is a U-Net (encoder of five levels with two 3x3 convolutions and
ReLU each, 2x2 average pooling between levels, decoder with nearest 2x
upsampling, concatenation with the encoder level of the same size, two 3x3
convolutions with ReLU, and a final 1x1 convolution).  `bf16=True` rounds the
input of every convolution to bfloat16 (round to nearest even), where the HIP
path stores its activations in bfloat16.

Parity unpinned: the surrogate is not part of the paper; its layers are
pinned by definitions (direct loops, adjoint identities, finite differences),
not by published values.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

D = torch.float64


def bf16_round(t: torch.Tensor) -> torch.Tensor:
    """Round to the nearest bfloat16 (ties to even), returned in t's dtype."""
    return t.to(torch.float32).to(torch.bfloat16).to(t.dtype)


def _nchw(x):
    return x.permute(0, 3, 1, 2)


def _nhwc(x):
    return x.permute(0, 2, 3, 1)


def conv(x, w, bias=None, relu=False):
    """x [n,h,w,cin]; w [cout, ks*ks, cin] with taps (ky, kx) row-major;
    y[p][co] = bias[co] + sum_t sum_ci x[p + (ky - ks/2, kx - ks/2)][ci] w[co][t][ci]
    with zero padding (cross-correlation, stride 1)."""
    cout, taps, cin = w.shape
    ks = int(round(taps ** 0.5))
    wk = w.reshape(cout, ks, ks, cin).permute(0, 3, 1, 2)
    y = _nhwc(F.conv2d(_nchw(x), wk, bias, padding=ks // 2))
    return torch.relu(y) if relu else y


def pool2(x):
    return _nhwc(F.avg_pool2d(_nchw(x), 2))


def up2(x):
    return _nhwc(F.interpolate(_nchw(x), scale_factor=2, mode="nearest"))


def mse(pred, target):
    """Sum of squared differences of the first target.shape[-1] channels."""
    ct = target.shape[-1]
    return ((pred[..., :ct] - target) ** 2).sum()


def adam_step(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Bias-corrected Adam; returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ the network
def unet_shapes(cin: int = 8, cout: int = 8, chans=(32, 64, 128, 256, 256)):
    """(name, cin, cout, ks) of every convolution, in forward order."""
    out = []
    c_prev = cin
    for lvl, c in enumerate(chans):
        out.append((f"e{lvl}a", c_prev, c, 3))
        out.append((f"e{lvl}b", c, c, 3))
        c_prev = c
    for lvl in range(len(chans) - 2, -1, -1):
        c = chans[lvl]
        out.append((f"d{lvl}a", c_prev + c, c, 3))
        out.append((f"d{lvl}b", c, c, 3))
        c_prev = c
    out.append(("head", c_prev, cout, 1))
    return out


def init_params(seed: int, cin: int = 8, cout: int = 8, chans=(32, 64, 128, 256, 256)) -> dict:
    """He-normal weights [cout, ks*ks, cin] and zero biases (FP64)."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, ci, co, ks in unet_shapes(cin, cout, chans):
        std = (2.0 / (ci * ks * ks)) ** 0.5 if name != "head" else (1.0 / (ci * ks * ks)) ** 0.5
        p[name + ".w"] = torch.tensor(g.standard_normal((co, ks * ks, ci)) * std, dtype=D)
        p[name + ".b"] = torch.zeros(co, dtype=D)
    return p


def unet_forward(p: dict, x: torch.Tensor, levels: int = 5, bf16: bool = False) -> torch.Tensor:
    """x [n,h,w,cin] (h, w divisible by 2^(levels-1)) -> [n,h,w,cout]."""
    q = bf16_round if bf16 else (lambda t: t)

    def c(name, t, relu=True):
        return conv(q(t), q(p[name + ".w"]), p[name + ".b"], relu)

    skips = []
    h = x
    for lvl in range(levels):
        if lvl:
            h = pool2(q(h))
        h = c(f"e{lvl}b", c(f"e{lvl}a", h))
        skips.append(h)
    for lvl in range(levels - 2, -1, -1):
        h = torch.cat([up2(q(h)), skips[lvl]], dim=-1)
        h = c(f"d{lvl}b", c(f"d{lvl}a", h))
    return c("head", h, relu=False)


def unet_loss_grads(p: dict, x, target, levels: int = 5, bf16: bool = False):
    """Loss (sum of squared differences / (pixels * target channels)) and its
    gradient with respect to every parameter, by autograd in FP64."""
    ps = {k: v.detach().clone().requires_grad_(True) for k, v in p.items()}
    y = unet_forward(ps, x, levels, bf16)
    n = target.numel()
    loss = mse(y, target) / n
    g = torch.autograd.grad(loss, list(ps.values()))
    return loss.detach(), dict(zip(ps.keys(), [t.detach() for t in g])), y.detach()


def _conv_dx(gz, w, xshape):
    """Gradient of conv(x, w) with respect to x for the output gradient gz (NHWC)."""
    cout, taps, cin = w.shape
    ks = int(round(taps ** 0.5))
    wk = w.reshape(cout, ks, ks, cin).permute(0, 3, 1, 2)
    n, h, wd, _ = xshape
    return _nhwc(torch.nn.grad.conv2d_input((n, cin, h, wd), wk, _nchw(gz), padding=ks // 2))


def _conv_dw(x, gz, ks):
    """Gradient of conv(x, w) with respect to w [cout, ks*ks, cin]."""
    cin, cout = x.shape[-1], gz.shape[-1]
    g = torch.nn.grad.conv2d_weight(_nchw(x), (cout, cin, ks, ks), _nchw(gz), padding=ks // 2)
    return g.permute(0, 2, 3, 1).reshape(cout, ks * ks, cin)


def _pool2_adjoint(g):
    """Adjoint of 2x2 average pooling: every input pixel gets a quarter."""
    return torch.repeat_interleave(torch.repeat_interleave(g, 2, 1), 2, 2) / 4


def _up2_adjoint(g):
    """Adjoint of nearest 2x upsampling: the sum over each 2x2 block."""
    n, h, w, c = g.shape
    return g.reshape(n, h // 2, 2, w // 2, 2, c).sum(dim=(2, 4))


def unet_grads_stored(p: dict, x, target, levels: int = 5, store=bf16_round):
    """Loss, parameter gradients and output of the U-Net, with the backward
    pass written out layer by layer (chain rule through each convolution,
    ReLU, pooling, upsampling and concatenation) and `store` applied to every
    tensor where the HIP path keeps it in bfloat16: the weights, the input,
    every activation after bias and ReLU, every pooled activation, the
    gradient of the squared error, and every gradient after its ReLU mask.
    All other quantities (sums, the network output, gradients with respect to
    convolution inputs, and the skip and pooling gradients, which are added
    before the mask of the level they reach) stay in the tensors' own dtype.
    With store = identity this is the exact gradient, the same as
    unet_loss_grads."""
    s = store
    W = {k: (s(v) if k.endswith(".w") else v) for k, v in p.items()}

    def fwd(name, t, relu=True):
        return conv(t, W[name + ".w"], W[name + ".b"], relu)

    acts, skips = {}, []
    h = s(x)
    for lvl in range(levels):
        if lvl:
            h = s(pool2(h))
        a = s(fwd(f"e{lvl}a", h))
        b = s(fwd(f"e{lvl}b", a))
        acts[f"e{lvl}"] = (h, a, b)
        skips.append(b)
        h = b
    for lvl in range(levels - 2, -1, -1):
        cat = torch.cat([up2(h), skips[lvl]], dim=-1)
        a = s(fwd(f"d{lvl}a", cat))
        b = s(fwd(f"d{lvl}b", a))
        acts[f"d{lvl}"] = (cat, a, b)
        h = b
    y = fwd("head", h, relu=False)
    ct, n = target.shape[-1], target.numel()
    loss = mse(y, target) / n
    gy = torch.zeros_like(y)
    gy[..., :ct] = 2 * (y[..., :ct] - target) / n
    gy = s(gy)

    grads = {}

    def back(name, gz, inp):
        """Parameter gradients of one convolution; returns the gradient of its input."""
        w = W[name + ".w"]
        grads[name + ".w"] = _conv_dw(inp, gz, int(round(w.shape[1] ** 0.5)))
        grads[name + ".b"] = gz.sum(dim=(0, 1, 2))
        return _conv_dx(gz, w, inp.shape)

    g = back("head", gy, h)
    skip_g = {}
    for lvl in range(levels - 1):  # decoder, the level next to the head first
        cat, a, b = acts[f"d{lvl}"]
        g = back(f"d{lvl}b", s(g * (b > 0)), a)
        gcat = back(f"d{lvl}a", s(g * (a > 0)), cat)
        cu = cat.shape[-1] - skips[lvl].shape[-1]
        skip_g[lvl] = gcat[..., cu:]
        g = _up2_adjoint(gcat[..., :cu])
    for lvl in range(levels - 1, -1, -1):  # encoder, the deepest level first
        inp, a, b = acts[f"e{lvl}"]
        g = back(f"e{lvl}b", s(g * (b > 0)), a)
        gx = back(f"e{lvl}a", s(g * (a > 0)), inp)
        if lvl:
            g = _pool2_adjoint(gx) + skip_g[lvl - 1]
    return loss.detach(), grads, y.detach()
