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
