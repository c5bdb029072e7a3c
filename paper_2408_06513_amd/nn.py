"""ctypes binding of the surrogate's layers (include/inim_nn.h).

Argument marshalling only: every layer runs in the HIP kernels of
libinim.so.  Tensors are torch device tensors in NHWC layout; BF16 tensors
are torch.bfloat16 (passed as their bit patterns), FP32 tensors float32.
"""
from __future__ import annotations

import ctypes

import torch

from . import capi

NN_EXPORTS = (
    "inim_nn_last_error", "inim_conv_forward", "inim_conv_backward_data", "inim_conv_workspace",
    "inim_conv_backward_weight", "inim_weight_transpose", "inim_f32_to_bf16", "inim_pool2", "inim_pool2_backward",
    "inim_upsample2_into", "inim_copy_channels_into", "inim_upsample2_backward", "inim_take_channels",
    "inim_relu_backward", "inim_mse", "inim_adam", "inim_nn_pack_density", "inim_nn_displacement", "inim_nn_field",
    "inim_nn_count_folds", "inim_nn_bin_moments", "inim_nn_pack_density_many", "inim_nn_field_many",
    "inim_nn_pack_input_many",
    "inim_concat_up2",
)

_bound = None


def lib() -> ctypes.CDLL:
    global _bound
    L = capi.lib()
    if _bound is L:
        return L
    vp, sz, i32, i64, f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.inim_nn_last_error.argtypes = []
    L.inim_nn_last_error.restype = ctypes.c_char_p
    sig = {
        "inim_conv_forward": [vp, i32, i32, i32, i32, vp, vp, i32, i32, i32, vp, vp, vp, sz, vp],
        "inim_conv_backward_data": [vp, i32, i32, i32, i32, vp, i32, i32, vp, vp, sz, vp],
        "inim_conv_workspace": [i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)],
        "inim_conv_backward_weight": [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, sz, vp],
        "inim_weight_transpose": [vp, i32, i32, i32, vp, vp],
        "inim_f32_to_bf16": [vp, i64, vp, vp],
        "inim_pool2": [vp, i32, i32, i32, i32, vp, vp],
        "inim_pool2_backward": [vp, i32, i32, i32, i32, vp, i32, vp],
        "inim_upsample2_into": [vp, i32, i32, i32, i32, vp, i32, i32, vp],
        "inim_copy_channels_into": [vp, i64, i32, vp, i32, i32, vp],
        "inim_concat_up2": [vp, i32, i32, i32, i32, vp, i32, vp, vp],
        "inim_upsample2_backward": [vp, i32, i32, i32, i32, i32, vp, vp],
        "inim_take_channels": [vp, i64, i32, i32, i32, vp, i32, vp],
        "inim_relu_backward": [vp, vp, i64, vp, vp],
        "inim_mse": [vp, i32, vp, i32, i64, vp, vp, vp, sz, vp],
        "inim_adam": [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp, vp],
        "inim_nn_pack_density": [vp, i32, f32, i32, vp, vp],
        "inim_nn_pack_density_many": [vp, i32, i32, vp, i32, vp, vp],
        "inim_nn_pack_input_many": [vp, vp, i32, i32, vp, i32, vp, vp],
        "inim_nn_field_many": [vp, i32, i32, i32, i32, vp, vp, vp],
        "inim_nn_displacement": [vp, i32, vp, vp],
        "inim_nn_field": [vp, i32, i32, i32, vp, vp, vp],
        "inim_nn_count_folds": [vp, i32, vp, vp],
        "inim_nn_bin_moments": [vp, i32, i32, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _bound = L
    return L


def _check(status: int):
    if status != capi.OK:
        msg = lib().inim_nn_last_error().decode() or capi.strerror(status)
        raise capi._ERR.get(status, capi.InimError)(status, msg)


def _p(t):
    """The device address of a contiguous device tensor (None stays NULL)."""
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("the layers take contiguous device tensors")
    return ctypes.c_void_p(t.data_ptr())


def _s(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _bf(t, name):
    if t is not None and t.dtype != torch.bfloat16:
        raise TypeError(f"{name} must be bfloat16")


def _f(t, name):
    if t is not None and t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")


def conv_workspace(imgs, h, w, cin, cout, ks) -> int:
    n = ctypes.c_size_t()
    _check(lib().inim_conv_workspace(imgs, h, w, cin, cout, ks, ctypes.byref(n)))
    return n.value


def _work(work, need, dev):
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    return work


def conv_forward(x, w, bias=None, relu=False, y16=None, y32=None, work=None):
    """x: [imgs, h, w, cin] bf16; w: [cout, ks*ks, cin] bf16 (ks from its shape)."""
    _bf(x, "x"), _bf(w, "w"), _f(bias, "bias"), _bf(y16, "y16"), _f(y32, "y32")
    imgs, h, wd, cin = x.shape
    cout, taps, cin2 = w.shape
    ks = int(round(taps ** 0.5))
    assert cin2 == cin and ks * ks == taps and x.is_contiguous() and w.is_contiguous()
    work = _work(work, conv_workspace(imgs, h, wd, cin, cout, ks), x.device)
    _check(lib().inim_conv_forward(_p(x), imgs, h, wd, cin, _p(w), _p(bias), cout, ks, 1 if relu else 0, _p(y16),
                                   _p(y32), _p(work), work.numel(), _s(x)))
    return y16, y32


def conv_backward_data(dy, wT, dx, work=None):
    """dy: [imgs, h, w, cout] bf16; wT: [cin, ks*ks, cout] bf16; dx: [imgs, h, w, cin] f32."""
    _bf(dy, "dy"), _bf(wT, "wT"), _f(dx, "dx")
    imgs, h, wd, cout = dy.shape
    cin, taps, cout2 = wT.shape
    ks = int(round(taps ** 0.5))
    assert cout2 == cout and dx.shape == (imgs, h, wd, cin)
    work = _work(work, conv_workspace(imgs, h, wd, cin, cout, ks), dy.device)
    _check(lib().inim_conv_backward_data(_p(dy), imgs, h, wd, cin, _p(wT), cout, ks, _p(dx), _p(work), work.numel(),
                                         _s(dy)))
    return dx


def conv_backward_weight(dy, x, ks, dw, db=None, work=None):
    _bf(dy, "dy"), _bf(x, "x"), _f(dw, "dw"), _f(db, "db")
    imgs, h, wd, cout = dy.shape
    cin = x.shape[3]
    work = _work(work, conv_workspace(imgs, h, wd, cin, cout, ks), dy.device)
    _check(lib().inim_conv_backward_weight(_p(dy), _p(x), imgs, h, wd, cin, cout, ks, _p(dw), _p(db), _p(work),
                                           work.numel(), _s(dy)))
    return dw, db


def weight_transpose(w, wT):
    cout, taps, cin = w.shape
    _check(lib().inim_weight_transpose(_p(w), cout, int(round(taps ** 0.5)), cin, _p(wT), _s(w)))
    return wT


def to_bf16(a, b):
    _check(lib().inim_f32_to_bf16(_p(a), a.numel(), _p(b), _s(a)))
    return b


def pool2(x, y):
    imgs, h, w, c = x.shape
    _check(lib().inim_pool2(_p(x), imgs, h, w, c, _p(y), _s(x)))
    return y


def pool2_backward(dy, dx, accumulate=False):
    imgs, h, w, c = dx.shape
    _check(lib().inim_pool2_backward(_p(dy), imgs, h, w, c, _p(dx), 1 if accumulate else 0, _s(dy)))
    return dx


def upsample2_into(x, y, c0=0):
    imgs, h, w, c = x.shape
    _check(lib().inim_upsample2_into(_p(x), imgs, h, w, c, _p(y), y.shape[3], c0, _s(x)))
    return y


def concat_up2(a, b, y):
    """y [imgs, 2h, 2w, ca + cb] = [upsample2(a) | b] in one launch."""
    imgs, h, w, ca = a.shape
    assert b.shape == (imgs, 2 * h, 2 * w, b.shape[3]) and y.shape == (imgs, 2 * h, 2 * w, ca + b.shape[3])
    _check(lib().inim_concat_up2(_p(a), imgs, h, w, ca, _p(b), b.shape[3], _p(y), _s(y)))
    return y


def copy_channels_into(x, y, c0):
    pixels = x.numel() // x.shape[-1]
    _check(lib().inim_copy_channels_into(_p(x), pixels, x.shape[-1], _p(y), y.shape[-1], c0, _s(x)))
    return y


def upsample2_backward(dy, da):
    imgs, h, w, ca = da.shape
    _check(lib().inim_upsample2_backward(_p(dy), imgs, h, w, dy.shape[3], ca, _p(da), _s(dy)))
    return da


def take_channels(dy, c0, out, accumulate=False):
    pixels = out.numel() // out.shape[-1]
    _check(lib().inim_take_channels(_p(dy), pixels, dy.shape[-1], c0, out.shape[-1], _p(out),
                                    1 if accumulate else 0, _s(dy)))
    return out


def relu_backward(g, act, g16):
    _check(lib().inim_relu_backward(_p(g), _p(act), g.numel(), _p(g16), _s(g)))
    return g16


def mse(pred, target, loss, grad=None, work=None):
    """pred [..., cp] f32, target [..., ct] f32 (ct <= cp); loss: 1-element f32."""
    pixels = pred.numel() // pred.shape[-1]
    if work is None:
        work = torch.empty(1024, dtype=torch.uint8, device=pred.device)
    _check(lib().inim_mse(_p(pred), pred.shape[-1], _p(target), target.shape[-1], pixels, _p(loss), _p(grad), _p(work),
                          work.numel(), _s(pred)))
    return loss


def pack_density(density, scale, x):
    """density [res, res] f32 -> x [res, res, c] bf16 (channel 0 = density * scale)."""
    _check(lib().inim_nn_pack_density(_p(density), density.shape[0], float(scale), x.shape[-1], _p(x), _s(x)))
    return x


def pack_density_many(density, scales, x):
    """density [k, res, res] f32 -> x [k, res, res, c] bf16 (channel 0 of
    raster q = density[q] * scales[q])."""
    k = density.shape[0]
    sc = (ctypes.c_float * k)(*[float(v) for v in scales])
    _check(lib().inim_nn_pack_density_many(_p(density), k, density.shape[1], sc, x.shape[-1], _p(x), _s(x)))
    return x


def pack_input_many(density, field, scales, x):
    """density [k, res, res] f32 and the method's one-step field [k, res, res, 2]
    -> x [k, res, res, c] bf16: channel 0 density[q] * scales[q], channels 1-2
    the field's displacement from the texel centres times 64."""
    k = density.shape[0]
    sc = (ctypes.c_float * k)(*[float(v) for v in scales])
    _check(lib().inim_nn_pack_input_many(_p(density), _p(field), k, density.shape[1], sc, x.shape[-1], _p(x), _s(x)))
    return x


def displacement(probe, res, out):
    _check(lib().inim_nn_displacement(_p(probe), res, _p(out), _s(out)))
    return out


def field(y, res, out, radius=0, work=None):
    if work is None:
        work = torch.empty_like(out)
    _check(lib().inim_nn_field(_p(y), y.shape[-1], res, radius, _p(out), _p(work), _s(out)))
    return out


def field_many(y, res, out, radius=0, work=None):
    """field for a stack of outputs: y [k, res, res, c] -> out [k, res, res, 2]."""
    if work is None:
        work = torch.empty_like(out)
    _check(lib().inim_nn_field_many(_p(y), y.shape[0], y.shape[-1], res, radius, _p(out), _p(work), _s(out)))
    return out


def count_folds(field_t, res, count):
    _check(lib().inim_nn_count_folds(_p(field_t), res, _p(count), _s(count)))
    return count


def bin_moments(counts, res, bin_px, out):
    _check(lib().inim_nn_bin_moments(_p(counts), res, bin_px, _p(out), _s(out)))
    return out


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, w16=None):
    _check(lib().inim_adam(_p(w), _p(g), _p(m), _p(v), w.numel(), lr, b1, b2, eps, step, _p(w16), _s(w)))
    return w
