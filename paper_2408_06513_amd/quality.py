"""ctypes binding of the layout quality measures (include/inim_quality.h).

The kernels return exact integer sums; the measures of Sec. 6 (numerical
tests) are the closed-form ratios of those sums given in the header.
Positions are float32 device tensors [n, 2].
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import capi

QUALITY_EXPORTS = ("inim_quality_last_error", "inim_quality_bins", "inim_quality_ordering", "inim_quality_trust")

_bound = None


def lib() -> ctypes.CDLL:
    global _bound
    L = capi.lib()
    if _bound is L:
        return L
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.inim_quality_last_error.argtypes = []
    L.inim_quality_last_error.restype = ctypes.c_char_p
    for name, args in {
        "inim_quality_bins": [vp, i32, i32, vp, vp],
        "inim_quality_ordering": [vp, vp, i32, vp, vp],
        "inim_quality_trust": [vp, vp, i32, i32, vp, vp],
    }.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _bound = L
    return L


def _check(status: int):
    if status != capi.OK:
        msg = lib().inim_quality_last_error().decode() or capi.strerror(status)
        raise capi._ERR.get(status, capi.InimError)(status, msg)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _s(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _pts(t, name):
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 2 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 [n, 2] tensor")
    return t.shape[0]


def _counter(n, dev):
    return torch.zeros(n, dtype=torch.int64, device=dev)


def bin_stats(counts: torch.Tensor, bin_px: int = 4, out=None) -> torch.Tensor:
    """Device int64 [3]: occupied texels, samples, sum of squared bin counts
    of a uint32 [res, res] count raster (added into `out` when given)."""
    res = counts.shape[0]
    if out is None:
        out = _counter(3, counts.device)
    _check(lib().inim_quality_bins(_p(counts), res, bin_px, _p(out), _s(counts)))
    return out


def ordering_counts(a: torch.Tensor, b: torch.Tensor, out=None) -> torch.Tensor:
    """Device int64 [3]: pairs kept along x, along y, along both."""
    n = _pts(a, "a")
    if _pts(b, "b") != n:
        raise ValueError("a and b differ in length")
    if out is None:
        out = _counter(3, a.device)
    _check(lib().inim_quality_ordering(_p(a), _p(b), n, _p(out), _s(a)))
    return out


def trust_penalty(a: torch.Tensor, b: torch.Tensor, k: int, out=None) -> torch.Tensor:
    """Device int64 [1]: the trustworthiness penalty sum."""
    n = _pts(a, "a")
    if _pts(b, "b") != n:
        raise ValueError("a and b differ in length")
    if out is None:
        out = _counter(1, a.device)
    _check(lib().inim_quality_trust(_p(a), _p(b), n, k, _p(out), _s(a)))
    return out


def texel_counts(xy: torch.Tensor, res: int) -> torch.Tensor:
    counts = torch.empty((res, res), dtype=torch.uint32, device=xy.device)
    capi.rasterize(xy, res, radius=0, counts=counts, want_density=False)
    return counts


def density_measures(xy: torch.Tensor, res: int, bin_px: int = 4) -> dict:
    """The regularity measure (std of the bin counts) and overplotting of a
    layout shown on a res x res raster."""
    occ, s1, s2 = bin_stats(texel_counts(xy, res), bin_px).tolist()
    nbins = (res // bin_px) ** 2
    mean = s1 / nbins
    n = xy.shape[0]
    return {"bin_std": math.sqrt(max(s2 / nbins - mean * mean, 0.0)),
            "overplotting": (n - occ) / n if n else 0.0}


def trustworthiness(a: torch.Tensor, b: torch.Tensor, k: int = 7) -> float:
    n = a.shape[0]
    return 1.0 - 2.0 * trust_penalty(a, b, k).item() / (n * k * (2 * n - 3 * k - 1))


def orthogonal_ordering(a: torch.Tensor, b: torch.Tensor) -> float:
    n = a.shape[0]
    return ordering_counts(a, b)[2].item() / (n * (n - 1) // 2)
