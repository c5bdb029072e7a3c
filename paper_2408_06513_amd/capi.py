"""Thin ctypes binding of libinim.so (include/inim.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Tensors are torch CUDA (HIP) tensors used as device memory; work is enqueued
on the current torch stream of the tensor's device.  The names mirror the C
entry points without the ``inim_`` prefix.  If the library is not built the
first call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinim.so")

OK, EINVAL, EDOMAIN, ERANGE, EWORKSPACE, EHIP = range(6)
U32, F32 = 0, 1
ALPHA, BETA, GAMMA, DELTA = 1, 2, 4, 8
ALPHA_T, BETA_T, GAMMA_T, DELTA_T = 16, 32, 64, 128
MASK_MIN = ALPHA | ALPHA_T
MASK_ALL = 0xFF
PLANES = ("alpha", "beta", "gamma", "delta", "alpha_t", "beta_t", "gamma_t", "delta_t")
STAGES = ("sort_unsort", "smooth_aggregate", "inim_scans", "inim_deform", "advect_splat", "total")

EXPORTS = (
    "inim_default_params", "inim_strerror", "inim_last_error", "inim_workspace_size",
    "inim_inim_workspace_size", "inim_rasterize", "inim_inim_u32", "inim_inim_f32",
    "inim_deform", "inim_advect", "inim_regularize", "inim_regularize_timed", "inim_sync_status",
    "inim_graph_create", "inim_graph_destroy", "inim_regularize_graph", "inim_regularize_probes",
    "inim_batch_workspace_size", "inim_regularize_batch", "inim_batch_autotune",
    "inim_rasterize_many", "inim_advect_many", "inim_regularize_noalloc",
    "inim_deform_density_workspace_size", "inim_deform_density",
)


class InimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class InvalidArgument(InimError, ValueError):
    pass


class DomainError(InimError, ValueError):
    pass


class SizeRangeError(InimError, OverflowError):
    pass


class WorkspaceError(InimError):
    pass


class HipError(InimError):
    pass


_ERR = {EINVAL: InvalidArgument, EDOMAIN: DomainError, ERANGE: SizeRangeError,
        EWORKSPACE: WorkspaceError, EHIP: HipError}


class Params(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_int32), ("sigma", ctypes.c_float), ("d0", ctypes.c_double)]


class BatchConfig(ctypes.Structure):
    """Launch shape of a batched call (inim_batch_config)."""
    _fields_ = [("waves_per_block", ctypes.c_int32), ("order", ctypes.c_int32)]

    def __repr__(self):
        return f"BatchConfig(waves_per_block={self.waves_per_block}, order={self.order})"


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libinim.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(python -m paper_2408_06513_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, u32, f64 = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_double)
    pp = ctypes.POINTER(Params)
    L.inim_default_params.argtypes = [pp]
    L.inim_default_params.restype = None
    L.inim_strerror.argtypes = [ctypes.c_int]
    L.inim_strerror.restype = ctypes.c_char_p
    L.inim_last_error.argtypes = []
    L.inim_last_error.restype = ctypes.c_char_p
    L.inim_workspace_size.argtypes = [i32, i64, pp, ctypes.POINTER(sz)]
    L.inim_inim_workspace_size.argtypes = [i32, ctypes.c_int, ctypes.POINTER(sz)]
    L.inim_rasterize.argtypes = [vp, i64, i32, pp, vp, vp, vp, sz, vp]
    L.inim_inim_u32.argtypes = [vp, i32, u32, vp, vp, vp, sz, vp]
    L.inim_inim_f32.argtypes = [vp, i32, u32, vp, vp, vp, sz, vp]
    L.inim_deform.argtypes = [vp, vp, ctypes.c_int, vp, i32, f64, vp, vp]
    L.inim_advect.argtypes = [vp, i32, vp, i64, vp, sz, vp]
    L.inim_deform_density_workspace_size.argtypes = [i32, ctypes.POINTER(sz)]
    L.inim_deform_density.argtypes = [vp, i32, f64, vp, vp, sz, vp]
    L.inim_rasterize_many.argtypes = [vp, vp, i32, i32, pp, vp, vp, vp, sz, vp]
    L.inim_advect_many.argtypes = [vp, i32, vp, vp, i32, vp, sz, vp]
    L.inim_regularize.argtypes = [vp, i64, i32, i32, pp, vp, sz, vp]
    L.inim_regularize_timed.argtypes = [vp, i64, i32, i32, pp, vp, sz, vp, ctypes.POINTER(f64)]
    L.inim_sync_status.argtypes = [vp, vp]
    L.inim_graph_create.argtypes = [ctypes.POINTER(vp)]
    L.inim_graph_destroy.argtypes = [vp]
    L.inim_regularize_graph.argtypes = [vp, i64, i32, i32, pp, vp, sz, vp, vp]
    L.inim_regularize_probes.argtypes = [vp, i64, vp, i64, i32, i32, pp, vp, sz, vp]
    L.inim_regularize_noalloc.argtypes = [vp, i64, i32, i32, pp, vp, vp]
    bp = ctypes.POINTER(BatchConfig)
    L.inim_batch_workspace_size.argtypes = [vp, vp, vp, i32, pp, ctypes.POINTER(sz)]
    L.inim_regularize_batch.argtypes = [vp, vp, vp, i32, i32, pp, bp, vp, sz, vp, vp]
    L.inim_batch_autotune.argtypes = [vp, vp, vp, i32, i32, pp, vp, sz, vp, bp, ctypes.POINTER(f64)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("inim_default_params", "inim_strerror", "inim_last_error"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        msg = lib().inim_last_error().decode() or lib().inim_strerror(status).decode()
        raise _ERR.get(status, InimError)(status, msg)


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def params(radius: int = 8, sigma: float | None = None, d0: float | None = None) -> Params:
    p = Params()
    lib().inim_default_params(ctypes.byref(p))
    p.radius = int(radius)
    p.sigma = float(sigma) if sigma is not None else 0.0
    p.d0 = float(d0) if d0 is not None else -1.0
    return p


def strerror(status: int) -> str:
    return lib().inim_strerror(status).decode()


def workspace_size(res: int, n: int, radius: int = 8, sigma=None, d0=None) -> int:
    out = ctypes.c_size_t()
    p = params(radius, sigma, d0)
    _check(lib().inim_workspace_size(res, n, ctypes.byref(p), ctypes.byref(out)))
    return out.value


def inim_workspace_size(res: int, dtype: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().inim_inim_workspace_size(res, dtype, ctypes.byref(out)))
    return out.value


def workspace(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer; torch's allocator aligns it to 512 bytes."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _xy(xy: torch.Tensor):
    if not (xy.is_cuda and xy.dtype == torch.float32 and xy.dim() == 2 and xy.shape[1] == 2
            and xy.is_contiguous()):
        raise ValueError("xy must be a contiguous float32 [n, 2] device tensor")
    return xy.shape[0]


def rasterize(xy: torch.Tensor, res: int, radius: int = 8, sigma=None, counts=None, density=None,
              ws=None, want_density: bool = True, check: bool = True):
    """Counts (uint32 [res, res]) and smoothed density (float32 [res, res]).
    With check=True the call synchronises and raises DomainError when a
    sample is NaN or outside the unit square (the rasters are then left
    incomplete); pass False under graph capture and call sync_status(ws)."""
    n = _xy(xy)
    dev = xy.device
    if counts is None:
        counts = torch.empty((res, res), dtype=torch.uint32, device=dev)
    if density is None and want_density:
        density = torch.empty((res, res), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(256, dev)
    p = params(radius, sigma)
    _check(lib().inim_rasterize(_ptr(xy), n, res, ctypes.byref(p), _ptr(counts), _ptr(density),
                                _ptr(ws), ws.numel(), _stream(xy)))
    if check:
        _check(sync_status(ws))
    return counts, density, ws


def inim(img: torch.Tensor, mask: int = MASK_MIN, planes=None, marg=None, ws=None, want_marg=True):
    """Integral images of a square uint32 or float32 raster.
    Returns (planes [popcount(mask), res, res], marg [6 res - 1] float64)."""
    if not (img.is_cuda and img.dim() == 2 and img.shape[0] == img.shape[1] and img.is_contiguous()):
        raise ValueError("img must be a contiguous square device raster")
    res = img.shape[0]
    if img.dtype == torch.uint32:
        dt, fn = U32, lib().inim_inim_u32
    elif img.dtype == torch.float32:
        dt, fn = F32, lib().inim_inim_f32
    else:
        raise ValueError("img must be uint32 or float32")
    k = bin(mask & 0xFF).count("1")
    if planes is None and k > 0:
        planes = torch.empty((k, res, res), dtype=img.dtype, device=img.device)
    if marg is None and want_marg:
        marg = torch.empty(6 * res - 1, dtype=torch.float64, device=img.device)
    if ws is None:
        ws = workspace(inim_workspace_size(res, dt), img.device)
    _check(fn(_ptr(img), res, mask, _ptr(planes), _ptr(marg), _ptr(ws), ws.numel(), _stream(img)))
    return planes, marg


def split_marg(marg, res: int) -> dict:
    M = 2 * res - 1
    return {"X": marg[:res], "Y": marg[res:2 * res], "U": marg[2 * res:2 * res + M],
            "V": marg[2 * res + M:2 * res + 2 * M], "C": marg[2 * res + 2 * M]}


def deform(alpha: torch.Tensor, alpha_t: torch.Tensor, marg: torch.Tensor, d0: float, field=None):
    """Per-texel deformation [res, res, 2] from alpha, alpha_t and the marginals."""
    res = alpha.shape[-1]
    dt = U32 if alpha.dtype == torch.uint32 else F32
    if field is None:
        field = torch.empty((res, res, 2), dtype=torch.float32, device=alpha.device)
    _check(lib().inim_deform(_ptr(alpha), _ptr(alpha_t), dt, _ptr(marg), res, float(d0), _ptr(field),
                             _stream(alpha)))
    return field


def deform_density_workspace_size(res: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().inim_deform_density_workspace_size(res, ctypes.byref(b)))
    return b.value


def deform_density(density: torch.Tensor, d0: float, field=None, ws=None) -> torch.Tensor:
    """The deformation field [res, res, 2] of a float density [res, res] with
    background d0: one iteration's integral images and map, fused."""
    res = density.shape[-1]
    if not (density.is_cuda and density.dtype == torch.float32 and density.is_contiguous()
            and tuple(density.shape) == (res, res)):
        raise ValueError("density must be a contiguous float32 [res, res] device tensor")
    if field is None:
        field = torch.empty((res, res, 2), dtype=torch.float32, device=density.device)
    elif not (field.is_cuda and field.dtype == torch.float32 and field.is_contiguous()
              and tuple(field.shape) == (res, res, 2)):
        raise ValueError("field must be a contiguous float32 [res, res, 2] device tensor")
    if ws is None:
        ws = workspace(deform_density_workspace_size(res), density.device)
    _check(lib().inim_deform_density(_ptr(density), res, float(d0), _ptr(field), _ptr(ws), ws.numel(),
                                     _stream(density)))
    return field


def advect(field: torch.Tensor, xy: torch.Tensor, ws=None, check: bool = True) -> torch.Tensor:
    """Bilinear advection of xy (in place) through field [res, res, 2].  With
    check=True the call synchronises and raises DomainError when a sample is
    NaN or outside the unit square (xy is then left unmoved); pass False
    under graph capture and call sync_status(ws)."""
    n = _xy(xy)
    res = field.shape[0]
    if ws is None:
        ws = workspace(256, xy.device)
    _check(lib().inim_advect(_ptr(field), res, _ptr(xy), n, _ptr(ws), ws.numel(), _stream(xy)))
    if check:
        _check(sync_status(ws))
    return xy


def _sets(xys):
    """Host arrays of the device pointers and sizes of several sample sets."""
    ns = [_xy(t) for t in xys]
    if len({t.device for t in xys}) > 1:
        raise ValueError("all sets must be on one device")
    k = len(xys)
    return (ctypes.c_void_p * k)(*[t.data_ptr() for t in xys]), (ctypes.c_int64 * k)(*ns), k


def rasterize_many(xys, res: int, radius: int = 8, sigma=None, counts=None, density=None, ws=None,
                   want_density: bool = True, check: bool = True):
    """rasterize for several sample sets in shared launches: counts (uint32
    [k, res, res]) and densities (float32 [k, res, res]), raster q for xys[q].
    One NaN or out-of-range sample in any set stops every set; check=True
    synchronises and raises DomainError then."""
    a, n, k = _sets(xys)
    dev = xys[0].device
    if counts is None:
        counts = torch.empty((k, res, res), dtype=torch.uint32, device=dev)
    if density is None and want_density:
        density = torch.empty((k, res, res), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(256, dev)
    p = params(radius, sigma)
    _check(lib().inim_rasterize_many(a, n, k, res, ctypes.byref(p), _ptr(counts), _ptr(density), _ptr(ws),
                                     ws.numel(), _stream(ws)))
    if check:
        _check(sync_status(ws))
    return counts, density, ws


def advect_many(field: torch.Tensor, xys, ws=None, check: bool = True):
    """advect for several sample sets in shared launches: xys[q] moves (in
    place) through field[q] ([k, res, res, 2]).  One NaN or out-of-range
    sample in any set leaves every set unmoved; check=True synchronises and
    raises DomainError then."""
    a, n, k = _sets(xys)
    res = field.shape[1]
    if ws is None:
        ws = workspace(256, xys[0].device)
    _check(lib().inim_advect_many(_ptr(field), res, a, n, k, _ptr(ws), ws.numel(), _stream(ws)))
    if check:
        _check(sync_status(ws))
    return xys


def regularize(xy: torch.Tensor, res: int, iters: int, radius: int = 8, sigma=None, d0=None,
               ws=None, check: bool = True) -> torch.Tensor:
    """The iterated regularisation, in place on xy.  With check=True the call
    synchronises and raises DomainError for NaN / out-of-range samples."""
    n = _xy(xy)
    p = params(radius, sigma, d0)
    if ws is None:
        ws = workspace(workspace_size(res, n, radius, sigma, d0), xy.device)
    _check(lib().inim_regularize(_ptr(xy), n, res, iters, ctypes.byref(p), _ptr(ws), ws.numel(),
                                 _stream(xy)))
    if check:
        _check(sync_status(ws))
    return xy


def regularize_noalloc(xy: torch.Tensor, res: int, iters: int, radius: int = 8, sigma=None, d0=None,
                       status: torch.Tensor | None = None, check: bool = False) -> torch.Tensor:
    """regularize on the library's static per-GPU scratch (no workspace; the
    call allocates nothing).  status: an int32 device tensor of at least one
    element for the call's status word, or None; check=True needs it."""
    n = _xy(xy)
    if status is not None and not (status.is_cuda and status.dtype == torch.int32 and status.numel() >= 1):
        raise ValueError("status must be an int32 device tensor")
    if check and status is None:
        raise ValueError("check=True needs a status tensor")
    p = params(radius, sigma, d0)
    _check(lib().inim_regularize_noalloc(_ptr(xy), n, res, iters, ctypes.byref(p), _ptr(status), _stream(xy)))
    if check:
        _check(sync_status(status))
    return xy


def regularize_probes(xy: torch.Tensor, probe: torch.Tensor, res: int, iters: int, radius: int = 8, sigma=None,
                      d0=None, ws=None, check: bool = True) -> tuple[torch.Tensor, torch.Tensor]:
    """regularize, also moving the probe points (float32 [m, 2], same device)
    by every iteration's deformation without splatting them: started at the
    texel centres they return the composite map on the texel lattice."""
    n = _xy(xy)
    m = _xy(probe)
    if probe.device != xy.device:
        raise ValueError("probe and xy must be on the same device")
    p = params(radius, sigma, d0)
    if ws is None:
        ws = workspace(workspace_size(res, n, radius, sigma, d0), xy.device)
    _check(lib().inim_regularize_probes(_ptr(xy), n, _ptr(probe), m, res, iters, ctypes.byref(p), _ptr(ws),
                                        ws.numel(), _stream(xy)))
    if check:
        _check(sync_status(ws))
    return xy, probe


def regularize_timed(xy: torch.Tensor, res: int, iters: int, radius: int = 8, sigma=None, d0=None,
                     ws=None) -> dict:
    """regularize with per-stage HIP-event timings (milliseconds, summed over iterations)."""
    n = _xy(xy)
    p = params(radius, sigma, d0)
    if ws is None:
        ws = workspace(workspace_size(res, n, radius, sigma, d0), xy.device)
    ms = (ctypes.c_double * 6)()
    _check(lib().inim_regularize_timed(_ptr(xy), n, res, iters, ctypes.byref(p), _ptr(ws), ws.numel(),
                                       _stream(xy), ms))
    return dict(zip(STAGES, list(ms)))


class Graph:
    """Handle of inim_regularize_graph: replays one captured regularisation."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().inim_graph_create(ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().inim_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def regularize_graph(xy: torch.Tensor, res: int, iters: int, graph: Graph, ws: torch.Tensor, radius: int = 8,
                     sigma=None, d0=None, check: bool = False) -> torch.Tensor:
    """regularize through a captured HIP graph (same results)."""
    n = _xy(xy)
    p = params(radius, sigma, d0)
    _check(lib().inim_regularize_graph(_ptr(xy), n, res, iters, ctypes.byref(p), _ptr(ws), ws.numel(),
                                       graph.handle, _stream(xy)))
    if check:
        _check(sync_status(ws))
    return xy


def _batch_arrays(xys, res):
    if len(xys) != len(res):
        raise ValueError("one raster size per plot")
    ns = [_xy(t) for t in xys]
    if len({t.device for t in xys}) > 1:
        raise ValueError("all plots must be on one device")
    k = len(xys)
    return ((ctypes.c_void_p * k)(*[t.data_ptr() for t in xys]), (ctypes.c_int64 * k)(*ns),
            (ctypes.c_int32 * k)(*[int(r) for r in res]), k)


def batch_workspace_size(xys, res, radius: int = 8, sigma=None, d0=None) -> int:
    a, n, r, k = _batch_arrays(xys, res)
    p = params(radius, sigma, d0)
    out = ctypes.c_size_t()
    _check(lib().inim_batch_workspace_size(a, n, r, k, ctypes.byref(p), ctypes.byref(out)))
    return out.value


def regularize_batch(xys, res, iters: int, radius: int = 8, sigma=None, d0=None, cfg: BatchConfig | None = None,
                     ws=None, graph: "Graph | None" = None, check: bool = True):
    """Regularises every plot (xys[k]: float32 [n_k, 2] on one device, raster
    res[k]) in shared launches, in place; same results as one regularize per plot."""
    a, n, r, k = _batch_arrays(xys, res)
    p = params(radius, sigma, d0)
    if ws is None:
        ws = workspace(batch_workspace_size(xys, res, radius, sigma, d0), xys[0].device)
    _check(lib().inim_regularize_batch(a, n, r, k, iters, ctypes.byref(p), ctypes.byref(cfg) if cfg else None,
                                       _ptr(ws), ws.numel(), graph.handle if graph else None, _stream(ws)))
    if check:
        _check(sync_status(ws))
    return xys


def batch_autotune(xys, res, iters: int, radius: int = 8, sigma=None, d0=None, ws=None) -> tuple[BatchConfig, float]:
    """Times every launch shape of regularize_batch on these plots (the plots
    are not modified); returns the fastest and its time in milliseconds."""
    a, n, r, k = _batch_arrays(xys, res)
    p = params(radius, sigma, d0)
    if ws is None:
        ws = workspace(batch_workspace_size(xys, res, radius, sigma, d0), xys[0].device)
    best = BatchConfig()
    ms = ctypes.c_double()
    _check(lib().inim_batch_autotune(a, n, r, k, iters, ctypes.byref(p), _ptr(ws), ws.numel(), _stream(ws),
                                     ctypes.byref(best), ctypes.byref(ms)))
    return best, ms.value


def sync_status(ws: torch.Tensor) -> int:
    return lib().inim_sync_status(_ptr(ws), _stream(ws))
