"""Python access to the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this; the library's product path never does.  Arrays are
numpy float64; positions are ``[n, 2]`` (x, y), rasters ``[N, N]`` indexed
``[j, i]`` (row j is y, column i is x, origin top-left).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PLANES = ("alpha", "beta", "gamma", "delta", "alpha_t", "beta_t", "gamma_t", "delta_t")
MASK_ALL = 0xFF
MASK_MIN = 0x11

OK, EINVAL, EDOMAIN = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint, ctypes.c_double
        L.oracle_check_points.argtypes = [dp, i64]
        L.oracle_counts.argtypes = [dp, i64, i32, dp]
        L.oracle_blur.argtypes = [dp, i32, i32, f64, dp]
        L.oracle_planes.argtypes = [dp, i32, u32, dp, dp]
        L.oracle_map.argtypes = [dp, i32, dp]
        L.oracle_defect.argtypes = [i32, f64, dp]
        L.oracle_deform.argtypes = [dp, i32, f64, dp]
        L.oracle_advect.argtypes = [dp, i32, dp, i64]
        L.oracle_regularize.argtypes = [dp, i64, i32, i32, i32, f64, f64]
        L.oracle_regularize_probes.argtypes = [dp, i64, dp, i64, i32, i32, i32, f64, f64]
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_set_threads.restype = i32
        L.oracle_set_threads(1)
        _lib = L
    return _lib


def set_threads(k: int) -> int:
    """Threads of the oracle's parallel loops (results do not depend on it);
    returns the number in force.  The default is one."""
    return int(lib().oracle_set_threads(int(k)))


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__("oracle status %d" % status)
        self.status = status


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(st: int):
    if st != OK:
        raise OracleError(st)


def counts(xy, res: int) -> np.ndarray:
    xy = _f64(xy).reshape(-1, 2)
    out = np.empty((res, res))
    _check(lib().oracle_counts(_p(xy), xy.shape[0], res, _p(out)))
    return out


def blur(c, radius: int = 8, sigma: float = 0.0) -> np.ndarray:
    c = _f64(c)
    out = np.empty_like(c)
    _check(lib().oracle_blur(_p(c), c.shape[0], radius, sigma, _p(out)))
    return out


def planes(d, mask: int = MASK_ALL):
    """Returns (planes [popcount(mask), N, N], marg dict with X, Y, U, V, C)."""
    d = _f64(d)
    N = d.shape[0]
    k = bin(mask & 0xFF).count("1")
    out = np.empty((k, N, N))
    M = 2 * N - 1
    marg = np.empty(2 * N + 2 * M + 1)
    _check(lib().oracle_planes(_p(d), N, mask, _p(out), _p(marg)))
    return out, split_marg(marg, N)


def split_marg(marg: np.ndarray, N: int) -> dict:
    M = 2 * N - 1
    return {"X": marg[:N], "Y": marg[N:2 * N], "U": marg[2 * N:2 * N + M],
            "V": marg[2 * N + M:2 * N + 2 * M], "C": float(marg[2 * N + 2 * M])}


def tmap(d) -> np.ndarray:
    """t(p; d) of eq. (map) at every texel centre: [N, N, 2]."""
    d = _f64(d)
    N = d.shape[0]
    out = np.empty((N, N, 2))
    _check(lib().oracle_map(_p(d), N, _p(out)))
    return out


def defect(res: int, d0: float = 1.0) -> np.ndarray:
    out = np.empty((res, res, 2))
    _check(lib().oracle_defect(res, d0, _p(out)))
    return out


def deform(dr, d0: float) -> np.ndarray:
    """T = p + t(p; d_r + d0) - t(p; d0) at every texel centre: [N, N, 2]."""
    dr = _f64(dr)
    N = dr.shape[0]
    out = np.empty((N, N, 2))
    _check(lib().oracle_deform(_p(dr), N, d0, _p(out)))
    return out


def advect(field, xy) -> np.ndarray:
    field = _f64(field)
    xy = _f64(xy).reshape(-1, 2).copy()
    _check(lib().oracle_advect(_p(field), field.shape[0], _p(xy), xy.shape[0]))
    return xy


def regularize(xy, res: int, iters: int, radius: int = 8, sigma: float = 0.0,
               d0: float = -1.0) -> np.ndarray:
    """The whole iteration in FP64; returns new positions (input untouched)."""
    xy = _f64(xy).reshape(-1, 2).copy()
    _check(lib().oracle_regularize(_p(xy), xy.shape[0], res, iters, radius, sigma, d0))
    return xy


def regularize_probes(xy, probe, res: int, iters: int, radius: int = 8, sigma: float = 0.0,
                      d0: float = -1.0) -> tuple[np.ndarray, np.ndarray]:
    """The iteration with passive probe points moved by the same deformations
    (the composite map at the probes); returns (samples, probes)."""
    xy = _f64(xy).reshape(-1, 2).copy()
    pr = _f64(probe).reshape(-1, 2).copy()
    _check(lib().oracle_regularize_probes(_p(xy), xy.shape[0], _p(pr), pr.shape[0], res, iters, radius, sigma, d0))
    return xy, pr


def regularize_status(xy, res: int, iters: int, radius: int = 8, sigma: float = 0.0,
                      d0: float = -1.0) -> tuple[int, np.ndarray]:
    xy = _f64(xy).reshape(-1, 2).copy()
    st = lib().oracle_regularize(_p(xy), xy.shape[0], res, iters, radius, sigma, d0)
    return st, xy
