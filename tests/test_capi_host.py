"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/inim.h, and rejects bad arguments
before touching device memory."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2408_06513_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header: str = "inim.h") -> set[str]:
    src = open(os.path.join(ROOT, "include", header)).read()
    return set(re.findall(r"\b(inim_[a-z0-9_]+)\s*\(", src))


def test_header_and_binding_agree():
    from paper_2408_06513_amd import nn, quality
    assert declared_symbols() == set(capi.EXPORTS)
    assert declared_symbols("inim_nn.h") == set(nn.NN_EXPORTS)
    assert declared_symbols("inim_quality.h") == set(quality.QUALITY_EXPORTS)
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert headers == ["inim.h", "inim_nn.h", "inim_quality.h"]


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    for name in declared_symbols() | declared_symbols("inim_nn.h") | declared_symbols("inim_quality.h"):
        assert hasattr(L, name), name


def test_defaults_and_strerror():
    p = capi.Params()
    capi.lib().inim_default_params(ctypes.byref(p))
    assert (p.radius, p.sigma, p.d0) == (8, 0.0, -1.0)  # sigma unset: radius / 2
    for s in range(6):
        assert capi.strerror(s)
    assert capi.strerror(99) == "unknown status"


def test_workspace_sizes():
    a = capi.workspace_size(1024, 10**6)
    assert a >= 1024 * 1024 * 16
    assert capi.workspace_size(1024, 10**6, radius=0) < a
    assert capi.inim_workspace_size(8192, capi.F32) > capi.inim_workspace_size(8192, capi.U32)
    for bad in (0, 1, 3, 1000, 32768):
        with pytest.raises(capi.InvalidArgument):
            capi.workspace_size(bad, 10)
    with pytest.raises(capi.InvalidArgument):
        capi.workspace_size(64, -1)
    with pytest.raises(capi.InvalidArgument):
        capi.workspace_size(64, 10, radius=40)


# The calls below fail validation before any pointer is used; they run only
# where no GPU is visible so that a validation bug could never reach a launch.
cpu_only = pytest.mark.skipif(__import__("torch").cuda.is_available(), reason="covered by the GPU tests")


@cpu_only
def test_argument_errors_return_before_launch():
    L = capi.lib()
    p = capi.params()
    nul = None
    assert L.inim_regularize(nul, 10, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.EINVAL      # xy NULL
    assert L.inim_regularize(nul, 0, 63, 2, ctypes.byref(p), nul, 0, nul) == capi.EINVAL       # res
    assert L.inim_regularize(nul, -1, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.EINVAL      # n < 0
    assert L.inim_regularize(nul, 0, 64, -2, ctypes.byref(p), nul, 0, nul) == capi.EINVAL      # iters
    assert L.inim_regularize(nul, 0, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.EWORKSPACE   # ws NULL
    assert L.inim_regularize(ctypes.c_void_p(0x1000), 2**32, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.ERANGE
    assert L.inim_inim_f32(nul, 64, 0x11, nul, nul, nul, 0, nul) == capi.EINVAL                # img NULL
    assert L.inim_inim_u32(ctypes.c_void_p(0x1000), 64, 0x1FF, nul, nul, nul, 0, nul) == capi.EINVAL
    assert L.inim_deform(nul, nul, 1, nul, 64, 1.0, nul, nul) == capi.EINVAL
    fk = ctypes.c_void_p(0x1000)
    assert L.inim_deform_density(nul, 64, 1.0, fk, fk, 1 << 30, nul) == capi.EINVAL              # density NULL
    assert L.inim_deform_density(fk, 100, 1.0, fk, fk, 1 << 30, nul) == capi.EINVAL              # res
    assert L.inim_deform_density(fk, 64, -1.0, fk, fk, 1 << 30, nul) == capi.EINVAL              # d0 < 0
    assert L.inim_deform_density(fk, 64, float("nan"), fk, fk, 1 << 30, nul) == capi.EINVAL      # d0 NaN
    assert L.inim_deform_density(fk, 64, 1.0, fk, nul, 1 << 30, nul) == capi.EWORKSPACE          # ws NULL
    assert L.inim_deform_density(fk, 64, 1.0, fk, fk, 1024, nul) == capi.EWORKSPACE              # ws too small
    assert capi.deform_density_workspace_size(1024) > 1024 * 1024 * 8
    assert L.inim_advect(nul, 64, nul, 5, nul, 0, nul) == capi.EINVAL
    fake = ctypes.c_void_p(0x1000)
    assert L.inim_regularize_probes(fake, 10, nul, 5, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.EINVAL
    assert L.inim_regularize_probes(fake, 10, fake, -1, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.EINVAL
    assert L.inim_regularize_probes(fake, 10, fake, 5, 64, 2, ctypes.byref(p), nul, 0, nul) == capi.EWORKSPACE
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    ns = (ctypes.c_int64 * 2)(10, 10)
    sz = ctypes.c_size_t()
    assert L.inim_batch_workspace_size(ptrs, ns, (ctypes.c_int32 * 2)(64, 32), 2, ctypes.byref(p),
                                       ctypes.byref(sz)) == capi.EINVAL                    # res < 64
    assert L.inim_batch_workspace_size(ptrs, ns, (ctypes.c_int32 * 2)(64, 64), 65, ctypes.byref(p),
                                       ctypes.byref(sz)) == capi.EINVAL                    # count > 64
    assert L.inim_batch_workspace_size(ptrs, ns, (ctypes.c_int32 * 2)(64, 128), 2, ctypes.byref(p),
                                       ctypes.byref(sz)) == capi.OK and sz.value > 0
    cfg = capi.BatchConfig(3, 0)
    assert L.inim_regularize_batch(ptrs, ns, (ctypes.c_int32 * 2)(64, 128), 2, 2, ctypes.byref(p), ctypes.byref(cfg),
                                   nul, 0, nul, nul) == capi.EINVAL                        # waves_per_block
    assert L.inim_sync_status(nul, nul) == capi.EWORKSPACE
    assert "NULL" in capi.lib().inim_last_error().decode()
    # the no-allocation variant: the same checks, then its size limit, all before any HIP call
    assert L.inim_regularize_noalloc(nul, 10, 64, 2, ctypes.byref(p), nul, nul) == capi.EINVAL        # xy NULL
    assert L.inim_regularize_noalloc(fake, 10, 100, 2, ctypes.byref(p), nul, nul) == capi.EINVAL      # res
    assert L.inim_regularize_noalloc(fake, 10, 64, -1, ctypes.byref(p), nul, nul) == capi.EINVAL      # iters
    assert L.inim_regularize_noalloc(fake, 2**32, 64, 2, ctypes.byref(p), nul, nul) == capi.ERANGE
    assert capi.workspace_size(2048, 10) > 64 << 20
    assert L.inim_regularize_noalloc(fake, 10, 2048, 2, ctypes.byref(p), nul, nul) == capi.EWORKSPACE
    assert "static scratch" in capi.lib().inim_last_error().decode()
    assert capi.workspace_size(1024, 3_000_000) > 64 << 20
    assert L.inim_regularize_noalloc(fake, 3_000_000, 1024, 2, ctypes.byref(p), nul, nul) == capi.EWORKSPACE


@cpu_only
def test_many_set_argument_errors_return_before_launch():
    from paper_2408_06513_amd import nn
    L, N = capi.lib(), nn.lib()
    nul, fake = None, ctypes.c_void_p(0x1000)
    ptrs = (ctypes.c_void_p * 65)(*([0x1000] * 65))
    ns = (ctypes.c_int64 * 65)(*([10] * 65))
    ws = ctypes.c_size_t(256)
    assert L.inim_rasterize_many(ptrs, ns, 65, 64, nul, fake, nul, fake, 256, nul) == capi.EINVAL   # > 64 sets
    assert L.inim_rasterize_many(ptrs, ns, 0, 64, nul, fake, nul, fake, 256, nul) == capi.EINVAL    # no set
    assert L.inim_rasterize_many(nul, ns, 2, 64, nul, fake, nul, fake, 256, nul) == capi.EINVAL     # xy NULL
    assert L.inim_rasterize_many(ptrs, ns, 2, 100, nul, fake, nul, fake, 256, nul) == capi.EINVAL   # res
    assert L.inim_rasterize_many(ptrs, ns, 2, 64, nul, nul, nul, fake, 256, nul) == capi.EINVAL     # counts NULL
    assert L.inim_rasterize_many(ptrs, ns, 2, 64, nul, fake, nul, fake, 8, nul) == capi.EWORKSPACE
    bad = (ctypes.c_int64 * 2)(10, -1)
    assert L.inim_rasterize_many(ptrs, bad, 2, 64, nul, fake, nul, fake, 256, nul) == capi.EINVAL   # n < 0
    assert L.inim_advect_many(fake, 64, ptrs, ns, 65, fake, 256, nul) == capi.EINVAL
    assert L.inim_advect_many(nul, 64, ptrs, ns, 2, fake, 256, nul) == capi.EINVAL                  # field NULL
    assert L.inim_advect_many(fake, 64, ptrs, ns, 2, nul, 0, nul) == capi.EWORKSPACE
    sc = (ctypes.c_float * 65)(*([1.0] * 65))
    assert N.inim_nn_pack_density_many(fake, 65, 64, sc, 8, fake, nul) == capi.EINVAL
    assert N.inim_nn_pack_density_many(fake, 2, 64, nul, 8, fake, nul) == capi.EINVAL              # scales NULL
    assert N.inim_nn_field_many(fake, 0, 8, 64, 2, fake, fake, nul) == capi.EINVAL
    assert N.inim_nn_field_many(fake, 2, 8, 64, 17, fake, fake, nul) == capi.EINVAL                # radius
    del ws


@cpu_only
def test_quality_argument_errors_return_before_launch():
    from paper_2408_06513_amd import quality
    L = quality.lib()
    nul, fake = None, ctypes.c_void_p(0x1000)
    assert L.inim_quality_bins(nul, 64, 4, fake, nul) == capi.EINVAL                 # counts NULL
    assert L.inim_quality_bins(fake, 64, 3, fake, nul) == capi.EINVAL                # bins do not tile
    assert L.inim_quality_bins(fake, 0, 1, fake, nul) == capi.EINVAL
    assert L.inim_quality_ordering(fake, fake, -1, fake, nul) == capi.EINVAL
    assert L.inim_quality_ordering(nul, fake, 5, fake, nul) == capi.EINVAL
    assert L.inim_quality_ordering(nul, nul, 0, fake, nul) == capi.OK                # no pairs: nothing to do
    assert L.inim_quality_trust(fake, nul, 10, 2, fake, nul) == capi.EINVAL
    assert L.inim_quality_trust(fake, fake, 10, 0, fake, nul) == capi.EINVAL
    assert L.inim_quality_trust(fake, fake, 10, 5, fake, nul) == capi.EINVAL          # 2k >= n
    assert b"2k < n" in L.inim_quality_last_error()
