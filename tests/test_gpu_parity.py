"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: uint32 integral images and counts bit-exact; float32 integral images
within 1e-6 relative per element (exact zero where the oracle is zero);
sample positions within 1e-5 of the domain width after the iterations.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2408_06513_amd import datagen as dg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def note(msg: str):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def capi():
    from paper_2408_06513_amd import capi as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def plane_list(mask):
    return [k for k in range(8) if mask >> k & 1]


# ------------------------------------------------------------------ integral images
RES_SMALL = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048]


@pytest.mark.parametrize("res", RES_SMALL + [4096])
@pytest.mark.parametrize("mask", [0xFF, 0x11])
def test_inim_u32_bit_exact(capi, dev, res, mask):
    note(f"inim_u32 res={res} mask={mask:#x}")
    img = dg.poisson_raster(res, res)
    planes, marg = capi.inim(to_dev(img, dev), mask)
    torch.cuda.synchronize()
    got = planes.cpu().numpy()
    ref, rm = oracle.planes(img.astype(np.float64), mask)
    assert ref.max() < 2**32
    assert np.array_equal(got.astype(np.float64), ref)
    m = capi.split_marg(marg.cpu().numpy(), res)
    for k in "XYUV":
        assert np.array_equal(m[k], rm[k]), k
    assert float(m["C"]) == rm["C"]


def assert_rel(got, ref, rtol):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bad = err > rtol * np.abs(ref)
    if bad.any():
        k = np.argwhere(bad)[0]
        raise AssertionError(f"{bad.sum()} elements off; first at {tuple(k)}: got {got[tuple(k)]!r} "
                             f"ref {ref[tuple(k)]!r} rel {err[tuple(k)] / max(abs(ref[tuple(k)]), 1e-300):.3e}")


@pytest.mark.parametrize("res", RES_SMALL + [4096])
@pytest.mark.parametrize("mask", [0xFF, 0x11])
def test_inim_f32_relative(capi, dev, res, mask):
    note(f"inim_f32 res={res} mask={mask:#x}")
    img = dg.lognormal_raster(res, res)
    planes, marg = capi.inim(to_dev(img, dev), mask)
    torch.cuda.synchronize()
    got = planes.cpu().numpy()
    ref, rm = oracle.planes(img.astype(np.float64), mask)
    assert_rel(got, ref, 1e-6)
    m = capi.split_marg(marg.cpu().numpy(), res)
    for k in "XYUV":
        np.testing.assert_allclose(m[k], rm[k], rtol=1e-12, atol=0)


@pytest.mark.parametrize("res", [256, 4096])
def test_inim_f32_correctly_rounded(capi, dev, res):
    """Float rasters of quarter-integers: every region sum is exact in FP64
    (below 2^53), so each float plane element must be that sum rounded to
    float once (nearest, ties to even), bit for bit; sums beyond 2^24
    exercise the rounding."""
    img = (dg.poisson_raster(7, res, lam=40.0).astype(np.float64) / 4.0).astype(np.float32)
    note(f"inim_f32 rounding res={res}")
    planes, _ = capi.inim(to_dev(img, dev), 0xFF)
    torch.cuda.synchronize()
    ref, _ = oracle.planes(img.astype(np.float64), 0xFF)
    assert ref.max() < 2.0**53 and (res < 4096 or ref.max() > 2.0**24)
    assert np.array_equal(planes.cpu().numpy(), ref.astype(np.float32))


@pytest.mark.parametrize("which", ["ones", "spike", "row", "checker"])
def test_inim_special_rasters(capi, dev, which):
    res = 64
    a = np.zeros((res, res), dtype=np.uint32)
    if which == "ones":
        a[:] = 1
    elif which == "spike":
        a[17, 40] = 7
    elif which == "row":
        a[5, :] = 3
    else:
        a[(np.add.outer(np.arange(res), np.arange(res)) % 2) == 0] = 1
    note(f"inim special {which}")
    for img in (a, a.astype(np.float32)):
        planes, _ = capi.inim(to_dev(img, dev), 0xFF)
        torch.cuda.synchronize()
        ref, _ = oracle.planes(a.astype(np.float64), 0xFF)
        assert np.array_equal(planes.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("mask", [0x11, 0x01, 0x10, 0x00])
@pytest.mark.parametrize("res", [2, 16, 64, 256])
def test_inim_min_masks(capi, dev, res, mask):
    """Calls for at most alpha and alpha_t (float rasters summed in double):
    each plane alone, both, and the marginals alone, on integer rasters in
    both types (exact), including the special rasters."""
    rng = np.random.default_rng(res + mask)
    specials = [rng.poisson(3.0, size=(res, res)).astype(np.uint32), np.ones((res, res), np.uint32)]
    spike = np.zeros((res, res), np.uint32)
    spike[res // 3, (2 * res) // 3] = 9
    specials.append(spike)
    for a in specials:
        ref, rm = oracle.planes(a.astype(np.float64), mask)
        for img in (a, a.astype(np.float32)):
            note(f"min masks res={res} mask={mask:#x} {img.dtype}")
            planes, marg = capi.inim(to_dev(img, dev), mask)
            torch.cuda.synchronize()
            if mask:
                assert np.array_equal(planes.cpu().numpy().astype(np.float64), ref)
            m = capi.split_marg(marg.cpu().numpy(), res)
            for k in "XYUV":
                assert np.array_equal(m[k], rm[k]), k
            assert float(m["C"]) == rm["C"]


@pytest.mark.parametrize("res", [256, 4096])
def test_inim_min_mask_correctly_rounded(capi, dev, res):
    """Quarter-integer float rasters through the double-accumulated alpha +
    alpha_t call: double sums are exact there, so both planes are the
    correctly rounded sums."""
    img = (dg.poisson_raster(7, res, lam=40.0).astype(np.float64) / 4.0).astype(np.float32)
    note(f"min mask rounding res={res}")
    planes, _ = capi.inim(to_dev(img, dev), 0x11)
    torch.cuda.synchronize()
    ref, _ = oracle.planes(img.astype(np.float64), 0x11)
    assert np.array_equal(planes.cpu().numpy(), ref.astype(np.float32))


def exact_alpha_alpha_t(q):
    """alpha and alpha_t of an int64 raster q[j, i] in exact integers: column
    prefix cp, alpha its row prefix, alpha_t = L + R - cp with the diagonal
    recurrences L(i,j) = cp(i,j) + L(i-1,j-1), R(i,j) = cp(i,j) + R(i+1,j-1)."""
    cp = np.cumsum(q, axis=0)
    alpha = np.cumsum(cp, axis=1)
    L = np.zeros_like(cp)
    R = np.zeros_like(cp)
    L[0], R[0] = cp[0], cp[0]
    for j in range(1, q.shape[0]):
        L[j, 0] = cp[j, 0]
        L[j, 1:] = cp[j, 1:] + L[j - 1, :-1]
        R[j, -1] = cp[j, -1]
        R[j, :-1] = cp[j, :-1] + R[j - 1, 1:]
    return alpha, L + R - cp


@pytest.mark.parametrize("res", [64, 1024])
def test_inim_min_mask_negative_values_take_exact_path(capi, dev, res):
    """A float raster with negative values: the double-accumulated alpha +
    alpha_t call hands itself to the exact 128-bit path on the device.  Quarter-integers in [-2, 2] plus a
    +2^60 and a -2^60 texel: sums over regions holding both spikes are small
    and exact only without double rounding (double accumulation would lose
    the quarters next to 2^60), so alpha and alpha_t must equal the exact
    integer sums, rounded once to float."""
    rng = np.random.default_rng(res)
    q = rng.integers(-8, 9, size=(res, res)).astype(np.int64)  # quarter units
    big = 1 << 62                                               # 2^60 in quarters
    q[res // 8, res // 6] = big
    q[(5 * res) // 8, (2 * res) // 3] = -big
    img = (q.astype(np.float64) / 4.0).astype(np.float32)
    assert np.array_equal(np.round(img.astype(np.float64) * 4).astype(np.int64), q)
    note(f"min mask negative res={res}")
    planes, _ = capi.inim(to_dev(img, dev), 0x11)
    torch.cuda.synchronize()
    got = planes.cpu().numpy().astype(np.float64)
    for k, ex in enumerate(exact_alpha_alpha_t(q)):
        small = np.abs(ex) < (1 << 53)
        assert np.array_equal(got[k][small], (ex[small].astype(np.float64) / 4.0).astype(np.float32))
        # near 2^60 (one spike inside): within one float unit of the exact sum
        exb = ex[~small].astype(np.float64) / 4.0
        assert np.all(np.abs(got[k][~small] - exb) <= np.spacing(np.abs(exb).astype(np.float32)))


@pytest.mark.parametrize("dtype", ["u32", "f32"])
def test_inim_full_size_8192(capi, dev, dtype):
    """The 8192 x 8192 workload in the benchmark's launch configuration,
    all eight planes, compared element by element; the alpha + alpha_t call
    the benchmark also times gives the same two planes and marginals."""
    res = 8192
    note(f"inim 8192 {dtype}")
    img = dg.poisson_raster(0, res) if dtype == "u32" else dg.lognormal_raster(0, res)
    dimg = to_dev(img, dev)
    planes, marg = capi.inim(dimg, 0xFF)
    pmin, mmin = capi.inim(dimg, 0x11)  # float rasters: summed in double
    torch.cuda.synchronize()
    if dtype == "u32":
        assert torch.equal(pmin[0], planes[0]) and torch.equal(pmin[1], planes[4]) and torch.equal(mmin, marg)
    del dimg
    img64 = img.astype(np.float64)
    for k in range(8):
        ref, rm = oracle.planes(img64, 1 << k)
        got = planes[k].cpu().numpy()
        if dtype == "u32":
            assert np.array_equal(got.astype(np.float64), ref[0]), oracle.PLANES[k]
        else:
            assert_rel(got, ref[0], 1e-6)
            if k in (0, 4):
                assert_rel(pmin[0 if k == 0 else 1].cpu().numpy(), ref[0], 1e-6)
        del ref
    for mm in (marg, mmin):
        m = capi.split_marg(mm.cpu().numpy(), res)
        for key in "XYUV":
            np.testing.assert_allclose(m[key], rm[key], rtol=1e-12 if dtype == "f32" else 0, atol=0)
        assert m["C"] == rm["C"] if dtype == "u32" else abs(m["C"] - rm["C"]) <= 1e-12 * rm["C"]


def test_inim_u32_largest_raster_16384(capi, dev):
    """The largest raster the library accepts, 16384 x 16384 uint32 (counts
    0..3, total below 2^32): all eight planes and the marginals bit-exact
    against the oracle."""
    res = 16384
    g = np.random.Generator(np.random.PCG64(16384))
    img = g.integers(0, 4, size=(res, res), dtype=np.uint32)
    note("inim 16384 u32")
    planes, marg = capi.inim(to_dev(img, dev), 0xFF)
    torch.cuda.synchronize()
    img64 = img.astype(np.float64)
    m = capi.split_marg(marg.cpu().numpy(), res)
    for k in range(8):
        ref, rm = oracle.planes(img64, 1 << k)
        assert np.array_equal(planes[k].cpu().numpy().astype(np.float64), ref[0]), oracle.PLANES[k]
        del ref
    for key in "XYUV":
        assert np.array_equal(m[key], rm[key]), key
    assert m["C"] == rm["C"]


# ------------------------------------------------------------------ rasterize
@pytest.mark.parametrize("res,radius", [(2, 8), (64, 3), (256, 8), (1024, 8), (256, 0), (512, 32)])
def test_rasterize(capi, dev, res, radius):
    note(f"rasterize res={res} r={radius}")
    xy = dg.plain_small(1)
    counts, density, _ = capi.rasterize(to_dev(xy, dev), res, radius=radius)
    torch.cuda.synchronize()
    rc = oracle.counts(xy, res)
    assert np.array_equal(counts.cpu().numpy().astype(np.float64), rc)
    rd = oracle.blur(rc, radius)
    got = density.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, rd, rtol=4e-6, atol=1e-6 * rd.max())


def test_rasterize_edges_and_duplicates(capi, dev):
    xy = np.array([[0, 0], [1, 1], [1, 0], [0, 1], [0.5, 0.5], [0.5, 0.5], [0.999999, 0.25]], np.float32)
    counts, _, _ = capi.rasterize(to_dev(xy, dev), 4, radius=0, want_density=False)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().astype(np.float64), oracle.counts(xy, 4))


# ------------------------------------------------------------------ deform / advect
@pytest.mark.parametrize("res", [2, 16, 256, 1024])
def test_deform_from_planes(capi, dev, res):
    note(f"deform res={res}")
    xy = dg.plain_small(2)
    rc = oracle.counts(xy, res)
    dr = oracle.blur(rc, 8).astype(np.float32)
    d0 = xy.shape[0] / res / res
    planes, marg = capi.inim(to_dev(dr, dev), 0x11)
    field = capi.deform(planes[0], planes[1], marg, d0)
    torch.cuda.synchronize()
    ref = oracle.deform(dr.astype(np.float64), d0)
    np.testing.assert_allclose(field.cpu().numpy(), ref, rtol=0, atol=1e-6)
    # counts (uint32 planes) as the density
    cnt = rc.astype(np.uint32)
    planes, marg = capi.inim(to_dev(cnt, dev), 0x11)
    field = capi.deform(planes[0], planes[1], marg, d0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(field.cpu().numpy(), oracle.deform(rc, d0), rtol=0, atol=1e-6)


@pytest.mark.parametrize("res", [2, 16, 64, 256, 1024])
def test_deform_density_fused(capi, dev, res):
    """inim_deform_density (the integral images in double with the map in
    their last pass, as in one iteration of the regularisation) against the
    oracle's map of the same float density: the bar of inim_deform."""
    note(f"deform_density res={res}")
    xy = dg.plain_small(2)
    rc = oracle.counts(xy, res)
    dr = oracle.blur(rc, 8).astype(np.float32)
    d0 = xy.shape[0] / res / res
    ws = capi.workspace(capi.deform_density_workspace_size(res), dev)
    g = to_dev(dr, dev)
    for dd in (d0, 0.0, 4.0 * d0):
        field = capi.deform_density(g, dd, ws=ws)
        torch.cuda.synchronize()
        ref = oracle.deform(dr.astype(np.float64), dd)
        np.testing.assert_allclose(field.cpu().numpy(), ref, rtol=0, atol=1e-6, err_msg=f"d0={dd}")
    # the same field again from the reused workspace, bit for bit
    again = capi.deform_density(g, d0, ws=ws)
    first = capi.deform_density(g, d0)
    assert torch.equal(again, first)


@pytest.mark.parametrize("res", [256, 1024])
def test_deform_density_is_the_methods_first_iteration(capi, dev, res):
    """rasterize + deform_density + advect moves the samples as one
    iteration of regularize does (the same density; the same integral-image
    and map kernels, the aggregate pass run apart from the smoothing): equal
    to rounding, and the rasters bit for bit."""
    note(f"first iteration via deform_density, res={res}")
    xy = to_dev(dg.plain_small(4), dev)
    one = xy.clone()
    capi.regularize(one, res, 1)
    counts, dens, _ = capi.rasterize(xy, res)
    ref_counts = torch.from_numpy(oracle.counts(xy.cpu().numpy(), res).astype(np.uint32))
    assert torch.equal(counts.cpu(), ref_counts)
    field = capi.deform_density(dens, xy.shape[0] / (res * res))
    moved = xy.clone()
    capi.advect(field, moved)
    torch.cuda.synchronize()
    np.testing.assert_allclose(moved.cpu().numpy(), one.cpu().numpy(), rtol=0, atol=1e-6)


def test_advect(capi, dev):
    res = 256
    xy = dg.plain_small(3)
    dr = oracle.blur(oracle.counts(xy, res), 8)
    T = oracle.deform(dr, xy.shape[0] / res / res)
    Tf = T.astype(np.float32)
    pts = np.concatenate([xy, np.array([[0, 0], [1, 1], [0, 1], [1, 0], [0.001, 0.999]], np.float32)])
    g = to_dev(pts, dev)
    capi.advect(to_dev(Tf, dev), g)
    torch.cuda.synchronize()
    ref = oracle.advect(Tf.astype(np.float64), pts)
    np.testing.assert_allclose(g.cpu().numpy(), ref, rtol=0, atol=2e-7)


# ------------------------------------------------------------------ regularize
def gpu_regularize(capi, dev, xy, res, iters, **kw):
    g = to_dev(xy, dev)
    capi.regularize(g, res, iters, **kw)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def test_regularize_small_config_parity_and_lockstep(capi, dev):
    """20k points, 256^2, r = 8, 4 iterations: final positions within 1e-5 of
    the oracle; each GPU iteration, restarted from the GPU's own previous
    positions, within 1e-6 of one oracle iteration."""
    xy = dg.plain_small(0)
    res, iters = 256, 4
    note("regularize C1 parity")
    got = gpu_regularize(capi, dev, xy, res, iters)
    ref = oracle.regularize(xy, res, iters)
    err = np.abs(got.astype(np.float64) - ref).max()
    note(f"C1 max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-5
    cur = xy.copy()
    for it in range(iters):
        nxt = gpu_regularize(capi, dev, cur, res, 1)
        one = oracle.regularize(cur, res, 1, d0=cur.shape[0] / res / res)
        step_err = np.abs(nxt.astype(np.float64) - one).max()
        assert step_err <= 1e-6, (it, step_err)
        cur = nxt


@pytest.mark.parametrize("seed", [1, 2])
def test_regularize_small_seeds(capi, dev, seed):
    xy = dg.plain_small(seed)
    note(f"regularize C1 seed={seed}")
    got = gpu_regularize(capi, dev, xy, 256, 4)
    assert np.abs(got - oracle.regularize(xy, 256, 4)).max() <= 1e-5


def test_regularize_large_config_parity(capi, dev):
    """1M points (8 clusters + 5% outliers), 1024^2, r = 8, 8 iterations, in
    the benchmark's launch configuration; every sample compared."""
    xy = dg.plain_large(0)
    note("regularize C2 parity (oracle takes a few seconds)")
    got = gpu_regularize(capi, dev, xy, 1024, 8)
    ref = oracle.regularize(xy, 1024, 8)
    err = np.abs(got.astype(np.float64) - ref).max()
    note(f"C2 max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("res,n,radius", [(2, 50, 8), (4, 7, 1), (64, 1, 8), (128, 3000, 0), (512, 5000, 32)])
def test_regularize_edge_sizes(capi, dev, res, n, radius):
    xy = dg.plain_small(4)[:n]
    note(f"regularize edge res={res} n={n} r={radius}")
    got = gpu_regularize(capi, dev, xy, res, 3, radius=radius)
    ref = oracle.regularize(xy, res, 3, radius=radius)
    assert np.abs(got - ref).max() <= 1e-5


@pytest.mark.parametrize("res,n,iters", [(256, 1, 2), (256, 70_001, 2), (512, 1_100_003, 1), (1024, 2_200_003, 1),
                                         (2048, 5, 2), (2048, 3_000, 2), (4096, 20_000, 1)])
def test_regularize_row_sorted_sizes(capi, dev, res, n, iters):
    """Rasters of 256^2 to 4096^2, where the samples are put in texel order by
    row buckets and a per-row sort in LDS: a single sample, a ragged count
    over the 256 sample tiles, tiles of more than one 4096-sample chunk, tiles
    of more than one round of the row histogram's loads (8192 samples), few
    samples on a large raster (the per-row sort takes two rows a block), the
    largest raster of that path."""
    xy = dg.plain_small(8)[:n] if n <= 20_000 else dg.plain_large(2, n=n)
    note(f"regularize row-sorted res={res} n={n}")
    got = gpu_regularize(capi, dev, xy, res, iters)
    assert np.abs(got - oracle.regularize(xy, res, iters)).max() <= 1e-5


def test_regularize_large_raster_8192(capi, dev):
    """8192^2, past the row-sorted range: the texel order from global ranks,
    the blur and the integral images in separate passes on 128 x 32 tiles,
    and the deformation from the general final pass."""
    xy = dg.plain_large(3, n=200_000)
    note("regularize res=8192 (oracle takes tens of seconds)")
    got = gpu_regularize(capi, dev, xy, 8192, 1)
    assert np.abs(got - oracle.regularize(xy, 8192, 1)).max() <= 1e-5


def test_regularize_crowded_row_and_texel(capi, dev):
    """150k samples in one texel row and 50k in one texel (512^2): the row and
    texel buckets far larger than a block."""
    g = np.random.Generator(np.random.PCG64(8))
    a = np.stack([g.random(150_000), 0.5 + g.random(150_000) / 512], 1)
    b = np.stack([0.25 + g.random(50_000) / 1024, 0.75 + g.random(50_000) / 1024], 1)
    xy = np.concatenate([a, b]).astype(np.float32)[g.permutation(200_000)]
    note("regularize crowded rows")
    got = gpu_regularize(capi, dev, xy, 512, 2)
    assert np.abs(got - oracle.regularize(xy, 512, 2)).max() <= 1e-5


def test_regularize_metamorphic_bitwise(capi, dev):
    """Duplicating every sample and permuting the input give bit-identical
    positions on the GPU too (counts are integers; scale invariance)."""
    xy = dg.plain_small(5)[:8000]
    a = gpu_regularize(capi, dev, xy, 256, 3)
    b = gpu_regularize(capi, dev, np.repeat(xy, 2, axis=0), 256, 3)
    assert np.array_equal(np.repeat(a, 2, axis=0), b)
    perm = dg.rng(3).permutation(xy.shape[0])
    c = gpu_regularize(capi, dev, xy[perm], 256, 3)
    assert np.array_equal(a[perm], c)
    d = gpu_regularize(capi, dev, xy, 256, 3)
    assert np.array_equal(a, d)


def test_regularize_lattice_fixed_point(capi, dev):
    xy = dg.lattice_points(64)
    got = gpu_regularize(capi, dev, xy, 64, 4)
    assert np.abs(got - xy).max() <= 1e-6


@pytest.mark.parametrize("res", [64, 256])
def test_regularize_noop_and_domain_error(capi, dev, res):
    empty = torch.empty((0, 2), dtype=torch.float32, device=dev)
    capi.regularize(empty, res, 3)
    xy = dg.plain_small(6)[:1000].copy()
    g0 = to_dev(xy, dev)
    capi.regularize(g0, res, 0)
    assert np.array_equal(g0.cpu().numpy(), xy)
    ws = capi.workspace(capi.workspace_size(res, 1000), dev)
    for bad in (np.nan, 1.5, -0.25):
        xb = xy.copy()
        xb[500, 1] = bad
        g = to_dev(xb, dev)
        with pytest.raises(capi.DomainError):
            capi.regularize(g, res, 3, ws=ws)
        assert np.array_equal(g.cpu().numpy(), xb, equal_nan=True)
    # the workspace recovers: a valid call after a failed one succeeds
    g = to_dev(xy, dev)
    capi.regularize(g, res, 2, ws=ws)
    assert np.abs(g.cpu().numpy() - oracle.regularize(xy, res, 2)).max() <= 1e-5


def test_advect_domain_error_leaves_xy(capi, dev):
    res = 16
    T = np.zeros((res, res, 2), np.float32)
    xy = np.array([[0.5, 0.5], [np.nan, 0.2]], np.float32)
    g = to_dev(xy, dev)
    ws = capi.workspace(256, dev)
    capi.advect(to_dev(T, dev), g, ws=ws, check=False)
    assert capi.sync_status(ws) == capi.EDOMAIN
    assert np.array_equal(g.cpu().numpy(), xy, equal_nan=True)
    with pytest.raises(capi.DomainError):  # the default: synchronise and raise
        capi.advect(to_dev(T, dev), g, ws=ws)
    assert np.array_equal(g.cpu().numpy(), xy, equal_nan=True)


def test_host_errors_with_device_buffers(capi, dev):
    xy = to_dev(dg.plain_small(0)[:100], dev)
    with pytest.raises(capi.InvalidArgument):
        capi.regularize(xy, 100, 2)
    with pytest.raises(capi.InvalidArgument):
        capi.regularize(xy, 64, -1)
    with pytest.raises(capi.InvalidArgument):
        capi.regularize(xy, 64, 2, radius=33)
    small = capi.workspace(1024, dev)
    with pytest.raises(capi.WorkspaceError):
        capi.regularize(xy, 64, 2, ws=small)
    img = torch.zeros((64, 64), dtype=torch.float32, device=dev)
    with pytest.raises(capi.InvalidArgument):
        capi.inim(img, 0x100)


def test_graph_replay_matches_eager(capi, dev):
    """The captured graph gives the eager result on every replay, with eager
    work and synchronisations between replays; changed arguments re-capture."""
    xy0 = dg.plain_small(7)
    res, iters = 256, 3
    eager = gpu_regularize(capi, dev, xy0, res, iters)
    g = capi.Graph()
    buf = to_dev(xy0, dev)
    ws = capi.workspace(capi.workspace_size(res, xy0.shape[0]), dev)
    for rep in range(4):
        buf.copy_(to_dev(xy0, dev))
        capi.regularize_graph(buf, res, iters, g, ws)
        torch.cuda.synchronize()
        assert capi.sync_status(ws) == capi.OK
        assert np.array_equal(buf.cpu().numpy(), eager), rep
        # unrelated eager work between replays
        other = gpu_regularize(capi, dev, xy0[:5000], 64, 1)
        assert other.shape == (5000, 2)
    buf.copy_(to_dev(xy0, dev))
    capi.regularize_graph(buf, res, iters + 1, g, ws)
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), gpu_regularize(capi, dev, xy0, res, iters + 1))
    g.close()
