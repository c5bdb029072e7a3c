"""The pins have teeth: plausible mistakes planted in a copy of the oracle
(on the CPU only) must each make at least one pin fail.

Each mutant is oracle.c with one textual change (a dropped term, a wrong
inequality, swapped anchors, an off-by-one border, ...), compiled to a
temporary library and run through a compact set of the checks of
test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2408_06513_amd import datagen as dg
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "alpha_exclusive_rows": ("        if (!rows_below) /* j' <= j: admit row j before evaluating it */",
                             "        if (0) /* mutant */"),
    "alpha_t_strict_v": ("            double s = 0.0; /* v' >= v */\n            for (int k = M - 1; k >= 0; --k) { s += acc[k]; run[k] = s; }",
                         "            double s = 0.0;\n            for (int k = M - 1; k >= 0; --k) { run[k] = s; s += acc[k]; }"),
    "drop_gamma_t_term": ("+ at * x + bt * 1.0 + gt * x + dt * 0.0;", "+ at * x + bt * 1.0 + dt * 0.0;"),
    "swap_q2_q4": ("double sx = al * q[0][0] + be * q[1][0] + ga * q[2][0] + de * q[3][0]",
                   "double sx = al * q[0][0] + be * q[3][0] + ga * q[2][0] + de * q[1][0]"),
    "anchor_sign": ("q[0][1] = 1.0 + y - x; q[2][0] = x - y;", "q[0][1] = 1.0 - y + x; q[2][0] = x - y;"),
    "map_over_C": ("t[2 * k] = sx / (2.0 * C);", "t[2 * k] = sx / C;"),
    "texel_corner": ("static double texel_pos(int k, int N) { return ((double)k + 0.5) / (double)N; }",
                     "static double texel_pos(int k, int N) { return ((double)k) / (double)N; }"),
    "mirror_off_by_one": ("    if (m >= N) m = 2 * N - 1 - m;", "    if (m >= N) m = 2 * N - 2 - m;"),
    "zero_border_blur": ("a += g[m + r] * c[(size_t)j * N + mirror(i + m, N)];",
                         "a += (i + m >= 0 && i + m < N) ? g[m + r] * c[(size_t)j * N + i + m] : 0.0;"),
    "no_defect": ("field[2 * k] = texel_pos(i, N) + t[2 * k] - defect[2 * k];", "field[2 * k] = t[2 * k];"),
    "clamped_fraction": ("    *f = s - (double)k; /* not clamped: the border cells extrapolate */",
                         "    *f = s - (double)k; if (*f < 0.0) *f = 0.0; if (*f > 1.0) *f = 1.0;"),
    "advect_weights_swapped": ("double v = (1.0 - fx) * (1.0 - fy) * a[comp] + fx * (1.0 - fy) * b[comp]",
                               "double v = (1.0 - fx) * (1.0 - fy) * a[comp] + fy * (1.0 - fx) * b[comp]"),
    "d0_dropped": ("for (size_t k = 0; k < NN; ++k) d[k] = dr[k] + d0; /* eq. (d0) */",
                   "for (size_t k = 0; k < NN; ++k) d[k] = dr[k];"),
    "splat_round": ("    int k = (int)floor(x * (double)N);", "    int k = (int)floor(x * (double)N + 0.5);"),
    "sigma_not_half_r": ("    if (!(sigma > 0.0)) sigma = 0.5 * (double)r;", "    if (!(sigma > 0.0)) sigma = (double)r;"),
}


def build_mutant(tmp_path, name: str) -> str:
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor of {name} not unique"
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"lib_{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", str(c),
                           "-o", str(so), "-lm"])
    return str(so)


def checks() -> list:
    """Compact pin checks; each returns True when it passes."""
    out = []

    def brute():
        d = dg.rng(8).integers(0, 9, size=(8, 8)).astype(np.float64)
        P, _ = oracle.planes(d)
        return np.array_equal(P, pins.brute_planes(d))

    def golden():
        d, rows = pins.load_golden()
        T = oracle.deform(d, 0.0)
        return all(np.allclose(T[int(r[1]), int(r[0])], r[14:16], atol=1e-15) for r in rows)

    def blur():
        c = dg.poisson_raster(4, 32).astype(np.float64)
        g = pins.gaussian_taps(3, 1.5)
        ref = ndimage.correlate1d(ndimage.correlate1d(c, g, axis=1, mode="reflect"), g, axis=0, mode="reflect")
        return np.allclose(oracle.blur(c, 3), ref, rtol=1e-13, atol=1e-12)

    def counts():
        xy = dg.plain_small(0)[:3000]
        h, _, _ = np.histogram2d(xy[:, 1].astype(np.float64), xy[:, 0].astype(np.float64), bins=64,
                                 range=[[0, 1], [0, 1]])
        return np.array_equal(oracle.counts(xy, 64), h)

    def affine():
        N = 16
        c = (np.arange(N) + 0.5) / N
        X, Y = np.meshgrid(c, c, indexing="xy")
        field = np.stack([0.75 * X + 0.125 * Y + 0.125, -0.0625 * X + 0.5 * Y + 0.25], axis=-1)
        xy = dg.rng(7).uniform(0, 1, size=(200, 2))
        ref = np.stack([0.75 * xy[:, 0] + 0.125 * xy[:, 1] + 0.125,
                        -0.0625 * xy[:, 0] + 0.5 * xy[:, 1] + 0.25], axis=1)
        return np.allclose(oracle.advect(field, xy), np.clip(ref, 0, 1), atol=1e-14)

    def lattice():
        xy = dg.lattice_points(16)
        return np.allclose(oracle.regularize(xy, 16, 2), xy.astype(np.float64), atol=1e-12)

    def default_sigma():
        c = np.zeros((32, 32))
        c[16, 16] = 1.0
        b = oracle.blur(c, 8)
        return np.isclose(b[16, 17] / b[16, 16], np.exp(-1 / (2 * 16.0)), rtol=1e-12)

    def background():
        N = 16
        dr = dg.rng(3).lognormal(0.0, 1.0, size=(N, N))
        c = (np.arange(N) + 0.5) / N
        P = np.stack(np.broadcast_arrays(c[None, :], c[:, None]), axis=-1)
        d1 = oracle.deform(dr, 0.5) - P
        d2 = oracle.deform(dr, 1.0) - P
        return np.allclose(d2, d1 * (dr.sum() + N * N * 0.5) / (dr.sum() + N * N * 1.0), rtol=1e-10, atol=1e-15)

    for f in (brute, golden, blur, counts, affine, lattice, default_sigma, background):
        try:
            out.append((f.__name__, bool(f())))
        except Exception:
            out.append((f.__name__, False))
    return out


def test_unmutated_oracle_passes_all_checks():
    assert all(ok for _, ok in checks()), checks()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_mutant_is_caught(tmp_path, monkeypatch, name):
    so = build_mutant(tmp_path, name)
    real = oracle.lib()
    mut = ctypes.CDLL(so)
    for fn in ("oracle_check_points", "oracle_counts", "oracle_blur", "oracle_planes", "oracle_map",
               "oracle_defect", "oracle_deform", "oracle_advect", "oracle_regularize"):
        getattr(mut, fn).argtypes = getattr(real, fn).argtypes
    monkeypatch.setattr(oracle, "_lib", mut)
    results = checks()
    failed = [n for n, ok in results if not ok]
    assert failed, f"mutant {name} passed every pin: {results}"
