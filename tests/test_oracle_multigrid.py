"""Pins of the oracle's multigrid march (Sec. 4.3: overlaid grids, coarsening ratio 2, a
fixed number of steps per grid, the last grid to depletion).

* Grid counts against the ones the paper lists (Secs. 4.3 and 5).
* Coarse-cell fields: volume-weighted means, checked against the closed form for fields
  linear in the cell-centre coordinates on a stretched grid.
* Grey isothermal slab: a ray that reaches the wall carries exactly exp(-kappa L) whatever
  grids its path runs through (the path length is unchanged by the change of grid).
* Geometry: every step on level L ends on a face of level L, its midpoint lies in the cell
  it was charged to, and the levels follow each other after mg_steps steps.
* A field constant on the blocks of the coarsest grid gives every ray the same value as the
  single-grid march (segments in one homogeneous block telescope).
* One level is the single-grid march, bit for bit.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1810_00188_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_level_counts_match_paper(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "multigrid_levels.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 8
    for n, levels in rows:
        assert orc.level_count(int(n), int(n), int(n)) == int(levels)
    assert orc.level_count(256, 128, 128) == 6      # limited by the shortest axis
    assert orc.level_count(24, 30, 24) == 2         # 30 -> 15 is odd: no third grid
    assert orc.level_count(5, 8, 8) == 1


def _stretched(n=16, ny=16, R=4):
    w = inputs.grey_slab(n=n, ny=ny, R=R)
    return w.replace(yf=inputs.tanh_faces(ny, 2.0) + 1.0)


def test_coarse_fields_volume_weighted_closed_form(orc):
    """T and x linear in the cell centres: the volume-weighted mean over a block of cells is
    the value at the middle of the block's extent on every axis (tanh-stretched y)."""
    w = _stretched()
    xc, yc, zc = inputs.centres(w.xf), inputs.centres(w.yf), inputs.centres(w.zf)
    X3, Y3, Z3 = np.meshgrid(xc, yc, zc, indexing="ij")
    T = (700.0 + 90.0 * X3 + 150.0 * Y3 - 60.0 * Z3).ravel()
    x = (0.1 + 0.02 * X3 - 0.01 * Y3 + 0.03 * Z3).ravel()
    w = w.replace(T=T, X=x[None, :])
    P = oracle.Problem(w, mg_levels=3)
    for L in (1, 2):
        Tl, Xl = orc.coarse_fields(P, L)
        b = 1 << L
        mx = 0.5 * (w.xf[:-1:b] + w.xf[b::b])
        my = 0.5 * (w.yf[:-1:b] + w.yf[b::b])
        mz = 0.5 * (w.zf[:-1:b] + w.zf[b::b])
        A, B, Cz = np.meshgrid(mx, my, mz, indexing="ij")
        np.testing.assert_allclose(Tl, (700.0 + 90.0 * A + 150.0 * B - 60.0 * Cz).ravel(), rtol=1e-13)
        np.testing.assert_allclose(Xl[0], (0.1 + 0.02 * A - 0.01 * B + 0.03 * Cz).ravel(), rtol=1e-12)
        # the plain mean of the cell values differs on the stretched axis (the weights matter)
        plain = T.reshape(16, 16, 16).reshape(16 // b, b, 16 // b, b, 16 // b, b).mean(axis=(1, 3, 5))
        assert np.max(np.abs(plain.ravel() - Tl)) > 1e-3


def test_multigrid_grey_slab_exact_per_ray(orc):
    kappa, T = 1.0, 1000.0
    w = inputs.grey_slab(n=16, ny=16, Lx=0.5, Ly=2.0, Lz=0.25, kappa=kappa, T=T)
    P = oracle.Problem(w, mg_levels=3, mg_steps=2)
    rng = np.random.default_rng(2)
    Ic = inputs.SIGMA * T ** 4 / np.pi
    nreach = 0
    for _ in range(300):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        i, j, k = rng.integers(0, 16, size=3)
        yc = (j + 0.5) * 2.0 / 16
        L = ((2.0 - yc) if d[1] > 0 else yc) / abs(d[1])
        tau_w = np.exp(-kappa * L)
        m = orc.march(P, (i, j, k), 0, 0, d, record=4096, multigrid=True)
        if tau_w > w.tol * (1 + 1e-9):
            assert m["end"] == (2 if d[1] > 0 else 1)
            assert m["acc"] == pytest.approx(tau_w * Ic, rel=1e-12)
            assert np.sum(m["ds"]) == pytest.approx(L, rel=1e-12)
            nreach += 1
    assert nreach > 100


def _level_faces(f, L):
    return f[:: 1 << L]


def test_multigrid_steps_end_on_level_faces(orc):
    """Each recorded step on level L: its end point lies on a face of level L, its midpoint
    inside the level-L cell it was charged to; levels advance after mg_steps steps."""
    w = _stretched(n=24, ny=48)
    w = w.replace(xf=inputs.uniform_faces(24, 1.3), zf=inputs.uniform_faces(24, 0.7), tol=0.0)
    S = 3
    P = oracle.Problem(w, mg_levels=4, mg_steps=S)
    Lx, Lz = w.xf[-1] - w.xf[0], w.zf[-1] - w.zf[0]
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(60):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ijk = rng.integers(0, [24, 48, 24])
        o = np.array([0.5 * (w.xf[ijk[0]] + w.xf[ijk[0] + 1]), 0.5 * (w.yf[ijk[1]] + w.yf[ijk[1] + 1]),
                      0.5 * (w.zf[ijk[2]] + w.zf[ijk[2] + 1])])
        m = orc.march(P, ijk, 0, 0, d, record=1 << 16, multigrid=True)
        lev, cells, ds = m["level"], m["cells"], m["ds"]
        n = len(ds)
        expect = np.minimum(np.arange(n) // S, 3)
        assert np.array_equal(lev, expect)
        t = np.cumsum(ds)
        for q in range(n):
            L = int(lev[q])
            xf, yf, zf = (_level_faces(a, L) for a in (w.xf, w.yf, w.zf))
            nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
            mid = o + (t[q] - 0.5 * ds[q]) * d
            end = o + t[q] * d
            ci, cj, ck = cells[q] // (ny * nz), (cells[q] // nz) % ny, cells[q] % nz
            mxw, mzw = np.mod(mid[0] - xf[0], Lx) + xf[0], np.mod(mid[2] - zf[0], Lz) + zf[0]
            assert xf[ci] - 1e-12 <= mxw <= xf[ci + 1] + 1e-12
            assert yf[cj] - 1e-12 <= mid[1] <= yf[cj + 1] + 1e-12
            assert zf[ck] - 1e-12 <= mzw <= zf[ck + 1] + 1e-12
            ex, ez = np.mod(end[0] - xf[0], Lx) + xf[0], np.mod(end[2] - zf[0], Lz) + zf[0]
            dist = min(np.min(np.abs(xf - ex)), np.min(np.abs(yf - end[1])), np.min(np.abs(zf - ez)),
                       abs(ex - xf[0] - Lx), abs(ez - zf[0] - Lz))
            assert dist < 1e-10
            checked += 1
    assert checked > 500


def test_block_constant_field_matches_single_grid(orc):
    """T and x constant on 4 x 4 x 4 blocks (the cells of the coarsest of three grids) but
    different between blocks: the coarse grids carry the same medium, and every ray has the
    single-grid value (tau = 0 cut-off, so every ray ends on a wall)."""
    w = inputs.channel(nx=16, ny=16, nz=16, R=8, nb=3, ng=2, march="f64")
    rng = np.random.default_rng(11)
    Tb = rng.uniform(500.0, 1100.0, size=(4, 4, 4))
    xb = rng.uniform(0.05, 0.2, size=(4, 4, 4))
    up = lambda a: np.repeat(np.repeat(np.repeat(a, 4, 0), 4, 1), 4, 2).ravel()  # noqa: E731
    w = w.replace(T=up(Tb), X=up(xb)[None, :], tol=0.0)
    cells = rng.choice(w.ncells, 40, replace=False)
    single = orc.trace_cells(oracle.Problem(w, mg_levels=1), cells)
    multi = orc.trace_cells(oracle.Problem(w, mg_levels=3, mg_steps=2), cells)
    for f in ("n", "g", "o", "k"):
        assert np.array_equal(single[f], multi[f])
    # a ray ends at a wall or where tau rounds to zero in an optically thick block; which of
    # the two comes first can depend on the segment lengths, the value cannot
    assert np.mean(multi["end"] == single["end"]) > 0.8
    assert np.all(multi["steps"] <= single["steps"])
    assert np.mean(multi["steps"]) < 0.8 * np.mean(single["steps"])
    np.testing.assert_allclose(multi["Y"], single["Y"], rtol=0, atol=1e-10 * np.max(single["absY"]))


def test_one_level_is_the_single_grid_march(orc):
    w = inputs.channel(nx=16, ny=16, nz=16, R=4, nb=3, ng=2, march="f64")
    P = oracle.Problem(w, mg_levels=1, mg_steps=2)
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ijk = rng.integers(0, 16, size=3)
        a = orc.march(P, ijk, 1, 1, d)
        b = orc.march(P, ijk, 1, 1, d, multigrid=True)
        assert (a["acc"], a["absacc"], a["steps"], a["end"]) == (b["acc"], b["absacc"], b["steps"], b["end"])


def test_too_many_levels_is_an_error(orc):
    w = inputs.channel(nx=16, ny=16, nz=16, R=4, nb=3, ng=2, march="f64")
    with pytest.raises(oracle.OracleError):
        orc.trace_cells(oracle.Problem(w, mg_levels=4), [0])
    with pytest.raises(oracle.OracleError):
        orc.trace_cells(oracle.Problem(w, mg_levels=2, mg_steps=0), [0])
