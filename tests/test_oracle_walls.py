"""Pins of the oracle's walls: emissivity below one with specular reflection (the wall factor
of Eq. 3, reading R14) and the closed box of Cases 3-4 of Table 1 (reading R15).

* Isothermal grey slab between reflecting walls: per ray the exact series
  sum_k eps_k tau_k (I_m - I_w,k) over the successive wall hits of the mirrored path.
* Closed isothermal grey box, black walls: per ray I_m exp(-kappa d) with d the distance to
  the first wall along the ray; with six reflecting walls of different temperatures and
  emissivities, the series over the wall hits of the unfolded straight line.
* Cells and walls at one temperature: every ray value is exactly zero, reflections or not.
* Cases 3 and 4 (the 'sin' field in a cold black cube, kappa 0.5 and 5): the Monte Carlo
  mean at cells on the line y = z ~ 0.5 against a direct quadrature of the radiative
  transfer equation for the continuous field (Sakurai's tabulated solution is not
  available; the quadrature stands in for it).
"""
import numpy as np
import pytest

import oracle
from paper_1810_00188_amd import inputs

SIG = inputs.SIGMA


def _unit(rng):
    d = rng.normal(size=3)
    return d / np.linalg.norm(d)


def _hits_series(o, d, lo, hi, eps, Iw, Im, kappa, nhit=4000):
    """Exact sum over the wall hits of a specularly reflected straight ray in the box
    [lo, hi]^3 (axes with lo = None are periodic): unfold each bounded axis; hit m of axis a
    is at t = (first wall distance + m L_a) / |d_a| on alternating sides."""
    ev = []
    for a in range(3):
        if lo[a] is None or d[a] == 0.0:
            continue
        L = hi[a] - lo[a]
        first = ((hi[a] - o[a]) if d[a] > 0 else (o[a] - lo[a])) / abs(d[a])
        side0 = 1 if d[a] > 0 else 0
        for m in range(nhit):
            ev.append((first + m * L / abs(d[a]), a, side0 ^ (m & 1)))
    ev.sort()
    acc, prod = 0.0, 1.0
    for t, a, side in ev:
        tau = np.exp(-kappa * t) * prod
        if tau < 1e-300:
            break
        e = eps[a][side]
        acc += e * tau * (Im - Iw[a][side])
        prod *= 1.0 - e
    return acc


@pytest.mark.parametrize("eps", [(0.3, 0.6), (0.0, 1.0), (0.1, 0.1)])
def test_reflecting_slab_per_ray_series(orc, eps):
    kappa, T, Tw = 1.0, 1000.0, (300.0, 500.0)
    w = inputs.grey_slab(n=4, ny=8, Lx=0.5, Ly=1.0, Lz=0.5, kappa=kappa, T=T)
    w = w.replace(T_walls=Tw, eps_walls=eps, tol=1e-15, max_steps=1 << 22)
    P = oracle.Problem(w)
    Im = SIG * T ** 4 / np.pi
    Iw = [None, [SIG * t ** 4 / np.pi for t in Tw], None]
    rng = np.random.default_rng(7)
    nref = 0
    for _ in range(150):
        d = _unit(rng)
        i, j, k = rng.integers(0, 4), rng.integers(0, 8), rng.integers(0, 4)
        o = np.array([(i + 0.5) / 8, (j + 0.5) / 8, (k + 0.5) / 8])
        m = orc.march(P, (i, j, k), 0, 0, d)
        ex = _hits_series(o, d, [None, 0.0, None], [None, 1.0, None], [None, eps, None], Iw, Im, kappa)
        assert m["acc"] == pytest.approx(ex, rel=1e-11, abs=1e-12 * Im)
        first = 1 if d[1] > 0 else 0                    # rays that reflect at least once
        d1 = ((1.0 - o[1]) if d[1] > 0 else o[1]) / abs(d[1])
        nref += eps[first] < 1.0 and np.exp(-kappa * d1) > 1e-10
    assert nref > 50


def test_closed_black_box_per_ray_exact(orc):
    kappa, T = 1.0, 1000.0
    w = inputs.grey_box(n=8, kappa=kappa, T=T)
    P = oracle.Problem(w)
    Im = SIG * T ** 4 / np.pi
    rng = np.random.default_rng(3)
    codes = {(0, 0): 4, (0, 1): 5, (1, 0): 1, (1, 1): 2, (2, 0): 6, (2, 1): 7}
    seen = set()
    for _ in range(300):
        d = _unit(rng)
        ijk = rng.integers(0, 8, size=3)
        o = (ijk + 0.5) / 8
        dist = [((1.0 - o[a]) if d[a] > 0 else o[a]) / abs(d[a]) for a in range(3)]
        a = int(np.argmin(dist))
        m = orc.march(P, ijk, 0, 0, d)
        tau_w = np.exp(-kappa * dist[a])
        if tau_w > w.tol * (1 + 1e-9):
            assert m["end"] == codes[(a, int(d[a] > 0))]
            assert m["acc"] == pytest.approx(tau_w * Im, rel=1e-12)
            seen.add(m["end"])
    assert seen == {1, 2, 4, 5, 6, 7}


def test_closed_reflecting_box_per_ray_series(orc):
    kappa, T = 0.75, 1000.0                       # exact in the FP32 table
    Tw6 = (300.0, 500.0, 700.0, 900.0, 0.0, 1200.0)
    eps6 = (0.2, 0.5, 0.0, 0.8, 0.35, 1.0)
    w = inputs.grey_box(n=6, kappa=kappa, T=T, L=1.0, T_walls6=Tw6, eps_walls6=eps6)
    w = w.replace(tol=1e-15, max_steps=1 << 22)
    P = oracle.Problem(w)
    Im = SIG * T ** 4 / np.pi
    Iw = [[SIG * t ** 4 / np.pi for t in Tw6[2 * a:2 * a + 2]] for a in range(3)]
    eps = [eps6[2 * a:2 * a + 2] for a in range(3)]
    rng = np.random.default_rng(11)
    for _ in range(120):
        d = _unit(rng)
        ijk = rng.integers(0, 6, size=3)
        o = (ijk + 0.5) / 6
        m = orc.march(P, ijk, 0, 0, d)
        ex = _hits_series(o, d, [0.0] * 3, [1.0] * 3, eps, Iw, Im, kappa)
        assert m["acc"] == pytest.approx(ex, rel=1e-11, abs=1e-12 * Im)


def test_uniform_temperature_zero_with_reflections(orc):
    w = inputs.grey_box(n=6, T=700.0, T_walls6=(700.0,) * 6, eps_walls6=(0.3, 0.0, 1.0, 0.5, 0.9, 0.2), R=8)
    rays = orc.trace_cells(oracle.Problem(w), np.arange(w.ncells))
    assert np.all(rays["Y"] == 0.0) and np.all(rays["steps"] > 0)
    ws = inputs.channel(nx=6, ny=6, nz=6, R=8, nb=4, ng=3, amp=0.0, march="f64")
    ws = ws.replace(T=np.full(ws.ncells, 700.0), T_walls=(700.0, 700.0), eps_walls=(0.25, 0.6))
    rays = orc.trace_cells(oracle.Problem(ws), np.arange(ws.ncells))
    assert np.all(rays["Y"] == 0.0)


def _rte_quadrature(r, kappa, nmu=48, nphi=96, ns=96):
    """div q = kappa (4 pi Ib(r) - G(r)) for the continuous field Ib = sin(pi x) sin(pi y)
    sin(pi z) in the unit cube with cold black walls: G = sum over directions of the path
    integral of kappa Ib exp(-kappa s) up to the wall (Gauss-Legendre in mu and s, midpoint
    in phi)."""
    xm, wm = np.polynomial.legendre.leggauss(nmu)
    xs, ws = np.polynomial.legendre.leggauss(ns)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    mu = xm[:, None]
    st = np.sqrt(1 - mu ** 2)
    D = np.stack([st * np.cos(phi)[None, :], np.broadcast_to(mu, (nmu, nphi)), st * np.sin(phi)[None, :]])
    sw = np.full((nmu, nphi), np.inf)
    for a in range(3):
        da = D[a]
        with np.errstate(divide="ignore"):
            sa = np.where(da > 0, (1 - r[a]) / da, np.where(da < 0, (0 - r[a]) / da, np.inf))
        sw = np.minimum(sw, sa)
    s = 0.5 * sw[..., None] * (xs + 1)
    P = r[:, None, None, None] + s[None] * D[..., None]
    Ib = np.prod(np.sin(np.pi * np.clip(P, 0.0, 1.0)), axis=0)
    path = np.sum(kappa * Ib * np.exp(-kappa * s) * ws, axis=-1) * 0.5 * sw
    G = np.sum(wm[:, None] * path) * (2 * np.pi / nphi)
    return kappa * (4 * np.pi * np.prod(np.sin(np.pi * r)) - G)


@pytest.mark.parametrize("kappa", [0.5, 5.0])
def test_sin_cube_cases_3_4_quadrature(orc, kappa):
    n = 20
    cells = [(i, 9, 9) for i in (1, 4, 9, 14)]
    est = np.zeros(len(cells))
    var = np.zeros(len(cells))
    K = 24
    for snap in range(K):
        w = inputs.sin_cube(n=n, kappa=kappa, R=160).replace(snap=snap)
        P = oracle.Problem(w)
        idx = [(i * n + j) * n + k for i, j, k in cells]
        dq, se, _ = orc.divergence(P, cells=idx)
        est += dq / K
        var += se ** 2 / K ** 2
    for q, (i, j, k) in enumerate(cells):
        r = (np.array([i, j, k]) + 0.5) / n
        ex = _rte_quadrature(r, kappa)
        assert abs(est[q] - ex) < 4.5 * np.sqrt(var[q]) + 6e-3 * abs(ex), (cells[q], est[q], ex, np.sqrt(var[q]))
