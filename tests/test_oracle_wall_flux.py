"""Pins of the oracle's wall flux (the net radiative flux from the gas into each black wall
face element: the wall terms of the rays that end on it, Eq. 3's wall factor with emissivity
one and Eq. 14's weight, times the source cell's volume over R and the element's area).

* Isothermal grey medium, black walls: every ray value is its wall term (gas terms and the
  residual vanish), so the wall power sum_f A_f q_f equals the gas power sum_c V_c divq_c
  exactly (to rounding) -- in the periodic channel and in the closed box.
* Grey isothermal slab, cold walls: the mean flux on each wall against its exact expectation
  for cell-centred emission, sum_j dy 2 kappa sigma T^4 E2(kappa y_j) (within the Monte Carlo
  error from the exact second moment), and that expectation against the continuum closed form
  sigma T^4 (1 - 2 E3(kappa L)).
* Cells and walls at one temperature: every element receives exactly zero.
* Per ray: the flux of a single-cell problem is the march's wall term at the element the ray
  reached (brute force over the recorded rays).
"""
import numpy as np
import pytest
from scipy.special import expn

import oracle
from paper_1810_00188_amd import inputs

SIG = inputs.SIGMA


def _areas_volumes(w):
    dx, dy, dz = np.diff(w.xf), np.diff(w.yf), np.diff(w.zf)
    V = (dx[:, None, None] * dy[None, :, None] * dz[None, None, :]).reshape(-1)
    A = {"x0": np.outer(dy, dz), "x1": np.outer(dy, dz), "y0": np.outer(dx, dz), "y1": np.outer(dx, dz),
         "z0": np.outer(dx, dy), "z1": np.outer(dx, dy)}
    return V, A


@pytest.mark.parametrize("closed", [False, True])
def test_isothermal_wall_power_equals_gas_power(closed):
    """Isothermal grey gas, cold black walls: sum over walls of A_f q_f == sum_c V_c divq_c."""
    if closed:
        w = inputs.grey_box(n=10, R=16, kappa=0.7, T=900.0)
    else:
        w = inputs.grey_slab(n=10, ny=12, Lx=0.8, Ly=1.5, Lz=0.6, kappa=0.7, T=900.0, R=16)
    P = oracle.Problem(w)
    q = oracle.split_walls(P, oracle.wall_flux(P))
    dq, _, _ = oracle.divergence(P)
    V, A = _areas_volumes(w)
    wall_power = sum(float((A[k] * q[k]).sum()) for k in q)
    gas_power = float((V * dq).sum())
    assert wall_power == pytest.approx(gas_power, rel=1e-12)
    if not closed:   # periodic x and z: nothing reaches an x or z wall
        assert not q["x0"].any() and not q["z1"].any()
    else:
        assert all(q[k].sum() > 0 for k in q)


def test_grey_slab_wall_flux_closed_form():
    """32^3 cells on a 1 x 2 x 1 box, kappa = 1, T = 1000 K, cold black walls, R = 16."""
    n, kappa, T, L = 32, 1.0, 1000.0, 2.0
    w = inputs.grey_slab(n=n, R=16, kappa=kappa, T=T)
    P = oracle.Problem(w)
    q = oracle.split_walls(P, oracle.wall_flux(P))
    dy = L / n
    y = (np.arange(n) + 0.5) * dy
    A = 4.0 * kappa * SIG * T ** 4
    m1 = 0.5 * A * expn(2, kappa * y)                 # E[Y_w] of one ray toward y = 0
    m2 = 0.5 * A * A * expn(2, 2 * kappa * y)         # E[Y_w^2]
    expect = float((dy * m1).sum())
    # the wall mean averages n^2 x n columns of R rays: Var = sum_j dy^2 Var_j / (n^2 R)
    sd = float(np.sqrt((dy ** 2 * (m2 - m1 ** 2)).sum() / (n * n * 16)))
    for k in ("y0", "y1"):
        assert abs(q[k].mean() - expect) < 4.5 * sd, (k, q[k].mean(), expect, sd)
    # the discrete expectation against the continuum: sigma T^4 (1 - 2 E3(kappa L))
    cont = SIG * T ** 4 * (1.0 - 2.0 * expn(3, kappa * L))
    assert expect == pytest.approx(cont, rel=2e-3)
    assert cont == pytest.approx(SIG * T ** 4 * 0.939734, rel=1e-5)   # E3(2) = 0.0301333 (tables)


def test_uniform_temperature_gives_zero_wall_flux():
    w = inputs.grey_box(n=6, R=8, kappa=1.3, T=700.0, T_walls6=(700.0,) * 6)
    q = oracle.wall_flux(oracle.Problem(w))
    assert not q.any()


def test_wall_flux_brute_force_single_cell():
    """A 1 x 3 x 1 column with one hot cell: the flux of every element is the sum of the
    recorded rays' wall terms that reached it, from the per-ray march."""
    w = inputs.grey_slab(n=1, ny=3, Lx=0.3, Ly=0.9, Lz=0.4, kappa=2.0, T=800.0, R=64)
    T = np.array([300.0, 800.0, 300.0])
    w = w.replace(T=T, T_walls=(300.0, 300.0))
    P = oracle.Problem(w)
    q = oracle.split_walls(P, oracle.wall_flux(P))
    rays = oracle.trace_cells(P, np.arange(3))
    V, A = _areas_volumes(w)
    # rebuild each ray's wall term from its march: ray value = w kappa acc, wall part = w kappa wacc
    expect = {"y0": 0.0, "y1": 0.0}
    for c in range(3):
        for r in range(w.R):
            ry = rays[c, r]
            if ry["end"] not in (1, 2):
                continue
            d = _direction(P, w, c, ry)
            m = oracle.march(P, (0, c, 0), int(ry["n"]), int(ry["g"]), d)
            assert m["end"] == ry["end"] and m["wall"] == (2 if ry["end"] == 1 else 3) and m["wface"] == 0
            wk = ry["Y"] / m["acc"] if m["acc"] != 0.0 else 0.0
            expect["y0" if ry["end"] == 1 else "y1"] += V[c] * wk * m["wacc"] / (w.R * A["y0"][0, 0])
    for k in ("y0", "y1"):
        assert q[k][0, 0] == pytest.approx(expect[k], rel=1e-12, abs=1e-300)
    assert q["y0"][0, 0] != 0.0 and q["y1"][0, 0] != 0.0


def _direction(P, w, c, ry):
    """The ray's direction from its Philox draw (the oracle's own generator, Eq. 9)."""
    key = np.array([w.seed & 0xFFFFFFFF, w.seed >> 32], dtype=np.uint32)
    ctr = np.array([c, (int(ry["n"]) << 16) | (int(ry["g"]) << 8) | int(ry["o"]), int(ry["k"]), (w.snap << 4) | 2],
                   dtype=np.uint32)
    v = oracle.philox(ctr, key)
    mu = 1.0 - 2.0 * ((float(v[0] >> 9) + 0.5) / 8388608.0)
    phi = 2.0 * np.pi * ((float(v[1] >> 9) + 0.5) / 8388608.0)
    s = np.sqrt((1.0 - mu) * (1.0 + mu))
    d = np.array([abs(s * np.cos(phi)), abs(mu), abs(s * np.sin(phi))])
    o = int(ry["o"])
    for a, bit in ((0, 1), (1, 2), (2, 4)):
        if o & bit:
            d[a] = -d[a]
    return d
