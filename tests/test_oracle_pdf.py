"""Pin of the oracle's T_max spectral pdf (Zhang's sampling, Eqs. 13 and 16-17) against a
closed form that does not go through the pdf code.

With the emission at T_max, e_{n,g} = pi dnu_n w_g kappa_{n,g}(T_max, xhat) I_n(T_max), as the
sampling pdf (p_{n,g} = e_{n,g} / E, E = sum e = kappa_P(T_max, xhat) sigma T_max^4, the
Planck mean of Eq. 13), the weight every ray of band n and g-point g carries,
w = 4 pi dnu_n w_g / (8 p(n, g, o)) with p(n, g, o) = p_{n,g} / 8, satisfies
    w kappa_{n,g}(T_max, xhat) I_n(T_max) = 4 kappa_P(T_max, xhat) sigma T_max^4
for every (n, g): the per-ray energy QE = 4 kappa_P sigma T_max^4 / N of the Initialize step
of Algorithm 1, times the ray count, is the same for every ray, and only the ratio
R_I = kappa_c I_c / (kappa(T_max) I(T_max)) differs.

The right-hand side is computed here from the blackbody fraction function alone: the table
is built so that its Planck mean has a closed form.  Species 1 absorbs only in the bands
[0, m), species 2 only in [m, nb), with k^s_{n,g}(T) = a_s phi^s_g (T / 1000 K)^beta_s and
sum_g w_g phi^s_g = 1, and the bands tile [nu_0, nu_end] with integer (uneven) widths.  Then
    kappa_P(T, x) sigma T^4 = sigma T^4 [x_1 a_1 (T/1000)^beta_1 (F(nu_0) - F(nu_m))
                                         + x_2 a_2 (T/1000)^beta_2 (F(nu_m) - F(nu_end))],
F(nu) the fraction of blackbody emission above nu at T (pinned to Planck's law in
test_inputs.py).  Uneven band widths, uneven Gauss weights, g-profiles that differ between
the species, species maxima that are not proportional to their means and a T_max cell that
is not the hottest-mean region make the identity fail for a pdf that drops dnu_n or w_g,
takes the mean instead of the largest mole fraction, or evaluates the tables anywhere but at
T_max.
"""
import numpy as np
import pytest

import oracle
from paper_1810_00188_amd import inputs


def _two_species_problem(seed=3):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 6, 5, 4
    nc = nx * ny * nz
    xf = inputs.uniform_faces(nx, 1.5)
    yf = inputs.uniform_faces(ny, 1.0)
    zf = inputs.uniform_faces(nz, 0.8)
    T = rng.uniform(300.0, 1150.0, nc)
    T[17] = 1200.0                                  # T_max, a table node (10 K spacing)
    X1 = rng.uniform(0.05, 0.15, nc)
    X1[40] = 0.31                                   # one cell far above the rest
    X2 = rng.uniform(0.02, 0.30, nc)
    X = np.stack([X1, X2])
    widths = np.array([300.0, 120.0, 700.0, 250.0, 900.0, 180.0, 460.0, 1300.0, 610.0])
    nu0 = 50.0
    nu_lo = nu0 + np.concatenate([[0.0], np.cumsum(widths)[:-1]])
    nb, m, ng = len(widths), 4, 5
    gx, wg = inputs.gauss_g_points(ng)
    phi = np.array([0.2, 0.6, 1.0, 1.9, 3.5])
    psi = np.array([4.0, 1.5, 0.9, 0.3, 0.05])
    phi = phi / np.sum(wg * phi)
    psi = psi / np.sum(wg * psi)
    a = (3.0, 11.0)
    beta = (0.7, 1.3)
    nT = 201
    Tg = 10.0 * np.arange(nT, dtype=np.float64)
    k = np.zeros((2, nb, ng, nT))
    k[0, :m] = a[0] * phi[None, :, None] * (Tg / 1000.0)[None, None, :] ** beta[0]
    k[1, m:] = a[1] * psi[None, :, None] * (Tg / 1000.0)[None, None, :] ** beta[1]
    Ib = inputs.band_planck_table(nu_lo, widths, Tg)
    kd = inputs.KDist(nu_lo=nu_lo, dnu=widths, gx=gx, wg=wg, k=k, Ib=Ib, T0=0.0, dT=10.0)
    w = inputs.Workload(name="two_species_pdf_pin", xf=xf, yf=yf, zf=zf, T=T, X=X, kd=kd,
                        T_walls=(300.0, 500.0), R=48, seed=11, march="f64")
    Tm = 1200.0
    xhat = X.max(axis=1)
    F = lambda nu: float(inputs.planck_fraction_above(inputs.C2 * nu / Tm)[0])
    nu_m, nu_end = nu_lo[m], nu_lo[-1] + widths[-1]
    E = inputs.SIGMA * Tm ** 4 * (xhat[0] * a[0] * (Tm / 1000.0) ** beta[0] * (F(nu0) - F(nu_m))
                                  + xhat[1] * a[1] * (Tm / 1000.0) ** beta[1] * (F(nu_m) - F(nu_end)))
    t = int(round(Tm / 10.0))
    kap_tmax = xhat[0] * k[0, :, :, t] + xhat[1] * k[1, :, :, t]     # [nb, ng] at T_max, xhat
    I_tmax = Ib[:, t]
    return w, E, kap_tmax, I_tmax


def test_plain_pdf_weights_carry_planck_mean_emission(orc):
    """Every stratum: 4 pi dnu_n w_g kappa(T_max) I(T_max) / p_{n,g} = 4 kappa_P sigma T_max^4."""
    w, E, kap, I = _two_species_problem()
    P = oracle.Problem(w)
    pdf = orc.plain_pdf(P)
    assert pdf.Tmax == 1200.0
    assert np.sum(pdf.p) == pytest.approx(1.0, abs=1e-14)
    emit = 4.0 * np.pi * w.kd.dnu[:, None] * w.kd.wg[None, :] * kap * I[:, None]
    live = kap > 0.0
    assert np.all(pdf.p[~live] == 0.0) and np.all(pdf.p[live] > 0.0)
    ratio = emit[live] / pdf.p[live] / (4.0 * E)
    assert np.max(np.abs(ratio - 1.0)) < 1e-12


def test_traced_rays_carry_planck_mean_emission(orc):
    """Per drawn ray (probability p(n, g, o) as the oracle's trace reports it): the weight
    w = 4 pi dnu_n w_g / (8 p) times kappa_{n,g}(T_max, xhat) I_n(T_max) is the per-ray energy
    of Algorithm 1's Initialize step times the ray count, 4 kappa_P(T_max) sigma T_max^4."""
    w, E, kap, I = _two_species_problem()
    P = oracle.Problem(w)
    recs = orc.trace_cells(P, np.arange(0, w.ncells, 7))
    n, g, p = recs["n"].ravel(), recs["g"].ravel(), recs["p"].ravel()
    assert np.any(n < 4) and np.any(n >= 4)      # both species' bands are drawn
    assert len(np.unique(n)) >= w.kd.nb - 1 and len(np.unique(g)) == w.kd.ng
    wt = 4.0 * np.pi * w.kd.dnu[n] * w.kd.wg[g] / (8.0 * p)
    ratio = wt * kap[n, g] * I[n] / (4.0 * E)
    assert np.max(np.abs(ratio - 1.0)) < 1e-12
