"""Exact expectations of the cell-centred ERMC estimate (test infrastructure only).

The Monte Carlo estimate of one cell (Sec. 2, Eqs. 1-3 and 12-14) is unbiased for

    div q(c) = sum_{n,g} dnu_n w_g kappa_{n,g}(c) * integral over 4 pi of
               [ sum_j tau_j alpha_j (I_n(c) - I_n(j)) + tau_wall (I_n(c) - I_n(T_wall)) ] dOmega

for a medium that is homogeneous inside each cell (Eq. 2) and emits from the cell centre.
When temperature and composition depend on y only, the direction integral over the
azimuth is trivial and the polar one reduces to exponential integrals,
integral_0^1 exp(-a / mu) dmu = E_2(a), giving the closed forms below.  They neglect the
transmissivity cut-off tol (bias below tol * max|I_c - I_j| per ray).
"""
from __future__ import annotations

import numpy as np
from scipy.special import expn

SIGMA = 5.670374419e-8  # Stefan-Boltzmann constant [W m^-2 K^-4]


def E2(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x == 0.0, 1.0, expn(2, np.maximum(x, 1e-300)))


def grey_slab_moments(y, L, kappa, T):
    """Mean and second moment of one ray's value for an isothermal grey slab between cold
    black walls at y = 0 and y = L (emission point at height y):
    Y = 4 kappa sigma T^4 exp(-kappa d / |mu|), mu uniform on (-1, 1), d the distance to the
    wall ahead; E[Y] = 2 kappa sigma T^4 (E2(kappa y) + E2(kappa (L - y))),
    E[Y^2] = (4 kappa sigma T^4)^2 (E2(2 kappa y) + E2(2 kappa (L - y))) / 2."""
    A = 4.0 * kappa * SIGMA * T ** 4
    m1 = 0.5 * A * (E2(kappa * y) + E2(kappa * (L - y)))
    m2 = 0.5 * A * A * (E2(2 * kappa * y) + E2(2 * kappa * (L - y)))
    return m1, m2


def grey_ray_value(d, mu_abs, kappa, T):
    """Exact value of one ray of the isothermal grey slab: 4 kappa sigma T^4 exp(-kappa d/|mu|)."""
    return 4.0 * kappa * SIGMA * T ** 4 * np.exp(-kappa * d / mu_abs)


def table_lerp(tab, T0, dT, T):
    """Linear interpolation of a uniform-in-T table (the precomputed tables of Sec. 2.2)."""
    tab = np.asarray(tab, dtype=np.float64)
    nT = tab.shape[-1]
    u = (np.asarray(T, dtype=np.float64) - T0) / dT
    if np.any(u < 0) or np.any(u > nT - 1):
        raise ValueError("temperature outside the table range")
    t = np.minimum(np.floor(u).astype(np.int64), nT - 2)
    f = u - t
    lo = np.take(tab, t, axis=-1)
    hi = np.take(tab, t + 1, axis=-1)
    return lo + f * (hi - lo)


def layered_properties(w, Trow, Xrow):
    """kappa[j, n, g] and I[j, n] of y-layers with temperatures Trow [ny], mole fractions
    Xrow [ns, ny]; walls I_w0[n], I_w1[n]."""
    kd = w.kd
    k = kd.k.astype(np.float64)                        # [ns, nb, ng, nT]
    kap = np.zeros((len(Trow), kd.nb, kd.ng))
    I = np.zeros((len(Trow), kd.nb))
    for j, T in enumerate(Trow):
        for s in range(kd.ns):
            kap[j] += Xrow[s][j] * table_lerp(k[s], kd.T0, kd.dT, T)
        I[j] = table_lerp(kd.Ib, kd.T0, kd.dT, T)
    Iw0 = table_lerp(kd.Ib, kd.T0, kd.dT, w.T_walls[0])
    Iw1 = table_lerp(kd.Ib, kd.T0, kd.dT, w.T_walls[1])
    return kap, I, Iw0, Iw1


def layered_divq(w, Trow, Xrow):
    """Exact expectation of every y-layer's estimate for a y-stratified medium between
    black walls (Cases 1-2 of Table 1 are instances), shape [ny]:

    div q(c) = sum_{n,g} pi dnu w kappa_c [ 4 I_c - 2 sum_{m, both sides}
               (E2(A_in,m) - E2(A_out,m)) I_m - 2 E2(A_top) I_w1 - 2 E2(A_bot) I_w0 ]

    with A the optical depth in y from the emission point (source half-cells included, as
    segments of the source layer m = c)."""
    kd = w.kd
    yf = np.asarray(w.yf, dtype=np.float64)
    ny = len(yf) - 1
    yc = 0.5 * (yf[:-1] + yf[1:])
    kap, I, Iw0, Iw1 = layered_properties(w, Trow, Xrow)
    pref = np.pi * kd.dnu[:, None] * kd.wg[None, :]              # [nb, ng]
    out = np.zeros(ny)
    for c in range(ny):
        Ic = I[c][:, None]                                       # [nb, 1]
        bracket = 4.0 * np.broadcast_to(Ic, kap[c].shape).copy()
        # upward
        A = np.zeros_like(kap[c])
        for m in range(c, ny):
            lo = yc[c] if m == c else yf[m]
            a_out = A + kap[m] * (yf[m + 1] - lo)
            bracket -= 2.0 * (E2(A) - E2(a_out)) * I[m][:, None]
            A = a_out
        bracket -= 2.0 * E2(A) * Iw1[:, None]
        # downward
        A = np.zeros_like(kap[c])
        for m in range(c, -1, -1):
            hi = yc[c] if m == c else yf[m + 1]
            a_out = A + kap[m] * (hi - yf[m])
            bracket -= 2.0 * (E2(A) - E2(a_out)) * I[m][:, None]
            A = a_out
        bracket -= 2.0 * E2(A) * Iw0[:, None]
        out[c] = np.sum(pref * kap[c] * bracket)
    return out


def optically_thin_limit(w, Trow, Xrow):
    """kappa -> 0 limit of the layered expectation (optically thin approximation, Sec. 1):
    div q -> 2 pi sum dnu w kappa_c (2 I_c - I_w0 - I_w1), shape [ny]."""
    kd = w.kd
    kap, I, Iw0, Iw1 = layered_properties(w, Trow, Xrow)
    pref = 2.0 * np.pi * kd.dnu[:, None] * kd.wg[None, :]
    return np.array([np.sum(pref * kap[c] * (2 * I[c] - Iw0 - Iw1)[:, None])
                     for c in range(len(Trow))])
