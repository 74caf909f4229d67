"""Pins of the CPU oracle against what the paper and the mathematics fix.

* Philox4x32-10 known-answer vectors (published with the generator) and uniformity.
* Grey isothermal slab: per-ray value exp(-kappa d / |mu|) exactly, per-layer mean against
  the E_2 closed form with the analytic variance (Table 1 set-up, verification cases).
* Layered 1-D media (Cases 1 and 2 of Table 1, and a non-grey stratified channel with a
  stretched y grid and hot/cold walls): exact E_2 expectations.
* Optically thin limit (Sec. 1) and uniform temperature (reciprocity: zero net exchange).
* The march against a brute-force segment construction on a small 3-D grid.
* Brute-force direction quadrature on a tiny 3-D grid with a random temperature field.
* Histogram of the sampled (band, g, octant) against the T_max pdf (Eqs. 13, 16-17), and
  the learned-allocation importance weights (any positive pdf keeps the mean unbiased).
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import closed_forms as cf
from paper_1810_00188_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------- Philox
def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert orc.philox(v[0:4], v[4:6]) == tuple(v[6:10])


def test_philox_uniformity(orc):
    n = 40000
    words = np.array([orc.philox([c, 7, 0, 0x11], [123, 0]) for c in range(n)], dtype=np.uint64)
    for col in range(4):
        u = (words[:, col].astype(np.float64) + 0.5) / 2.0 ** 32
        h, _ = np.histogram(u, bins=64, range=(0, 1))
        assert stats.chisquare(h).pvalue > 1e-4
    # adjacent counters are uncorrelated
    u0 = words[:, 0].astype(np.float64)
    assert abs(np.corrcoef(u0[:-1], u0[1:])[0, 1]) < 0.03


# ---------------------------------------------------------------- grey slab (P1)
def test_grey_slab_march_exact_per_ray(orc):
    """Isothermal grey medium, cold black walls: a ray that reaches the wall carries exactly
    tau = exp(-kappa L) with L = d / |mu|, whatever its path through the periodic x/z."""
    kappa, T = 1.0, 1000.0
    w = inputs.grey_slab(n=8, ny=16, Lx=0.5, Ly=2.0, Lz=0.25, kappa=kappa, T=T)
    P = oracle.Problem(w)
    rng = np.random.default_rng(1)
    Ic = inputs.SIGMA * T ** 4 / np.pi
    hmax = np.sqrt((0.5 / 8) ** 2 + (2.0 / 16) ** 2 + (0.25 / 8) ** 2)
    nreach = ncut = 0
    for _ in range(400):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        i, j, k = rng.integers(0, 8), rng.integers(0, 16), rng.integers(0, 8)
        yc = (j + 0.5) * 2.0 / 16
        dist = (2.0 - yc) if d[1] > 0 else yc
        L = dist / abs(d[1])
        tau_w = np.exp(-kappa * L)
        m = orc.march(P, (i, j, k), 0, 0, d)
        if tau_w > w.tol * (1 + 1e-9):
            assert m["end"] == (2 if d[1] > 0 else 1)
            assert m["acc"] == pytest.approx(tau_w * Ic, rel=1e-12)
            nreach += 1
        elif tau_w * np.exp(kappa * hmax) < w.tol * (1 - 1e-9):
            assert m["end"] == 0 and m["acc"] == 0.0
            ncut += 1
    assert nreach > 100 and ncut > 10


def test_grey_slab_layer_means_closed_form(orc):
    """32^3 grid on a 1 x 2 x 1 box, kappa = 1, T = 1000 K, R = 16 (the grey isothermal
    slab): every y-layer mean lies within its standard error of
    2 kappa sigma T^4 (E2(kappa y) + E2(kappa (L - y)))."""
    w = inputs.grey_slab(n=32, R=16)
    dq, se, steps = orc.divergence(oracle.Problem(w))
    lay = dq.reshape(32, 32, 32).mean(axis=(0, 2))
    y = (np.arange(32) + 0.5) / 16
    m1, m2 = cf.grey_slab_moments(y, 2.0, 1.0, 1000.0)
    sd = np.sqrt((m2 - m1 ** 2) / (32 * 32 * 16))
    z = (lay - m1) / sd
    assert np.all(np.abs(z) < 4.5), z
    assert np.sum(z ** 2) < stats.chi2.ppf(1 - 1e-4, 32)
    # reference values (scipy E_n): y = 1/32 and y = 0.96875
    assert m1[0] == pytest.approx(104005.322, rel=1e-8)
    assert m1[15] == pytest.approx(33721.764, rel=1e-7)
    assert steps > 0


# ------------------------------------------------------------ layered media (P2)
def _layered_case(profile, n_y=16, R=2048):
    """Cases 1 (lin1) and 2 (parab) of Table 1 over a 1 m slab, grey kappa = 1, black walls;
    the slab normal is y here, x and z periodic."""
    w = inputs.grey_slab(n=2, ny=n_y, Lx=1.0, Ly=1.0, Lz=1.0, kappa=1.0, R=R)
    yc = (np.arange(n_y) + 0.5) / n_y
    if profile == "lin1":
        Trow, walls = 500.0 + 1000.0 * yc, (500.0, 1500.0)
    else:
        Trow, walls = 500.0 - 2000.0 * yc ** 2 + 2000.0 * yc, (500.0, 500.0)
    T = np.broadcast_to(Trow[None, :, None], (2, n_y, 2)).reshape(-1).copy()
    return w.replace(T=T, T_walls=walls), Trow


@pytest.mark.parametrize("profile", ["lin1", "parab"])
def test_paper_cases_1_2_closed_form(orc, profile):
    w, Trow = _layered_case(profile)
    dq, se, _ = orc.divergence(oracle.Problem(w))
    ex = cf.layered_divq(w, Trow, np.ones((1, len(Trow))))
    lay = dq.reshape(2, -1, 2).mean(axis=(0, 2))
    sd = np.sqrt((se.reshape(2, -1, 2) ** 2).mean(axis=(0, 2)) / 4)
    z = (lay - ex) / sd
    assert np.all(np.abs(z) < 4.5), z


def test_nongrey_stratified_channel_closed_form(orc):
    """y-stratified non-grey H2O+CO2 channel, tanh-stretched y, walls at 400 / 900 K."""
    w = inputs.channel(nx=2, ny=12, nz=2, R=3000, nb=5, ng=4, amp=0.0, stretch=2.0,
                       co2=True, march="f64").replace(T_walls=(400.0, 900.0))
    dq, se, _ = orc.divergence(oracle.Problem(w))
    Trow = w.T.reshape(2, 12, 2)[0, :, 0]
    Xrow = w.X.reshape(2, 2, 12, 2)[:, 0, :, 0]
    ex = cf.layered_divq(w, Trow, Xrow)
    lay = dq.reshape(2, 12, 2).mean(axis=(0, 2))
    sd = np.sqrt((se.reshape(2, 12, 2) ** 2).mean(axis=(0, 2)) / 4)
    z = (lay - ex) / sd
    assert np.all(np.abs(z) < 4.5), z


def test_optically_thin_limit(orc):
    """kappa -> 0: the estimate tends to 2 pi sum dnu w kappa (2 I_c - I_w0 - I_w1) with an
    O(kappa L) correction; the relative gap must shrink linearly in kappa."""
    gaps = []
    for kappa in (1e-2, 1e-3):
        w = inputs.grey_slab(n=2, ny=4, Lx=1, Ly=1, Lz=1, kappa=kappa, R=400)
        w = w.replace(T=np.full(16, 1000.0), T_walls=(500.0, 300.0), tol=0.0)
        dq, se, _ = orc.divergence(oracle.Problem(w))
        Trow = np.full(4, 1000.0)
        ota = cf.optically_thin_limit(w, Trow, np.ones((1, 4)))
        ex = cf.layered_divq(w, Trow, np.ones((1, 4)))
        lay = dq.reshape(2, 4, 2).mean(axis=(0, 2))
        sd = np.sqrt((se.reshape(2, 4, 2) ** 2).mean(axis=(0, 2)) / 4)
        assert np.all(np.abs(lay - ex) < 4.5 * sd + 1e-9 * np.abs(ex))
        gaps.append(np.max(np.abs(ex - ota) / ota))
    assert gaps[0] < 0.1 and gaps[1] < gaps[0] / 5


def test_uniform_temperature_gives_exact_zero(orc):
    """Cells and walls at one temperature: every exchange term vanishes (reciprocity)."""
    w = inputs.channel(nx=6, ny=6, nz=6, R=8, nb=4, ng=3, amp=0.0, march="f64")
    w = w.replace(T=np.full(w.ncells, 700.0), T_walls=(700.0, 700.0))
    P = oracle.Problem(w)
    rays = orc.trace_cells(P, np.arange(w.ncells))
    assert np.all(rays["Y"] == 0.0) and np.all(rays["steps"] > 0)


# ------------------------------------------------------------------ march geometry
def _segments_brute_force(P, w, ijk, d, tmax):
    """Independent DDA: all parameters where the ray crosses any x, y or z face plane
    (periodic images included) up to tmax, sorted; each gap's midpoint locates its cell."""
    xf, yf, zf = w.xf, w.yf, w.zf
    Lx, Lz = xf[-1] - xf[0], zf[-1] - zf[0]
    o = np.array([0.5 * (xf[ijk[0]] + xf[ijk[0] + 1]), 0.5 * (yf[ijk[1]] + yf[ijk[1] + 1]),
                  0.5 * (zf[ijk[2]] + zf[ijk[2] + 1])])
    ts = [0.0, tmax]
    for ax, f, L in ((0, xf, Lx), (2, zf, Lz)):
        reps = int(np.ceil(abs(d[ax]) * tmax / L)) + 2
        planes = (f[:-1][None, :] + L * np.arange(-reps, reps + 1)[:, None]).ravel()
        t = (planes - o[ax]) / d[ax]
        ts.extend(t[(t > 0) & (t < tmax)])
    t = (yf - o[1]) / d[1]
    ts.extend(t[(t > 0) & (t < tmax)])
    ts = np.unique(np.array(ts))
    cells, ds = [], []
    for a, b in zip(ts[:-1], ts[1:]):
        p = o + 0.5 * (a + b) * d
        i = np.searchsorted(xf, xf[0] + np.mod(p[0] - xf[0], Lx), side="right") - 1
        k = np.searchsorted(zf, zf[0] + np.mod(p[2] - zf[0], Lz), side="right") - 1
        j = np.searchsorted(yf, p[1], side="right") - 1
        cells.append((i * w.ny + j) * w.nz + k)
        ds.append(b - a)
    return np.array(cells), np.array(ds)


def test_march_matches_brute_force_segments(orc):
    import dataclasses
    w = inputs.channel(nx=5, ny=7, nz=3, R=1, nb=3, ng=2, amp=0.1, stretch=1.5,
                       march="f64").replace(T_walls=(500.0, 800.0), tol=0.0)
    # thin the medium (kappa_P ~ 0.05 m^-1) so that every ray reaches a wall
    w = w.replace(kd=dataclasses.replace(w.kd, k=(w.kd.k * np.float32(0.005))))
    P = oracle.Problem(w)
    rng = np.random.default_rng(7)
    kd = w.kd
    for trial in range(60):
        d = rng.normal(size=3)
        d[1] *= rng.choice([1.0, 0.05])                 # include grazing rays
        d /= np.linalg.norm(d)
        ijk = (rng.integers(0, 5), rng.integers(0, 7), rng.integers(0, 3))
        n, g = rng.integers(0, 3), rng.integers(0, 2)
        m = orc.march(P, ijk, n, g, d, record=100000)
        yc = 0.5 * (w.yf[ijk[1]] + w.yf[ijk[1] + 1])
        twall = ((w.yf[-1] - yc) if d[1] > 0 else (yc - w.yf[0])) / abs(d[1])
        cells, ds = _segments_brute_force(P, w, ijk, d, twall)
        keep = ds > 1e-12 * twall                        # zero-length corner segments
        mc, md = m["cells"], m["ds"]
        mkeep = md > 1e-12 * twall
        np.testing.assert_array_equal(mc[mkeep], cells[keep])
        np.testing.assert_allclose(md[mkeep], ds[keep], rtol=1e-9, atol=1e-12 * twall)
        # value from the brute-force segments: sum tau alpha (I_c - I_j) + wall term
        c0 = (ijk[0] * w.ny + ijk[1]) * w.nz + ijk[2]
        kap = sum(w.X[s] * cf.table_lerp(kd.k[s, n, g].astype(float), kd.T0, kd.dT, w.T)
                  for s in range(kd.ns))
        I = cf.table_lerp(kd.Ib[n], kd.T0, kd.dT, w.T)
        Iw = cf.table_lerp(kd.Ib[n], kd.T0, kd.dT, w.T_walls[1 if d[1] > 0 else 0])
        tau, acc = 1.0, 0.0
        for c, s in zip(cells, ds):
            a = -np.expm1(-kap[c] * s)
            acc += tau * a * (I[c0] - I[c])
            tau *= 1 - a
        acc += tau * (I[c0] - Iw)
        assert m["acc"] == pytest.approx(acc, rel=1e-10, abs=1e-12 * abs(I[c0]))
        assert m["end"] == (2 if d[1] > 0 else 1)


# ----------------------------------------------------- brute-force quadrature (P5)
@pytest.mark.slow
def test_direction_quadrature_tiny_3d(orc):
    """4 x 4 x 4 grid, random temperatures, 2 bands x 2 g: the Monte Carlo mean of a cell
    equals sum_{n,g} dnu w kappa_c * integral over directions of the march, computed with
    a product Gauss-Legendre (mu, per hemisphere) x midpoint (phi) rule."""
    w = inputs.channel(nx=4, ny=4, nz=4, R=20000, nb=2, ng=2, amp=0.0, march="f64")
    rng = np.random.default_rng(11)
    w = w.replace(T=rng.uniform(400, 1200, 64), T_walls=(300.0, 1000.0),
                  xf=inputs.uniform_faces(4, 1.0), zf=inputs.uniform_faces(4, 1.0))
    P = oracle.Problem(w)
    kd = w.kd
    cells = [(1, 0, 2), (2, 2, 1)]
    mu_x, mu_w = np.polynomial.legendre.leggauss(48)
    mu_x, mu_w = 0.5 * (mu_x + 1), 0.5 * mu_w
    nphi = 64
    phis = 2 * np.pi * (np.arange(nphi) + 0.5) / nphi
    for ijk in cells:
        c = (ijk[0] * 4 + ijk[1]) * 4 + ijk[2]
        rays = orc.trace_cells(P, [c])[0]
        mc, se = rays["Y"].mean(), rays["Y"].std(ddof=1) / np.sqrt(len(rays))
        quad = 0.0
        for n in range(2):
            for g in range(2):
                kap = w.X[0][c] * cf.table_lerp(kd.k[0, n, g].astype(float), kd.T0, kd.dT, w.T[c])
                integral = 0.0
                for sgn in (1.0, -1.0):
                    for mu, wm in zip(mu_x, mu_w):
                        s = np.sqrt(1 - mu * mu)
                        for ph in phis:
                            d = np.array([s * np.cos(ph), sgn * mu, s * np.sin(ph)])
                            integral += wm * (2 * np.pi / nphi) * orc.march(P, ijk, n, g, d)["acc"]
                quad += kd.dnu[n] * kd.wg[g] * kap * integral
        assert abs(mc - quad) < 4.5 * se + 2e-3 * abs(quad), (mc, quad, se)


# --------------------------------------------------------- spectral pdf (P7, P10)
def test_plain_pdf_histogram(orc):
    w = inputs.channel(nx=8, ny=8, nz=8, R=64, nb=6, ng=4, amp=0.05, march="f64")
    P = oracle.Problem(w)
    pdf = orc.plain_pdf(P)
    assert pdf.Tmax == max(w.T.max(), max(w.T_walls))
    assert np.sum(pdf.p) == pytest.approx(1.0, abs=1e-14)
    assert pdf.cdf_b[-1] == 1.0 and np.all(np.diff(pdf.cdf_b) >= 0)
    assert np.all(pdf.cdf_g[:, -1] == 1.0)
    rays = orc.trace_cells(P, np.arange(w.ncells)).ravel()
    h = np.zeros((6, 4, 8))
    np.add.at(h, (rays["n"], rays["g"], rays["o"]), 1)
    expect = np.repeat(pdf.p[:, :, None] / 8, 8, axis=2) * len(rays)
    m = expect > 5
    assert stats.chisquare(h[m], expect[m] * h[m].sum() / expect[m].sum()).pvalue > 1e-4
    np.testing.assert_allclose(rays["p"], pdf.p[rays["n"], rays["g"]] / 8, rtol=1e-15)
    # ordinal k counts earlier rays of the same cell in the same stratum
    r0 = orc.trace_cells(P, [5])[0]
    for r in range(w.R):
        same = [(r0["n"][q], r0["g"][q], r0["o"][q]) == (r0["n"][r], r0["g"][r], r0["o"][r])
                for q in range(r)]
        assert r0["k"][r] == sum(same)


def test_learned_pdf_importance_weights_unbiased(orc):
    """An arbitrary (even adversarial) per-cell allocation pdf mixed with 10 % of the plain
    one leaves every layer mean on the exact expectation."""
    w = inputs.channel(nx=2, ny=6, nz=2, R=4000, nb=3, ng=3, amp=0.0, march="f64")
    w = w.replace(T_walls=(350.0, 950.0))
    rng = np.random.default_rng(3)
    q = rng.gamma(0.3, size=(w.ncells, 3, 3, 8))
    q[:, 0] *= 50.0                                   # push most rays into band 0
    P = oracle.Problem(w, q_cell=q, mix_eps=0.1)
    dq, se, _ = orc.divergence(P)
    Trow = w.T.reshape(2, 6, 2)[0, :, 0]
    ex = cf.layered_divq(w, Trow, w.X.reshape(1, 2, 6, 2)[:, 0, :, 0])
    lay = dq.reshape(2, 6, 2).mean(axis=(0, 2))
    sd = np.sqrt((se.reshape(2, 6, 2) ** 2).mean(axis=(0, 2)) / 4)
    assert np.all(np.abs(lay - ex) < 4.5 * sd), (lay - ex) / sd
    rays = orc.trace_cells(P, [0, 7])
    qn = q[[0, 7]] / q[[0, 7]].sum(axis=(1, 2, 3), keepdims=True)
    pl = orc.plain_pdf(oracle.Problem(w)).p
    mix = 0.9 * qn + 0.1 * np.repeat(pl[None, :, :, None] / 8, 8, axis=3)
    for a in range(2):
        r = rays[a]
        np.testing.assert_allclose(r["p"], mix[a][r["n"], r["g"], r["o"]], rtol=1e-12)


def test_out_of_range_temperature_is_an_error(orc):
    w = inputs.grey_slab(n=4, R=2)
    T = w.T.copy()
    T[3] = 2500.0
    with pytest.raises(oracle.OracleError):
        orc.divergence(oracle.Problem(w.replace(T=T)))
    T[3] = np.nan
    with pytest.raises(oracle.OracleError):
        orc.divergence(oracle.Problem(w.replace(T=T)))
    for eps in ((1.5, 1.0), (1.0, -0.1), (np.nan, 1.0)):       # emissivity outside [0, 1]
        with pytest.raises(oracle.OracleError):
            orc.divergence(oracle.Problem(w.replace(eps_walls=eps)))
