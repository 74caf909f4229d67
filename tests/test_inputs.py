"""Pins of the seeded input generators (tables, grids, fields) against independent
mathematics: direct quadrature of Planck's law, textbook values, quadrature exactness."""
import numpy as np
import pytest
from scipy import integrate

from paper_1810_00188_amd import inputs

H = 6.62607015e-34      # Planck constant [J s]
C0 = 2.99792458e8       # speed of light [m/s]
KB = 1.380649e-23       # Boltzmann constant [J/K]


def planck_wavenumber(nu_cm, T):
    """Spectral blackbody intensity per unit wavenumber [W m^-2 sr^-1 (cm^-1)^-1]."""
    nu = 100.0 * nu_cm                                   # m^-1
    return 100.0 * 2.0 * H * C0 ** 2 * nu ** 3 / np.expm1(H * C0 * nu / (KB * T))


def test_second_radiation_constant_matches_codata():
    assert inputs.C2 == pytest.approx(100.0 * H * C0 / KB, rel=1e-9)
    sigma = 2 * np.pi ** 5 * KB ** 4 / (15 * H ** 3 * C0 ** 2)
    assert inputs.SIGMA == pytest.approx(sigma, rel=1e-9)


@pytest.mark.parametrize("zeta", [0.05, 0.3, 1.0, 2.5, 4.965114, 10.0, 30.0])
def test_fraction_series_matches_direct_quadrature(zeta):
    val, _ = integrate.quad(lambda x: x ** 3 * np.exp(-x) / -np.expm1(-x), zeta, np.inf,
                            epsabs=0, epsrel=1e-13)
    ref = 15.0 / np.pi ** 4 * val
    assert inputs.planck_fraction_above(zeta)[0] == pytest.approx(ref, rel=1e-10)


def test_fraction_at_wien_peak_is_one_quarter():
    # textbook: a quarter of blackbody emission lies below lambda T = 2898 um K
    zeta = inputs.C2 / 0.2897771955
    assert inputs.planck_fraction_above(zeta)[0] == pytest.approx(0.25005, abs=2e-5)
    assert inputs.planck_fraction_above(0.0)[0] == 1.0


@pytest.mark.parametrize("T", [300.0, 1000.0, 2000.0])
def test_band_average_matches_planck_law(T):
    nu_lo, dnu = np.array([200.0, 2700.0, 9700.0]), np.array([500.0, 100.0, 500.0])
    tab = inputs.band_planck_table(nu_lo, dnu, np.array([T]))
    for n in range(3):
        val, _ = integrate.quad(planck_wavenumber, nu_lo[n], nu_lo[n] + dnu[n], args=(T,),
                                epsabs=0, epsrel=1e-12)
        assert tab[n, 0] == pytest.approx(val / dnu[n], rel=1e-9)


def test_band_table_zero_kelvin_and_grey():
    tab = inputs.band_planck_table(np.array([200.0]), np.array([100.0]), np.array([0.0, 10.0]))
    assert tab[0, 0] == 0.0 and tab[0, 1] >= 0.0
    g = inputs.grey_kdist(2.0)
    assert g.Ib[0, 100] == pytest.approx(inputs.SIGMA * 1000.0 ** 4 / np.pi, rel=1e-15)
    assert np.all(g.k == 2.0)


def test_gauss_points_integrate_polynomials_exactly():
    gx, wg = inputs.gauss_g_points(7)
    assert np.sum(wg) == pytest.approx(1.0, abs=1e-15)
    for p in range(14):
        assert np.sum(wg * gx ** p) == pytest.approx(1.0 / (p + 1), rel=1e-13)


def test_bf16_round_ties_to_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e-3],
                 dtype=np.float32)
    r = inputs.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # halfway, even mantissa kept
    assert r[2] == np.float32(1.0 + 2 ** -6)  # halfway, rounds up to even
    assert r[3] == 1.0
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert np.all(inputs.bf16_bits(r).astype(np.uint32) << 16 == r.view(np.uint32))


def test_fourier_field_bounds_and_periodicity():
    xf = inputs.uniform_faces(16, 4 * np.pi)
    zf = inputs.uniform_faces(8, 2 * np.pi)
    yf = inputs.tanh_faces(12)
    xi = inputs.fourier_field(inputs.centres(xf), inputs.centres(yf), inputs.centres(zf),
                              4 * np.pi, 2 * np.pi, -1.0, 1.0, 8, 3)
    assert np.max(np.abs(xi)) == pytest.approx(1.0, abs=1e-15)
    # shifting x by the box length leaves every mode unchanged
    xi2 = inputs.fourier_field(inputs.centres(xf) + 4 * np.pi, inputs.centres(yf),
                               inputs.centres(zf), 4 * np.pi, 2 * np.pi, -1.0, 1.0, 8, 3)
    np.testing.assert_allclose(xi, xi2, atol=1e-12)


def test_tanh_faces_monotone_and_clustered():
    f = inputs.tanh_faces(128, 2.0)
    d = np.diff(f)
    assert f[0] == -1.0 and f[-1] == 1.0 and np.all(d > 0)
    assert d[0] < d[64] / 5


def test_synthetic_kdist_planck_mean_target():
    kd = inputs.synthetic_kdist(20, 7, [5], [100.0])
    t = 100  # 1000 K
    num = np.pi * np.sum(kd.dnu[:, None] * kd.Ib[:, t:t + 1] * kd.wg[None, :]
                         * kd.k[0, :, :, t].astype(np.float64))
    assert num / (inputs.SIGMA * 1000.0 ** 4) == pytest.approx(100.0, rel=1e-6)
    assert kd.k.dtype == np.float32 and np.all(kd.k[..., 0] == 0.0)
    kb = inputs.synthetic_kdist(4, 3, [5], [100.0], k_dtype="bf16")
    assert np.all(inputs.bf16_round(kb.k) == kb.k)


def test_channel_fields_in_range():
    w = inputs.channel(nx=8, ny=8, nz=8, amp=0.05, species_amp=0.2, co2=True)
    assert w.T.min() > 300 and w.T.max() < 1000 * 1.05 + 1e-9
    assert np.all(w.T == w.T.astype(np.float32))
    assert w.X.shape == (2, 512)
    assert np.all(np.abs(w.X / 0.1 - 1.0) <= 0.2 + 1e-6)


def test_fourier_field_equals_the_direct_sum():
    """The matrix-product evaluation of the separable modes equals the sum of cosines."""
    xc, yc, zc = np.linspace(0.1, 12, 7), np.linspace(-0.9, 0.9, 5), np.linspace(0.1, 6, 6)
    f = inputs.fourier_field(xc, yc, zc, 4 * np.pi, 2 * np.pi, -1.0, 1.0, 8, 3)
    rng = np.random.default_rng(3)
    a, b, c = rng.integers(-8, 9, 8), rng.integers(-8, 9, 8), rng.integers(0, 5, 8)
    ph = rng.uniform(0, 2 * np.pi, 8)
    X, Y, Z = np.meshgrid(xc, yc, zc, indexing="ij")
    S = sum(np.cos(2 * np.pi * (a[m] * X / (4 * np.pi) + b[m] * Z / (2 * np.pi)) + c[m] * np.pi * (Y + 1) / 2 + ph[m])
            for m in range(8))
    assert np.abs(f - (S / np.abs(S).max()).ravel()).max() < 1e-13
