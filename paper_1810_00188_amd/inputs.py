"""Seeded synthetic inputs for the reciprocal Monte Carlo radiative heat-source solver.

Everything in this module is an *input* of the method, never a step of it:

* grids, given as face coordinates (x and z periodic, y bounded by two walls);
* temperature and mole-fraction fields on the cell centres;
* the narrow-band correlated-k tables the paper precomputes before marching
  (Sec. 2.1 and the interpolation tables of Sec. 2.2): band-averaged blackbody
  intensities and absorption coefficients on a uniform temperature grid, plus the
  band widths and the Gauss quadrature weights of the g-points.

The CPU oracle and the HIP library both consume these arrays.  Nothing here draws a
ray, evaluates a probability, marches or accumulates a heat source.  The paper's real
inputs (HITRAN-derived narrow-band tables, DNS snapshots) are not available, so every
array is generated from a seed with the shapes and value ranges of the paper's
workloads (Sec. 2.3, Sec. 6); the recipes are stated next to each generator.

Storage convention: cell (i, j, k) of an nx x ny x nz grid has natural index
c = (i * ny + j) * nz + k (k fastest), the ordering of the paper's thread-to-cell map
(Algorithm 2).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SIGMA = 5.670374419e-8   # Stefan-Boltzmann constant [W m^-2 K^-4]
C2 = 1.4387768775039337  # second radiation constant h c / k_B [cm K] (exact SI constants)

TAG_FIELD_NOTE = "field generators use numpy PCG64 streams seeded per field"


# ----------------------------------------------------------------------------- grids
def uniform_faces(n: int, length: float, origin: float = 0.0) -> np.ndarray:
    """n+1 equally spaced face coordinates covering [origin, origin + length]."""
    f = origin + length * (np.arange(n + 1, dtype=np.float64) / n)
    f[-1] = origin + length
    return f


def tanh_faces(n: int, gamma: float = 2.0) -> np.ndarray:
    """Wall-clustered faces on [-1, 1]: y_j = -tanh(gamma (1 - 2 j / n)) / tanh(gamma)."""
    j = np.arange(n + 1, dtype=np.float64)
    f = -np.tanh(gamma * (1.0 - 2.0 * j / n)) / np.tanh(gamma)
    f[0], f[-1] = -1.0, 1.0
    return f


def centres(faces: np.ndarray) -> np.ndarray:
    return 0.5 * (faces[:-1] + faces[1:])


# ---------------------------------------------------------------- spectral tables
def planck_fraction_above(zeta) -> np.ndarray:
    """Fraction of blackbody emission at wavenumbers above nu, zeta = C2 nu / T.

    Textbook series (e.g. Modest, Radiative Heat Transfer, Sec. 1.6):
    F = 15/pi^4 sum_m exp(-m zeta)/m (zeta^3 + 3 zeta^2/m + 6 zeta/m^2 + 6/m^3).
    F(0) = 1, F(inf) = 0.
    """
    z = np.atleast_1d(np.asarray(zeta, dtype=np.float64))
    out = np.zeros_like(z)
    out[z == 0.0] = 1.0
    pos = (z > 0.0) & np.isfinite(z)
    if np.any(pos):
        zp = z[pos]
        mmax = int(min(np.ceil(45.0 / zp.min()) + 4, 2_000_000))
        acc = np.zeros_like(zp)
        for m in range(1, mmax + 1):
            e = np.exp(-m * zp)
            if not np.any(e > 0.0):
                break
            acc += e / m * (zp ** 3 + 3.0 * zp ** 2 / m + 6.0 * zp / m ** 2 + 6.0 / m ** 3)
        out[pos] = acc * (15.0 / np.pi ** 4)
    return out


def band_planck_table(nu_lo: np.ndarray, dnu: np.ndarray, Tgrid: np.ndarray) -> np.ndarray:
    """Band-averaged blackbody intensity I_n(T) [W m^-2 sr^-1 (cm^-1)^-1], shape [nb][nT].

    I_n(T) = sigma T^4 / pi * (F(nu_lo) - F(nu_hi)) / dnu_n, with F the fraction of emission
    above a wavenumber; I_n(0 K) = 0.
    """
    nb, nT = len(nu_lo), len(Tgrid)
    out = np.zeros((nb, nT), dtype=np.float64)
    for t, T in enumerate(Tgrid):
        if T <= 0.0:
            continue
        F_lo = planck_fraction_above(C2 * np.asarray(nu_lo) / T)
        F_hi = planck_fraction_above(C2 * (np.asarray(nu_lo) + np.asarray(dnu)) / T)
        out[:, t] = SIGMA * T ** 4 / np.pi * (F_lo - F_hi) / dnu
    return out


def gauss_g_points(ng: int) -> Tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre abscissae and weights on [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(ng)
    return 0.5 * (x + 1.0), 0.5 * w


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """Raw bfloat16 bit patterns (uint16) of values that are already bf16-representable."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    return (u >> 16).astype(np.uint16)


@dataclass
class KDist:
    """Narrow-band correlated-k tables on a uniform temperature grid T0 + t*dT."""
    nu_lo: np.ndarray          # [nb] lower band edge [cm^-1]
    dnu: np.ndarray            # [nb] band width [cm^-1]
    gx: np.ndarray             # [ng] g abscissae in (0, 1)
    wg: np.ndarray             # [ng] quadrature weights, sum 1
    k: np.ndarray              # float32 [ns][nb][ng][nT], m^-1 per unit mole fraction
    Ib: np.ndarray             # float64 [nb][nT]
    T0: float = 0.0
    dT: float = 10.0
    k_dtype: str = "f32"       # "f32" or "bf16" (then every k value is bf16-representable)

    @property
    def nb(self): return self.k.shape[1]

    @property
    def ng(self): return self.k.shape[2]

    @property
    def ns(self): return self.k.shape[0]

    @property
    def nT(self): return self.k.shape[3]

    @property
    def nu_c(self): return self.nu_lo + 0.5 * self.dnu

    def Tgrid(self) -> np.ndarray:
        return self.T0 + self.dT * np.arange(self.nT, dtype=np.float64)


def grey_kdist(kappa: float, nT: int = 201, T0: float = 0.0, dT: float = 10.0) -> KDist:
    """One band, one g-point: k = kappa at every temperature and dnu * I = sigma T^4 / pi."""
    Tg = T0 + dT * np.arange(nT, dtype=np.float64)
    k = np.full((1, 1, 1, nT), kappa, dtype=np.float32)
    Ib = (SIGMA * Tg ** 4 / np.pi)[None, :]
    return KDist(nu_lo=np.array([0.0]), dnu=np.array([1.0]), gx=np.array([0.5]),
                 wg=np.array([1.0]), k=k, Ib=Ib, T0=T0, dT=dT)


def planck_mean(kd: KDist, k_species: np.ndarray, T: float) -> float:
    """Planck-mean absorption coefficient of one species table at T (table nodes only)."""
    t = int(round((T - kd.T0) / kd.dT))
    Tn = kd.T0 + t * kd.dT
    e = np.pi * np.sum(kd.dnu[:, None] * kd.Ib[:, t:t + 1] * kd.wg[None, :]
                       * k_species[:, :, t].astype(np.float64))
    return float(e / (SIGMA * Tn ** 4))


def synthetic_kdist(nb: int, ng: int, species_seeds: Sequence[int],
                    kP_targets: Sequence[float], nu_min: float = 200.0,
                    nu_max: float = 10200.0, nT: int = 201, T0: float = 0.0,
                    dT: float = 10.0, k_dtype: str = "f32") -> KDist:
    """Seeded synthetic narrow-band correlated-k tables.

    Per species and band n (own PCG64 stream per species seed):
    k_{n,g}(T) = k_n exp(s_n Phi^{-1}(g)) (T / 1000 K)^{a_n} with a_n ~ U[0.5, 1.5],
    s_n ~ U[1, 2.5], log10 k_n ~ U[-1, 2] (log-normal in g, power law in T), then scaled by
    one constant so that the species' Planck-mean coefficient at 1000 K equals kP_targets[s]
    (m^-1 per unit mole fraction).  Bands tile [nu_min, nu_max] contiguously.
    """
    from scipy.special import ndtri
    dnu = np.full(nb, (nu_max - nu_min) / nb)
    nu_lo = nu_min + dnu * np.arange(nb)
    gx, wg = gauss_g_points(ng)
    Tg = T0 + dT * np.arange(nT, dtype=np.float64)
    Ib = band_planck_table(nu_lo, dnu, Tg)
    ks = []
    for seed, target in zip(species_seeds, kP_targets):
        rng = np.random.default_rng(seed)
        a = rng.uniform(0.5, 1.5, nb)
        s = rng.uniform(1.0, 2.5, nb)
        k0 = 10.0 ** rng.uniform(-1.0, 2.0, nb)
        kk = (k0[:, None, None] * np.exp(s[:, None, None] * ndtri(gx)[None, :, None])
              * (Tg[None, None, :] / 1000.0) ** a[:, None, None])
        tmp = KDist(nu_lo, dnu, gx, wg, kk[None].astype(np.float32), Ib, T0, dT)
        scale = target / planck_mean(tmp, kk, 1000.0)
        ks.append(kk * scale)
    k = np.stack(ks).astype(np.float32)
    if k_dtype == "bf16":
        k = bf16_round(k)
    elif k_dtype != "f32":
        raise ValueError(k_dtype)
    return KDist(nu_lo=nu_lo, dnu=dnu, gx=gx, wg=wg, k=k, Ib=Ib, T0=T0, dT=dT, k_dtype=k_dtype)


# ------------------------------------------------------------------------ fields
def fourier_field(xc, yc, zc, Lx, Lz, ylo, yhi, nmodes: int, seed: int) -> np.ndarray:
    """xi = S / max|S| on the cell centres, S = sum_m cos(2 pi (a_m x/Lx + b_m z/Lz)
    + c_m pi (y - ylo)/(yhi - ylo) + phi_m), integer a, b in [-8, 8], c in [0, 4],
    phi in [0, 2 pi).  Periodic in x and z; |xi| <= 1 with equality somewhere.
    Returned in natural order, shape [nx*ny*nz]."""
    rng = np.random.default_rng(seed)
    a = rng.integers(-8, 9, nmodes)
    b = rng.integers(-8, 9, nmodes)
    c = rng.integers(0, 5, nmodes)
    ph = rng.uniform(0.0, 2.0 * np.pi, nmodes)
    # each mode is separable, cos(u + v + w) = Re(e^{iu} e^{iv} e^{iw}), so the sum over modes
    # is one matrix product: S[(i, j), k] = Re(sum_m A[(i, j), m] E[m, k])
    ex = np.exp(1j * 2.0 * np.pi * np.outer(xc / Lx, a))                                   # [nx, m]
    ey = np.exp(1j * (np.outer((yc - ylo) / (yhi - ylo), c) * np.pi + ph[None, :]))      # [ny, m]
    ez = np.exp(1j * 2.0 * np.pi * np.outer(b, zc / Lz))                                   # [m, nz]
    A = (ex[:, None, :] * ey[None, :, :]).reshape(len(xc) * len(yc), nmodes)
    S = np.real(A @ ez).reshape(len(xc), len(yc), len(zc))
    mx = np.max(np.abs(S))
    return (S / mx if mx > 0 else S).reshape(-1)


def as_f32_exact(a: np.ndarray) -> np.ndarray:
    """float64 copy holding float32-representable values (fields handed over in FP32)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# --------------------------------------------------------------------- workloads
@dataclass
class Workload:
    """One field snapshot plus the solver options used on it."""
    name: str
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    T: np.ndarray              # float64 [ncells], natural order
    X: np.ndarray              # float64 [ns][ncells] mole fractions
    kd: KDist
    T_walls: Tuple[float, float] = (0.0, 0.0)     # walls at y = yf[0] and y = yf[-1]
    eps_walls: Tuple[float, float] = (1.0, 1.0)
    R: int = 16
    seed: int = 0
    snap: int = 0
    tol: float = 1e-6
    max_steps: int = 65536
    march: str = "f64"         # "f64" or "f32" ray marching
    accum: str = "f64"         # per-cell sum: "f64", "comp32" (Neumaier FP32) or "f32"
    field_dtype: str = "f64"   # dtype the T / X fields are handed over in
    mg_levels: int = 1         # overlaid grid levels of the multigrid march (1: DNS grid only)
    mg_steps: int = 5          # steps per level before the ray falls onto the next coarser grid
    closed: bool = False       # walls on x and z too (closed box) instead of periodic x / z
    T_walls_x: Tuple[float, float] = (0.0, 0.0)     # closed box: walls at x = xf[0], x = xf[-1]
    eps_walls_x: Tuple[float, float] = (1.0, 1.0)
    T_walls_z: Tuple[float, float] = (0.0, 0.0)     # closed box: walls at z = zf[0], z = zf[-1]
    eps_walls_z: Tuple[float, float] = (1.0, 1.0)

    @property
    def nx(self): return len(self.xf) - 1

    @property
    def ny(self): return len(self.yf) - 1

    @property
    def nz(self): return len(self.zf) - 1

    @property
    def ncells(self): return self.nx * self.ny * self.nz

    @property
    def nrays(self): return self.ncells * self.R

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def grey_slab(n: int = 32, R: int = 16, T: float = 1000.0, kappa: float = 1.0,
              Lx: float = 1.0, Ly: float = 2.0, Lz: float = 1.0, ny: Optional[int] = None,
              T_walls=(0.0, 0.0), seed: int = 0) -> Workload:
    """Grey isothermal slab: n^3 cells on an Lx x Ly x Lz box, periodic x/z, black walls
    at y = 0 and y = Ly, uniform T, grey kappa, FP64 march and sums."""
    ny = n if ny is None else ny
    xf, yf, zf = uniform_faces(n, Lx), uniform_faces(ny, Ly), uniform_faces(n, Lz)
    nc = n * ny * n
    return Workload(name=f"grey_slab_{n}x{ny}x{n}", xf=xf, yf=yf, zf=zf,
                    T=np.full(nc, T), X=np.ones((1, nc)), kd=grey_kdist(kappa),
                    T_walls=tuple(T_walls), R=R, seed=seed, march="f64", accum="f64")


def grey_box(n: int = 16, R: int = 16, T: float = 1000.0, kappa: float = 1.0, L: float = 1.0,
             T_walls6=(0.0,) * 6, eps_walls6=(1.0,) * 6, seed: int = 0) -> Workload:
    """Closed cube of side L with n^3 cells, walls on all six faces (temperatures and
    emissivities in the order x0, x1, y0, y1, z0, z1), uniform T, grey kappa, FP64 march."""
    f = uniform_faces(n, L)
    nc = n ** 3
    return Workload(name=f"grey_box_{n}", xf=f, yf=f.copy(), zf=f.copy(), T=np.full(nc, T), X=np.ones((1, nc)),
                    kd=grey_kdist(kappa), T_walls=(T_walls6[2], T_walls6[3]), eps_walls=(eps_walls6[2], eps_walls6[3]),
                    R=R, seed=seed, march="f64", accum="f64", closed=True,
                    T_walls_x=(T_walls6[0], T_walls6[1]), eps_walls_x=(eps_walls6[0], eps_walls6[1]),
                    T_walls_z=(T_walls6[4], T_walls6[5]), eps_walls_z=(eps_walls6[4], eps_walls6[5]))


def sin_cube(n: int = 20, kappa: float = 0.5, R: int = 64, seed: int = 0) -> Workload:
    """Cases 3 and 4 of Table 1: a 1 m cube with cold black walls, grey kappa (0.5 or 5),
    T = (sin(pi x) sin(pi y) sin(pi z) pi / sigma)^(1/4) at the cell centres, so that
    sigma T^4 / pi = sin(pi x) sin(pi y) sin(pi z).  The Planck table has 0.5 K nodes up to
    200 K (the field peaks at 86.3 K)."""
    f = uniform_faces(n, 1.0)
    c = centres(f)
    S = np.sin(np.pi * c)
    T = (np.einsum("i,j,k->ijk", S, S, S).reshape(-1) * np.pi / SIGMA) ** 0.25
    nc = n ** 3
    return Workload(name=f"sin_cube_{n}_k{kappa:g}", xf=f, yf=f.copy(), zf=f.copy(), T=T, X=np.ones((1, nc)),
                    kd=grey_kdist(kappa, nT=401, T0=0.0, dT=0.5), T_walls=(0.0, 0.0), R=R, seed=seed,
                    march="f64", accum="f64", closed=True)


def cube_3dimens(n: int = 64, R: int = 32, nb: int = 20, ng: int = 7, kP: float = 10.0, table_seed: int = 0,
                 eps_walls: float = 1.0, march: str = "f32", seed: int = 0) -> Workload:
    """Case 12 of Table 1: a 1 m cube of H2O at 1 atm with walls at 500 K on all six faces,
    T = 500 - 2000 (x y z)^2 + 2000 x y z at the cell centres.  Seeded synthetic correlated-k
    tables (nb bands x ng g-points, Planck mean kP at 1000 K) stand in for the H2O data."""
    f = uniform_faces(n, 1.0)
    c = centres(f)
    P = np.einsum("i,j,k->ijk", c, c, c).reshape(-1)
    T = as_f32_exact(500.0 - 2000.0 * P ** 2 + 2000.0 * P)
    kd = synthetic_kdist(nb, ng, [table_seed * 16], [kP / 1.0], k_dtype="f32")
    nc = n ** 3
    e = (eps_walls, eps_walls)
    return Workload(name=f"cube_3dimens_{n}_nb{nb}_ng{ng}", xf=f, yf=f.copy(), zf=f.copy(), T=T,
                    X=np.ones((1, nc)), kd=kd, T_walls=(500.0, 500.0), eps_walls=e, R=R, seed=seed, march=march,
                    accum="f64", field_dtype="f32", closed=True, T_walls_x=(500.0, 500.0), eps_walls_x=e,
                    T_walls_z=(500.0, 500.0), eps_walls_z=e)


def channel(nx: int = 64, ny: int = 64, nz: int = 64, R: int = 32, nb: int = 20,
            ng: int = 7, nmodes: int = 8, amp: float = 0.05, field_seed: int = 0,
            table_seed: int = 0, stretch: Optional[float] = None, x_h2o: float = 0.1,
            species_amp: float = 0.0, co2: bool = False, k_dtype: str = "f32",
            T_wall: float = 300.0, kP: float = 10.0, seed: int = 0, march: str = "f32",
            accum: str = "f64", name: Optional[str] = None) -> Workload:
    """Non-grey channel snapshot on the paper's DNS box (x in [0, 4 pi], y in [-1, 1],
    z in [0, 2 pi]; Sec. 6), black walls at T_wall.

    T = (600 + 400 (1 - y^2)) (1 + amp xi_T); x_s = xbar_s (1 + species_amp xi_s), with
    independent Fourier fields xi (field seeds field_seed*16 + 0, +1, +2).  Synthetic NB-CK
    tables: nb bands over 200-10200 cm^-1, ng Gauss g-points, Planck mean kP at 1000 K and
    the nominal composition (split evenly over the species).  Fields are handed over in FP32.
    """
    Lx, Lz = 4.0 * np.pi, 2.0 * np.pi
    xf, zf = uniform_faces(nx, Lx), uniform_faces(nz, Lz)
    yf = tanh_faces(ny, stretch) if stretch else uniform_faces(ny, 2.0, -1.0)
    xc, yc, zc = centres(xf), centres(yf), centres(zf)
    xi = fourier_field(xc, yc, zc, Lx, Lz, -1.0, 1.0, nmodes, field_seed * 16 + 0)
    Y = np.broadcast_to(yc[None, :, None], (nx, ny, nz)).reshape(-1)
    T = as_f32_exact((600.0 + 400.0 * (1.0 - Y ** 2)) * (1.0 + amp * xi))
    xbar = [x_h2o] + ([0.1] if co2 else [])
    Xs = []
    for s, xb in enumerate(xbar):
        if species_amp > 0.0:
            xs = fourier_field(xc, yc, zc, Lx, Lz, -1.0, 1.0, nmodes, field_seed * 16 + 1 + s)
            Xs.append(as_f32_exact(xb * (1.0 + species_amp * xs)))
        else:
            Xs.append(as_f32_exact(np.full(nx * ny * nz, xb)))
    ns = len(xbar)
    kd = synthetic_kdist(nb, ng, [table_seed * 16 + s for s in range(ns)],
                         [kP / ns / xb for xb in xbar], k_dtype=k_dtype)
    nm = name or f"channel_{nx}x{ny}x{nz}_nb{nb}_ng{ng}"
    return Workload(name=nm, xf=xf, yf=yf, zf=zf, T=T, X=np.stack(Xs), kd=kd,
                    T_walls=(T_wall, T_wall), R=R, seed=seed, march=march, accum=accum,
                    field_dtype="f32")


def channel64(**kw) -> Workload:
    """Non-grey channel, 64^3, 20 bands x 7 g, R = 32, FP32 march, FP64 sums."""
    base = dict(nx=64, ny=64, nz=64, R=32, nb=20, ng=7, nmodes=8, amp=0.05)
    base.update(kw)
    return channel(**base)


def dns256(k_dtype: str = "bf16", **kw) -> Workload:
    """DNS-size snapshot: 256 x 128 x 128, tanh-stretched y (gamma 2), 64 modes at 10 %,
    H2O and CO2 at 0.1 each with independent +-20 % fluctuations, 100 bands x 16 g,
    R = 64, FP32 march."""
    base = dict(nx=256, ny=128, nz=128, R=64, nb=100, ng=16, nmodes=64, amp=0.10,
                stretch=2.0, species_amp=0.2, co2=True, k_dtype=k_dtype)
    base.update(kw)
    return channel(**base)


def batch12(R: int = 32, scale: int = 1) -> List[Workload]:
    """Twelve snapshots of uneven size: three each of 64^3, 96x64x64, 128^3 and 192x96x96
    (divided by `scale` per axis for small tests), stretched y, 50 bands x 8 g, field seeds
    0..11, sharing one table set."""
    shapes = [(64, 64, 64), (96, 64, 64), (128, 128, 128), (192, 96, 96)]
    out = []
    kd = None
    for s in range(12):
        nx, ny, nz = (d // scale for d in shapes[s // 3])
        w = channel(nx=nx, ny=ny, nz=nz, R=R, nb=50, ng=8, nmodes=8, amp=0.05,
                    field_seed=s, stretch=2.0, name=f"batch_s{s}_{nx}x{ny}x{nz}")
        if kd is None:
            kd = w.kd
        out.append(w.replace(kd=kd, snap=s))
    return out
