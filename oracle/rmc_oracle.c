/*
 * rmc_oracle.c -- plain, slow FP64 reference of the emission-based reciprocal Monte Carlo
 * (ERMC) radiative heat source on a Cartesian grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is checked
 * against; it is called from the tests, from the smoke check and from the CPU-baseline
 * leg of the benchmark, never from the product path.  It shares no code, header, table
 * or constant generator with the HIP library: the only common ground is the published
 * definition of the Philox4x32-10 generator (Salmon et al., SC'11), implemented here
 * independently, and the seeded input arrays produced by the input generators.
 *
 * What is computed (Silvestri & Pecnik, "A fast GPU Monte Carlo radiative heat transfer
 * implementation for coupling with direct numerical simulation"):
 *   - exchange integral, Sec. 2 Eq. (1), with cell absorptivity alpha = 1 - exp(-kappa l)
 *     (Eq. 2) and path transmissivity tau = prod(1 - alpha) (Eq. 3);
 *   - isotropic direction sampling by inversion (Eqs. 4 and 9);
 *   - the ERMC form Q_i = sum_j Q_{i->j} (1 - I_b(T_j)/I_b(T_i)) (Sec. 2, after Eq. 11)
 *     with Zhang's T_max spectral sampling and the R_I reweighting (Eqs. 13-14);
 *   - narrow-band / g-point discretisation of the spectral pdf with two independent draws
 *     (Sec. 2.1, Eqs. 15-17), inverted as a search on the cumulative sums;
 *   - the march of Algorithm 1: start at the cell centre, step to the nearest face,
 *     accumulate tau * alpha * (I_b(source) - I_b(cell)), stop when tau <= tol and dump the
 *     residual tau * (I_b(source) - I_b(last cell)) (Algorithm 1, March procedure);
 *   - linear interpolation of the precomputed Planck and absorption tables in T
 *     (Sec. 2.2, interpBlackbody / interpAbsorpCoeff).
 *
 * Readings where the paper is silent (each stated where it is used):
 *   R1 emission point = cell centre (Algorithm 1) rather than uniform in the volume (Eq. 4);
 *   R2 polar axis of theta = y (wall normal);
 *   R3 uniform variates from a 32-bit word w: the spectral / octant draws use
 *      U_a(w) = (w + 0.5) 2^-32 (exact in double, decisions taken in double); the direction
 *      draws use U_d(w) = ((w >> 9) + 0.5) 2^-23, exact in float and double; neither is
 *      ever 0 or 1;
 *   R4 walls (y = y_0 and y = y_ny; in a closed box also x and z, R15) absorb the fraction
 *      eps_w of the transmissivity that reaches them and emit I_b(T_wall): one wall term
 *      tau eps_w (I_src - I_b(T_wall)), then tau *= 1 - eps_w (the wall factor of Eq. 3);
 *      a black wall (eps_w = 1) ends the ray;
 *   R5 ties between face crossings step all tied axes together (vector compare);
 *   R6 temperatures outside the table range are an error (no clamping);
 *   R7 mixture: kappa_{n,g} = sum_s x_s k^s_{n,g}(T) on a shared g grid;
 *   R8 T_max = max over cells and walls; the sampling pdf uses, per species, the largest
 *      mole fraction in the domain (any positive pdf keeps the estimator unbiased);
 *   R9 the ray value is written w * sum tau alpha (I_c - I_j), algebraically equal to the
 *      QE R_I (Ib2/Ib1 - 1) form of Algorithm 1 but without dividing by I_b(T_i);
 *   R10 alpha = -expm1(-kappa ds), the same quantity as Eq. (2) without cancellation;
 *   R11 the residual uses I_b of the last cell marched, as in Algorithm 1's formula;
 *   R12 each ray also draws a direction octant ("cone") o uniformly, p(n,g,o) = p(n,g)/8,
 *       and its direction is drawn inside that octant; together isotropic;
 *   R13 if nothing emits at T_max (sum of e_{n,g} is zero) the pdf is uniform over (n,g):
 *       every ray value is then zero and any positive pdf gives that exactly.
 *   R14 the reflection law of Eq. 3 is not stated: the part 1 - eps_w of a ray goes on by
 *       specular reflection -- the origin and the direction component are mirrored on the
 *       wall plane, so the ray keeps its parameter and goes on from the point it hit, in the
 *       cell next to the wall; walls hit at the same point are taken in the order x, y, z;
 *   R15 closed box (Cases 3-4 and 12 of Table 1): x and z bounded by walls as y is, each of
 *       the six walls with its own temperature and emissivity; otherwise x and z are periodic.
 *
 * Multigrid march (Sec. 4.3 and the grid counts of Sec. 5), readings:
 *   M1 levels: coarsening ratio 2 on every axis together; a further level exists while every
 *      axis of the current level has an even number of cells whose half is at least 3 (this
 *      reproduces the paper's grid counts: 3 for 16^3, 4 for 32^3, 5 for 48^3 and 64^3, 6 for
 *      96^3 to 160^3, 7 for 192^3).  Level L has every 2^L-th face of the DNS grid;
 *   M2 coarse-cell temperature and mole fractions: volume-weighted means over the 2^L x 2^L
 *      x 2^L DNS cells the coarse cell covers (on uniform spacing this is also the trilinear
 *      interpolation at the coarse cell centre); properties from the tables at those values;
 *   M3 a ray takes mg_steps steps on each level (the source cell's step counts on the DNS
 *      level), then continues from its current point on the next coarser level (the coarse
 *      cell holding the DNS cell it is in, next-face parameters from that level's faces);
 *      on the last level it runs to depletion.  Source intensity and source kappa stay the
 *      DNS cell's; the residual uses the last cell marched, on whatever level.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_OUT_OF_RANGE 3
#define ORC_UNSUPPORTED 4

#define TAG_ALLOC 1u
#define TAG_DIR 2u

typedef struct {
    int nx, ny, nz;
    const double *xf, *yf, *zf;   /* face coordinates: nx+1, ny+1, nz+1 */
    const double *T;              /* [ncells], natural order (i*ny + j)*nz + k */
    int ns;
    const double *X;              /* [ns][ncells] mole fractions */
    double Tw[2], epsw[2];        /* wall temperature / emissivity at y = yf[0], y = yf[ny] */
    int nb, ng, nT;
    double T0, dT;
    const double *dnu;            /* [nb] band widths [cm^-1] */
    const double *wg;             /* [ng] quadrature weights */
    const double *k;              /* [ns][nb][ng][nT] */
    const double *Ib;             /* [nb][nT] */
    int R;
    uint64_t seed;
    uint32_t snap;
    double tol;
    int max_steps;
    const double *q_cell;         /* optional [ncells][nb][ng][8] allocation pdf per cell */
    double mix_eps;               /* weight of the plain pdf mixed into q_cell */
    int mg_levels;                /* grid levels of the multigrid march (M1); <= 1: DNS grid only */
    int mg_steps;                 /* steps per level before the next coarser one (M3) */
    int closed;                   /* R15: walls on x and z too (else periodic) */
    double Tx[2], epsx[2];        /* closed box: walls at x = xf[0], x = xf[nx] */
    double Tz[2], epsz[2];        /* closed box: walls at z = zf[0], z = zf[nz] */
} orc_problem;

typedef struct {
    double Y;        /* ray value, W m^-3 */
    double absY;     /* same sum with |I_c - I_j| (scale for relative comparisons) */
    double p;        /* probability p(n,g,o) the ray was drawn with */
    int n, g, o, k;  /* band, g-point, octant, ordinal among equal (n,g,o) of the cell */
    int steps;       /* ray-cell steps (DDA segments) */
    int end;         /* 0: tau <= tol, 1 / 2: black wall at y0 / y1, 3: step cap,
                        4 / 5: black wall at x0 / x1, 6 / 7: black wall at z0 / z1 */
} orc_ray;

/* ------------------------------------------------------------------ Philox4x32-10
 * Counter-based generator of Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplications with the
 * round keys bumped by the Weyl constants between rounds. */
static void mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, x0, &hi0, &lo0);
        mulhilo(0xCD9E8D57u, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* R3: spectral/octant variate, 32 bits plus one half ulp -> (0, 1), exact in double. */
static double u01a(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }
/* R3: direction variate, top 23 bits plus one half ulp -> (0, 1), exact in float and double. */
static double u01d(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

/* ---------------------------------------------------------------- tables (Sec. 2.2) */
static int lerp_table(const double *tab, int nT, double T0, double dT, double T, double *out)
{
    double u = (T - T0) / dT;
    if (!(u >= 0.0 && u <= (double)(nT - 1))) return ORC_OUT_OF_RANGE;   /* R6, also NaN */
    int t = (int)floor(u);
    if (t > nT - 2) t = nT - 2;
    double f = u - (double)t;
    *out = tab[t] + f * (tab[t + 1] - tab[t]);
    return ORC_OK;
}

static const double *ktab(const orc_problem *P, int s, int n, int g)
{
    return P->k + (((size_t)s * P->nb + n) * P->ng + g) * (size_t)P->nT;
}

/* kappa_{n,g} at temperature T and composition x[0..ns) (R7). */
static int kappa_at(const orc_problem *P, int n, int g, double T, const double *x, size_t xstride,
                    double *out)
{
    double kap = 0.0;
    for (int s = 0; s < P->ns; ++s) {
        double ks;
        int e = lerp_table(ktab(P, s, n, g), P->nT, P->T0, P->dT, T, &ks);
        if (e) return e;
        kap += x[s * xstride] * ks;
    }
    *out = kap;
    return ORC_OK;
}

static int planck_at(const orc_problem *P, int n, double T, double *out)
{
    return lerp_table(P->Ib + (size_t)n * P->nT, P->nT, P->T0, P->dT, T, out);
}

static size_t ncells_of(const orc_problem *P) { return (size_t)P->nx * P->ny * P->nz; }

static int cell_kappa(const orc_problem *P, size_t c, int n, int g, double *out)
{
    return kappa_at(P, n, g, P->T[c], P->X + c, ncells_of(P), out);
}

static int cell_planck(const orc_problem *P, size_t c, int n, double *out)
{
    return planck_at(P, n, P->T[c], out);
}

/* ------------------------------------------------ spectral pdf at T_max (Eqs. 13, 16)
 * e_{n,g} = pi dnu_n w_g kappa_{n,g}(T_max, xhat) I_n(T_max); p = e / sum e.
 * cdf_b[n] = sum_{n' <= n} sum_g e_{n',g} / E, cdf_g[n][g] = sum_{g' <= g} e_{n,g'} / e_n,
 * the last entry of each forced to 1.  The sums run sequentially in index order. */
int orc_plain_pdf(const orc_problem *P, double *p, double *cdf_b, double *cdf_g, double *Tmax_out)
{
    size_t nc = ncells_of(P);
    double Tmax = P->Tw[0] > P->Tw[1] ? P->Tw[0] : P->Tw[1];
    if (P->closed)
        for (int q = 0; q < 2; ++q) {
            if (P->Tx[q] > Tmax) Tmax = P->Tx[q];
            if (P->Tz[q] > Tmax) Tmax = P->Tz[q];
        }
    for (size_t c = 0; c < nc; ++c)
        if (P->T[c] > Tmax) Tmax = P->T[c];
    double *xhat = (double *)malloc(sizeof(double) * (P->ns > 0 ? P->ns : 1));
    for (int s = 0; s < P->ns; ++s) {            /* R8 */
        double m = 0.0;
        for (size_t c = 0; c < nc; ++c)
            if (P->X[(size_t)s * nc + c] > m) m = P->X[(size_t)s * nc + c];
        xhat[s] = m;
    }
    double E = 0.0;
    int err = ORC_OK;
    double *e = (double *)malloc(sizeof(double) * P->nb * P->ng);
    double *eb = (double *)malloc(sizeof(double) * P->nb);
    for (int n = 0; n < P->nb && !err; ++n) {
        double In;
        err = planck_at(P, n, Tmax, &In);
        eb[n] = 0.0;
        for (int g = 0; g < P->ng && !err; ++g) {
            double kap = 0.0;
            err = kappa_at(P, n, g, Tmax, xhat, 1, &kap);
            double v = M_PI * P->dnu[n] * P->wg[g] * kap * In;
            e[n * P->ng + g] = v;
            eb[n] += v;
        }
        E += eb[n];
    }
    if (!err && !(E > 0.0)) {      /* R13: nothing emits at T_max, every ray value is 0 */
        E = 0.0;
        for (int n = 0; n < P->nb; ++n) {
            eb[n] = 0.0;
            for (int g = 0; g < P->ng; ++g) { e[n * P->ng + g] = 1.0; eb[n] += 1.0; }
            E += eb[n];
        }
    }
    if (!err) {
        double run = 0.0;
        for (int n = 0; n < P->nb; ++n) {
            run += eb[n];
            cdf_b[n] = run / E;
            double rg = 0.0;
            for (int g = 0; g < P->ng; ++g) {
                rg += e[n * P->ng + g];
                p[n * P->ng + g] = e[n * P->ng + g] / E;
                cdf_g[n * P->ng + g] = eb[n] > 0.0 ? rg / eb[n] : (double)(g + 1) / P->ng;
            }
            cdf_g[n * P->ng + P->ng - 1] = 1.0;
        }
        cdf_b[P->nb - 1] = 1.0;
    }
    if (Tmax_out) *Tmax_out = Tmax;
    free(e); free(eb); free(xhat);
    return err;
}

/* first index i with u < cdf[i] (inversion of Eq. 17 as a search on cumulative sums) */
static int search_cdf(const double *cdf, int n, double u)
{
    for (int i = 0; i < n; ++i)
        if (u < cdf[i]) return i;
    return n - 1;
}

/* ----------------------------------------------------------- march (Algorithm 1) */
typedef struct {
    double acc, absacc;
    int steps, end;
    double wacc;     /* wall term tau_w eps (I_src - I_w) of the black wall that ended the ray */
    int wall;        /* that wall: 0 x0, 1 x1, 2 y0, 3 y1, 4 z0, 5 z1; -1 none */
    int wface;       /* its face element: (j, k) on x walls, (i, k) on y, (i, j) on z, row-major */
} orc_march_out;

static double face_coord(const double *f, int n, int local, int wrap)
{
    return f[local] + (double)wrap * (f[n] - f[0]);
}

/* Wall (axis a: 0 x, 1 y, 2 z; side 0 low, 1 high): temperature, emissivity, end code. */
static void wall_of(const orc_problem *P, int a, int side, double *Tw, double *eps, int *code)
{
    if (a == 1) { *Tw = P->Tw[side]; *eps = P->epsw[side]; *code = 1 + side; }
    else if (a == 0) { *Tw = P->Tx[side]; *eps = P->epsx[side]; *code = 4 + side; }
    else { *Tw = P->Tz[side]; *eps = P->epsz[side]; *code = 6 + side; }
}

/* Wall terms of the walls the last step ended on (hit[a]: 0 none, 1 low, 2 high), in the
 * order x, y, z (R4, R14): tau eps (I_src - I_w) each, tau *= 1 - eps; the ray is mirrored
 * on every reflecting wall (cell index back to the wall cell, origin and direction component
 * mirrored, next-face parameter of that axis from the mirrored origin).  Returns 1 when a
 * black wall ends the ray (*end set), 0 otherwise, or an error code in *err. */
static int walls(const orc_problem *P, int n, const int hit[3], const int nn[3], const double *const f[3],
                 int idx[3], const int wrap[3], double o[3], double dd[3], int sg[3], double tn[3], double Isrc,
                 double *tau, double *acc, double *absacc, int *end, double *wacc, int *wall, int *err)
{
    for (int a = 0; a < 3; ++a) {
        if (!hit[a]) continue;
        const int side = hit[a] - 1;
        double Tw, eps, Iw;
        int code;
        wall_of(P, a, side, &Tw, &eps, &code);
        if ((*err = planck_at(P, n, Tw, &Iw))) return 0;
        const double term = *tau * eps * (Isrc - Iw);
        *acc += term;
        *absacc += *tau * eps * fabs(Isrc - Iw);
        *tau *= 1.0 - eps;
        if (eps == 1.0) { *end = code; *wacc = term; *wall = 2 * a + side; return 1; }
        idx[a] = side ? nn[a] - 1 : 0;                          /* R14 */
        o[a] = 2.0 * f[a][side ? nn[a] : 0] - o[a];
        dd[a] = -dd[a];
        sg[a] = -sg[a];
        tn[a] = (face_coord(f[a], nn[a], idx[a] + (sg[a] > 0), wrap[a]) - o[a]) / dd[a];
    }
    return 0;
}

/* March one ray from the centre of cell (ci,cj,ck) (R1) along unit direction d for band n,
 * g-point g.  x and z are periodic unless the box is closed (R15); walls per R4 and R14.  If
 * rec_cells is non-null, the natural index and the segment length of each step are
 * recorded. */
int orc_march(const orc_problem *P, int ci, int cj, int ck, int n, int g, const double d[3],
              orc_march_out *res, int64_t *rec_cells, double *rec_ds, int rec_max)
{
    const int nn[3] = {P->nx, P->ny, P->nz};
    const double *const f[3] = {P->xf, P->yf, P->zf};
    const int per[3] = {!P->closed, 0, !P->closed};
    size_t csrc = ((size_t)ci * nn[1] + cj) * nn[2] + ck;
    double o[3] = {0.5 * (P->xf[ci] + P->xf[ci + 1]), 0.5 * (P->yf[cj] + P->yf[cj + 1]),
                   0.5 * (P->zf[ck] + P->zf[ck + 1])};
    double dd[3] = {d[0], d[1], d[2]}, tn[3];
    int idx[3] = {ci, cj, ck}, wrap[3] = {0, 0, 0}, sg[3];
    for (int a = 0; a < 3; ++a) {
        sg[a] = dd[a] > 0.0 ? 1 : -1;
        tn[a] = (face_coord(f[a], nn[a], idx[a] + (sg[a] > 0), wrap[a]) - o[a]) / dd[a];
    }
    double Isrc, Ilast, t = 0.0, tau = 1.0, acc = 0.0, absacc = 0.0, wacc = 0.0;
    int wall = -1;
    int e = cell_planck(P, csrc, n, &Isrc);
    if (e) return e;
    Ilast = Isrc;
    int steps = 0, end = 0;
    while (tau > P->tol && steps < P->max_steps) {
        double te = tn[0] < tn[1] ? tn[0] : tn[1];
        if (tn[2] < te) te = tn[2];
        double ds = te - t;
        size_t c = ((size_t)idx[0] * nn[1] + idx[1]) * nn[2] + idx[2];
        double kap, Ij;
        if ((e = cell_kappa(P, c, n, g, &kap)) || (e = cell_planck(P, c, n, &Ij))) return e;
        double alpha = -expm1(-kap * ds);                        /* Eq. 2, R10 */
        acc += tau * alpha * (Isrc - Ij);
        absacc += tau * alpha * fabs(Isrc - Ij);
        tau *= 1.0 - alpha;                                      /* Eq. 3 */
        if (rec_cells && steps < rec_max) { rec_cells[steps] = (int64_t)c; rec_ds[steps] = ds; }
        ++steps;
        t = te;
        Ilast = Ij;
        int hit[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {                            /* R5: every tied axis steps */
            if (tn[a] != te) continue;
            idx[a] += sg[a];
            if (per[a]) {
                if (idx[a] == nn[a]) { idx[a] = 0; ++wrap[a]; }
                if (idx[a] < 0) { idx[a] = nn[a] - 1; --wrap[a]; }
            } else if (idx[a] < 0 || idx[a] >= nn[a]) {
                hit[a] = idx[a] < 0 ? 1 : 2;
                continue;
            }
            tn[a] = (face_coord(f[a], nn[a], idx[a] + (sg[a] > 0), wrap[a]) - o[a]) / dd[a];
        }
        if (hit[0] | hit[1] | hit[2]) {
            int stop = walls(P, n, hit, nn, f, idx, wrap, o, dd, sg, tn, Isrc, &tau, &acc, &absacc, &end, &wacc,
                             &wall, &e);
            if (e) return e;
            if (stop) break;
        }
    }
    if (wall >= 0) {   /* the face element the ray reached: in-plane indices, clamped to the grid */
        int cl[3];
        for (int a = 0; a < 3; ++a) cl[a] = idx[a] < 0 ? 0 : (idx[a] >= nn[a] ? nn[a] - 1 : idx[a]);
        const int a = wall / 2;
        res->wface = a == 0 ? cl[1] * nn[2] + cl[2] : (a == 1 ? cl[0] * nn[2] + cl[2] : cl[0] * nn[1] + cl[1]);
    } else {
        res->wface = -1;
    }
    res->wacc = wacc;
    res->wall = wall;
    if (end == 0 && steps >= P->max_steps && tau > P->tol) end = 3;
    acc += tau * (Isrc - Ilast);                                 /* residual dump, R11 */
    absacc += tau * fabs(Isrc - Ilast);
    res->acc = acc;
    res->absacc = absacc;
    res->steps = steps;
    res->end = end;
    return ORC_OK;
}

/* ------------------------------------------- multigrid march (Sec. 4.3, readings M1-M3) */
#define ORC_MAX_LEV 8

typedef struct {
    int nlev;
    int n[ORC_MAX_LEV][3];        /* cells per axis of each level */
    const double *f[ORC_MAX_LEV][3];  /* face coordinates of each level */
    const double *T[ORC_MAX_LEV];     /* cell temperatures, natural order of the level */
    const double *X[ORC_MAX_LEV];     /* [ns][cells of the level] */
    double *owned[ORC_MAX_LEV][5];    /* coarse-level arrays allocated here */
} orc_levels;

/* M1: number of levels the grid allows. */
int orc_level_count(int nx, int ny, int nz)
{
    int L = 1;
    while (L < ORC_MAX_LEV && nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx / 2 >= 3 && ny / 2 >= 3 &&
           nz / 2 >= 3) {
        nx /= 2; ny /= 2; nz /= 2;
        ++L;
    }
    return L;
}

/* M2: volume-weighted mean of T and of each mole fraction over the DNS cells of every cell of
 * level L (written out over the DNS cells, not level by level). */
static void coarse_fields(const orc_problem *P, int L, double *T_out, double *X_out)
{
    const int b = 1 << L, mx = P->nx >> L, my = P->ny >> L, mz = P->nz >> L;
    const size_t nc = ncells_of(P), ncl = (size_t)mx * my * mz;
    for (int I = 0; I < mx; ++I)
        for (int J = 0; J < my; ++J)
            for (int K = 0; K < mz; ++K) {
                double vs = 0.0, ts = 0.0, xs[8] = {0};
                for (int i = I * b; i < (I + 1) * b; ++i)
                    for (int j = J * b; j < (J + 1) * b; ++j)
                        for (int k = K * b; k < (K + 1) * b; ++k) {
                            double v = (P->xf[i + 1] - P->xf[i]) * (P->yf[j + 1] - P->yf[j]) *
                                       (P->zf[k + 1] - P->zf[k]);
                            size_t c = ((size_t)i * P->ny + j) * P->nz + k;
                            vs += v;
                            ts += v * P->T[c];
                            for (int s = 0; s < P->ns && s < 8; ++s) xs[s] += v * P->X[(size_t)s * nc + c];
                        }
                size_t cl = ((size_t)I * my + J) * mz + K;
                T_out[cl] = ts / vs;
                for (int s = 0; s < P->ns && s < 8; ++s) X_out[(size_t)s * ncl + cl] = xs[s] / vs;
            }
}

int orc_coarse_fields(const orc_problem *P, int L, double *T_out, double *X_out)
{
    if (L < 0 || L >= orc_level_count(P->nx, P->ny, P->nz) || P->ns > 8) return ORC_INVALID;
    coarse_fields(P, L, T_out, X_out);
    return ORC_OK;
}

static void free_levels(orc_levels *G)
{
    for (int L = 0; L < ORC_MAX_LEV; ++L)
        for (int q = 0; q < 5; ++q) {
            free(G->owned[L][q]);
            G->owned[L][q] = 0;
        }
}

static int build_levels(const orc_problem *P, orc_levels *G)
{
    memset(G, 0, sizeof *G);
    int nl = P->mg_levels < 1 ? 1 : P->mg_levels;
    if (nl > orc_level_count(P->nx, P->ny, P->nz) || P->ns > 8) return ORC_INVALID;
    G->nlev = nl;
    for (int L = 0; L < nl; ++L) {
        int n[3] = {P->nx >> L, P->ny >> L, P->nz >> L};
        const double *f0[3] = {P->xf, P->yf, P->zf};
        for (int a = 0; a < 3; ++a) G->n[L][a] = n[a];
        if (L == 0) {
            for (int a = 0; a < 3; ++a) G->f[0][a] = f0[a];
            G->T[0] = P->T;
            G->X[0] = P->X;
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            double *f = malloc(sizeof(double) * (n[a] + 1));
            for (int q = 0; q <= n[a]; ++q) f[q] = f0[a][q << L];
            G->owned[L][a] = f;
            G->f[L][a] = f;
        }
        size_t ncl = (size_t)n[0] * n[1] * n[2];
        double *T = malloc(sizeof(double) * ncl), *X = malloc(sizeof(double) * ncl * P->ns);
        coarse_fields(P, L, T, X);
        G->owned[L][3] = T;
        G->owned[L][4] = X;
        G->T[L] = T;
        G->X[L] = X;
    }
    return ORC_OK;
}

/* March of one ray on the overlaid grids (M3); otherwise step for step the march of
 * orc_march.  Recorded cells carry their level in bits 48 and up. */
static int march_levels(const orc_problem *P, const orc_levels *G, int ci, int cj, int ck, int n, int g,
                        const double d[3], orc_march_out *res, int64_t *rec_cells, double *rec_ds, int rec_max)
{
    int L = 0, lsteps = 0;
    int nn[3] = {G->n[0][0], G->n[0][1], G->n[0][2]};
    const double *f[3] = {G->f[0][0], G->f[0][1], G->f[0][2]};
    const int per[3] = {!P->closed, 0, !P->closed};
    size_t csrc = ((size_t)ci * P->ny + cj) * P->nz + ck;
    double o[3] = {0.5 * (P->xf[ci] + P->xf[ci + 1]), 0.5 * (P->yf[cj] + P->yf[cj + 1]),
                   0.5 * (P->zf[ck] + P->zf[ck + 1])};
    double dd[3] = {d[0], d[1], d[2]}, tn[3];
    int idx[3] = {ci, cj, ck}, wrap[3] = {0, 0, 0}, sg[3];
    for (int a = 0; a < 3; ++a) {
        sg[a] = dd[a] > 0.0 ? 1 : -1;
        tn[a] = (face_coord(f[a], nn[a], idx[a] + (sg[a] > 0), wrap[a]) - o[a]) / dd[a];
    }
    double Isrc, Ilast, t = 0.0, tau = 1.0, acc = 0.0, absacc = 0.0, wacc = 0.0;
    int wall = -1;
    int e = cell_planck(P, csrc, n, &Isrc);
    if (e) return e;
    Ilast = Isrc;
    int steps = 0, end = 0;
    while (tau > P->tol && steps < P->max_steps) {
        if (L + 1 < G->nlev && lsteps == P->mg_steps) {         /* M3: fall onto the coarser grid */
            ++L;
            lsteps = 0;
            for (int a = 0; a < 3; ++a) {
                nn[a] = G->n[L][a];
                f[a] = G->f[L][a];
                idx[a] /= 2;
                tn[a] = (face_coord(f[a], nn[a], idx[a] + (sg[a] > 0), wrap[a]) - o[a]) / dd[a];
            }
        }
        double te = tn[0] < tn[1] ? tn[0] : tn[1];
        if (tn[2] < te) te = tn[2];
        double ds = te - t;
        size_t c = ((size_t)idx[0] * nn[1] + idx[1]) * nn[2] + idx[2], ncl = (size_t)nn[0] * nn[1] * nn[2];
        double kap, Ij;
        if ((e = kappa_at(P, n, g, G->T[L][c], G->X[L] + c, ncl, &kap)) ||
            (e = planck_at(P, n, G->T[L][c], &Ij)))
            return e;
        double alpha = -expm1(-kap * ds);                        /* Eq. 2, R10 */
        acc += tau * alpha * (Isrc - Ij);
        absacc += tau * alpha * fabs(Isrc - Ij);
        tau *= 1.0 - alpha;                                      /* Eq. 3 */
        if (rec_cells && steps < rec_max) { rec_cells[steps] = (int64_t)c | ((int64_t)L << 48); rec_ds[steps] = ds; }
        ++steps;
        ++lsteps;
        t = te;
        Ilast = Ij;
        int hit[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {                            /* R5 */
            if (tn[a] != te) continue;
            idx[a] += sg[a];
            if (per[a]) {
                if (idx[a] == nn[a]) { idx[a] = 0; ++wrap[a]; }
                if (idx[a] < 0) { idx[a] = nn[a] - 1; --wrap[a]; }
            } else if (idx[a] < 0 || idx[a] >= nn[a]) {
                hit[a] = idx[a] < 0 ? 1 : 2;
                continue;
            }
            tn[a] = (face_coord(f[a], nn[a], idx[a] + (sg[a] > 0), wrap[a]) - o[a]) / dd[a];
        }
        if (hit[0] | hit[1] | hit[2]) {
            int stop = walls(P, n, hit, nn, f, idx, wrap, o, dd, sg, tn, Isrc, &tau, &acc, &absacc, &end, &wacc,
                             &wall, &e);
            if (e) return e;
            if (stop) break;
        }
    }
    if (wall >= 0) {   /* the face element the ray reached: in-plane indices, clamped to the grid */
        int cl[3];
        for (int a = 0; a < 3; ++a) cl[a] = idx[a] < 0 ? 0 : (idx[a] >= nn[a] ? nn[a] - 1 : idx[a]);
        const int a = wall / 2;
        res->wface = a == 0 ? cl[1] * nn[2] + cl[2] : (a == 1 ? cl[0] * nn[2] + cl[2] : cl[0] * nn[1] + cl[1]);
    } else {
        res->wface = -1;
    }
    res->wacc = wacc;
    res->wall = wall;
    if (end == 0 && steps >= P->max_steps && tau > P->tol) end = 3;
    acc += tau * (Isrc - Ilast);                                 /* R11 */
    absacc += tau * fabs(Isrc - Ilast);
    res->acc = acc;
    res->absacc = absacc;
    res->steps = steps;
    res->end = end;
    return ORC_OK;
}

/* One ray of the multigrid march with the problem's mg_levels / mg_steps (levels built per
 * call: for tests of single rays). */
int orc_march_mg(const orc_problem *P, int ci, int cj, int ck, int n, int g, const double d[3],
                 orc_march_out *res, int64_t *rec_cells, double *rec_ds, int rec_max)
{
    orc_levels G;
    int e = build_levels(P, &G);
    if (!e) e = march_levels(P, &G, ci, cj, ck, n, g, d, res, rec_cells, rec_ds, rec_max);
    free_levels(&G);
    return e;
}

/* ------------------------------------------------------------ ray sampling per cell */
typedef struct {
    const double *p, *cdf_b, *cdf_g;   /* plain pdf and its cumulative sums */
} orc_plain;

/* Learned-allocation pdf of one cell: p_c(n,g,o) = (1 - eps) q_c(n,g,o) / sum q_c
 * + eps p(n,g)/8, with its band, g|n and o|n,g cumulative sums (sequential FP64). */
static void cell_pdf(const orc_problem *P, const orc_plain *pl, size_t c, double *pc,
                     double *cb, double *cg, double *co)
{
    const int nb = P->nb, ng = P->ng;
    const double *q = P->q_cell + c * (size_t)nb * ng * 8;
    double qs = 0.0;
    for (int i = 0; i < nb * ng * 8; ++i) qs += q[i];
    for (int n = 0; n < nb; ++n)
        for (int g = 0; g < ng; ++g)
            for (int o = 0; o < 8; ++o) {
                int i = (n * ng + g) * 8 + o;
                pc[i] = (1.0 - P->mix_eps) * (q[i] / qs) + P->mix_eps * (pl->p[n * ng + g] / 8.0);
            }
    double tot = 0.0;
    for (int i = 0; i < nb * ng * 8; ++i) tot += pc[i];
    double run = 0.0;
    for (int n = 0; n < nb; ++n) {
        double bn = 0.0;
        for (int i = 0; i < ng * 8; ++i) bn += pc[n * ng * 8 + i];
        run += bn;
        cb[n] = run / tot;
        double rg = 0.0;
        for (int g = 0; g < ng; ++g) {
            double gn = 0.0;
            for (int o = 0; o < 8; ++o) gn += pc[(n * ng + g) * 8 + o];
            rg += gn;
            cg[n * ng + g] = rg / bn;
            double ro = 0.0;
            for (int o = 0; o < 8; ++o) {
                ro += pc[(n * ng + g) * 8 + o];
                co[(n * ng + g) * 8 + o] = ro / gn;
            }
            co[(n * ng + g) * 8 + 7] = 1.0;
        }
        cg[n * ng + ng - 1] = 1.0;
    }
    cb[nb - 1] = 1.0;
    for (int i = 0; i < nb * ng * 8; ++i) pc[i] /= tot;
}

/* Start of wall w's face elements in the flat wall-flux layout x0 [ny][nz], x1, y0 [nx][nz],
 * y1, z0 [nx][ny], z1. */
static int wall_offset(const orc_problem *P, int w)
{
    const int fx = P->ny * P->nz, fy = P->nx * P->nz, fz = P->nx * P->ny;
    const int a = w / 2, side = w % 2;
    return a == 0 ? side * fx : (a == 1 ? 2 * fx + side * fy : 2 * fx + 2 * fy + side * fz);
}

/* All R rays of cell (ci,cj,ck): draws (Algorithm 1, Initialize), march, ray value. */
static int trace_cell(const orc_problem *P, const orc_plain *pl, const orc_levels *G, int ci, int cj, int ck,
                      orc_ray *out, double *work, double *yw_out, int *wf_out)
{
    const int nb = P->nb, ng = P->ng, R = P->R;
    size_t c = ((size_t)ci * P->ny + cj) * P->nz + ck;
    uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
    double *pc = 0, *cb = 0, *cg = 0, *co = 0;
    if (P->q_cell) {
        pc = work;
        cb = pc + (size_t)nb * ng * 8;
        cg = cb + nb;
        co = cg + (size_t)nb * ng;
        cell_pdf(P, pl, c, pc, cb, cg, co);
    }
    double kap_src;
    for (int r = 0; r < R; ++r) {
        uint32_t ctr[4] = {(uint32_t)c, (uint32_t)r, 0u, (P->snap << 4) | TAG_ALLOC}, w[4];
        orc_philox(ctr, key, w);
        int n, g, o;
        double prob;
        if (!P->q_cell) {                 /* Eqs. 16-17 at T_max, octant uniform (R12) */
            n = search_cdf(pl->cdf_b, nb, u01a(w[0]));
            g = search_cdf(pl->cdf_g + (size_t)n * ng, ng, u01a(w[1]));
            o = (int)floor(8.0 * u01a(w[2]));
            prob = pl->p[n * ng + g] / 8.0;
        } else {
            n = search_cdf(cb, nb, u01a(w[0]));
            g = search_cdf(cg + (size_t)n * ng, ng, u01a(w[1]));
            o = search_cdf(co + ((size_t)n * ng + g) * 8, 8, u01a(w[2]));
            prob = pc[(n * ng + g) * 8 + o];
        }
        int kord = 0;
        for (int r2 = 0; r2 < r; ++r2)
            if (out[r2].n == n && out[r2].g == g && out[r2].o == o) ++kord;
        out[r].n = n; out[r].g = g; out[r].o = o; out[r].k = kord; out[r].p = prob;
    }
    for (int r = 0; r < R; ++r) {
        orc_ray *ry = &out[r];
        uint32_t ctr[4] = {(uint32_t)c, ((uint32_t)ry->n << 16) | ((uint32_t)ry->g << 8) | (uint32_t)ry->o,
                           (uint32_t)ry->k, (P->snap << 4) | TAG_DIR}, v[4];
        orc_philox(ctr, key, v);
        /* Eq. 9 with the polar axis along y (R2): mu = cos(theta) = 1 - 2 R_theta,
         * phi = 2 pi R_phi; signs set by the octant bits (R12). */
        double mu = 1.0 - 2.0 * u01d(v[0]);
        double phi = 2.0 * M_PI * u01d(v[1]);
        double s = sqrt((1.0 - mu) * (1.0 + mu));
        double d[3] = {fabs(s * cos(phi)), fabs(mu), fabs(s * sin(phi))};
        if (ry->o & 1) d[0] = -d[0];
        if (ry->o & 2) d[1] = -d[1];
        if (ry->o & 4) d[2] = -d[2];
        orc_march_out m;
        int e = G->nlev > 1 ? march_levels(P, G, ci, cj, ck, ry->n, ry->g, d, &m, 0, 0, 0)
                            : orc_march(P, ci, cj, ck, ry->n, ry->g, d, &m, 0, 0, 0);
        if (e) return e;
        if ((e = cell_kappa(P, c, ry->n, ry->g, &kap_src))) return e;
        /* Eq. 14 with R9: w = 4 pi dnu_n w_g / (8 p(n,g,o)) over the octant-resolved pdf */
        double wgt = 4.0 * M_PI * P->dnu[ry->n] * P->wg[ry->g] / (8.0 * ry->p);
        ry->Y = wgt * kap_src * m.acc;
        ry->absY = wgt * kap_src * m.absacc;
        ry->steps = m.steps;
        ry->end = m.end;
        if (yw_out) {   /* the wall part of the ray value and the wall face element it went to */
            yw_out[r] = m.wall >= 0 ? wgt * kap_src * m.wacc : 0.0;
            wf_out[r] = m.wall >= 0 ? wall_offset(P, m.wall) + m.wface : -1;
        }
    }
    return ORC_OK;
}

static int check_problem(const orc_problem *P)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1 || P->nb < 1 || P->ng < 1 || P->ng > 255 ||
        P->nb > 65535 || P->ns < 1 || P->nT < 2 || P->R < 1 || !(P->dT > 0.0) ||
        P->max_steps < 1 || !(P->tol >= 0.0) || P->mg_levels > orc_level_count(P->nx, P->ny, P->nz) ||
        (P->mg_levels > 1 && (P->mg_steps < 1 || P->ns > 8)))
        return ORC_INVALID;
    for (int q = 0; q < 2; ++q)                                  /* R4: 0 <= eps <= 1 */
        if (!(P->epsw[q] >= 0.0 && P->epsw[q] <= 1.0) ||
            (P->closed && !(P->epsx[q] >= 0.0 && P->epsx[q] <= 1.0 && P->epsz[q] >= 0.0 && P->epsz[q] <= 1.0)))
            return ORC_INVALID;
    return ORC_OK;
}

/* Per-ray records of all R rays of each listed cell (natural indices). */
int orc_trace_cells(const orc_problem *P, int ncell, const int64_t *cells, orc_ray *out)
{
    int err = check_problem(P);
    if (err) return err;
    double *p = malloc(sizeof(double) * P->nb * P->ng), *cb = malloc(sizeof(double) * P->nb),
           *cg = malloc(sizeof(double) * P->nb * P->ng);
    err = orc_plain_pdf(P, p, cb, cg, 0);
    orc_plain pl = {p, cb, cg};
    orc_levels G;
    if (!err) err = build_levels(P, &G);
    else memset(&G, 0, sizeof G);
    size_t wsz = P->q_cell ? (size_t)P->nb * P->ng * 8 * 2 + P->nb + P->nb * P->ng : 1;
    if (!err) {
#pragma omp parallel
        {
            double *work = malloc(sizeof(double) * wsz);
            int myerr = 0;
#pragma omp for schedule(dynamic, 4)
            for (int q = 0; q < ncell; ++q) {
                int64_t c = cells[q];
                int ci = (int)(c / ((int64_t)P->ny * P->nz));
                int cj = (int)((c / P->nz) % P->ny);
                int ck = (int)(c % P->nz);
                int e = trace_cell(P, &pl, &G, ci, cj, ck, out + (size_t)q * P->R, work, 0, 0);
                if (e) myerr = e;
            }
#pragma omp critical
            if (myerr && !err) err = myerr;
            free(work);
        }
    }
    free_levels(&G);
    free(p); free(cb); free(cg);
    return err;
}

/* Cell estimate: mean of the R ray values, its standard error, total ray-cell steps. */
int orc_divergence(const orc_problem *P, int ncell, const int64_t *cells, double *divq,
                   double *stderr_out, int64_t *steps_total, int nthreads)
{
    int err = check_problem(P);
    if (err) return err;
    size_t nc = ncells_of(P);
    int64_t nlist = cells ? ncell : (int64_t)nc;
    double *p = malloc(sizeof(double) * P->nb * P->ng), *cb = malloc(sizeof(double) * P->nb),
           *cg = malloc(sizeof(double) * P->nb * P->ng);
    err = orc_plain_pdf(P, p, cb, cg, 0);
    orc_plain pl = {p, cb, cg};
    orc_levels G;
    if (!err) err = build_levels(P, &G);
    else memset(&G, 0, sizeof G);
    size_t wsz = P->q_cell ? (size_t)P->nb * P->ng * 8 * 2 + P->nb + P->nb * P->ng : 1;
    int64_t steps = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    if (!err) {
#pragma omp parallel reduction(+ : steps)
        {
            orc_ray *rays = malloc(sizeof(orc_ray) * P->R);
            double *work = malloc(sizeof(double) * wsz);
            int myerr = 0;
#pragma omp for schedule(dynamic, 16)
            for (int64_t q = 0; q < nlist; ++q) {
                int64_t c = cells ? cells[q] : q;
                int ci = (int)(c / ((int64_t)P->ny * P->nz));
                int cj = (int)((c / P->nz) % P->ny);
                int ck = (int)(c % P->nz);
                int e = trace_cell(P, &pl, &G, ci, cj, ck, rays, work, 0, 0);
                if (e) { myerr = e; continue; }
                double sum = 0.0;
                for (int r = 0; r < P->R; ++r) { sum += rays[r].Y; steps += rays[r].steps; }
                double mean = sum / P->R, ss = 0.0;
                for (int r = 0; r < P->R; ++r) ss += (rays[r].Y - mean) * (rays[r].Y - mean);
                divq[q] = mean;
                if (stderr_out) stderr_out[q] = P->R > 1 ? sqrt(ss / (P->R - 1) / P->R) : 0.0;
            }
#pragma omp critical
            if (myerr && !err) err = myerr;
            free(rays); free(work);
        }
    }
    if (steps_total) *steps_total = steps;
    free_levels(&G);
    free(p); free(cb); free(cg);
    return err;
}

/* Net radiative flux from the gas into every wall face element [W m^-2] (black walls, one
 * grid): each ray that ended on a black wall carries the wall part of its value, Y_w = w
 * kappa_src tau_w (I_src - I_w) (the wall factor of Eq. 3 with emissivity 1, the weight of
 * Eq. 14); the element receives V_c Y_w / (R A_f) from it, V_c its source cell's volume and
 * A_f the element's area -- the cell's net power exchange with that element, whose expected
 * sum over the gas is the gas-to-wall part of the wall's net radiative flux.  Sums run over the
 * cells in natural order and their rays in order.  q: 2 (ny nz + nx nz + nx ny) doubles,
 * layout of wall_offset.  Reflecting walls or multigrid: ORC_UNSUPPORTED. */
int orc_wall_flux(const orc_problem *P, double *q)
{
    int err = check_problem(P);
    if (err) return err;
    for (int w = 0; w < 2; ++w)
        if (P->epsw[w] != 1.0 || (P->closed && (P->epsx[w] != 1.0 || P->epsz[w] != 1.0)))
            return ORC_UNSUPPORTED;
    if (P->mg_levels > 1) return ORC_UNSUPPORTED;
    const size_t nc = ncells_of(P);
    const int R = P->R;
    double *p = malloc(sizeof(double) * P->nb * P->ng), *cb = malloc(sizeof(double) * P->nb),
           *cg = malloc(sizeof(double) * P->nb * P->ng);
    double *yw = malloc(sizeof(double) * nc * R);
    int *wf = malloc(sizeof(int) * nc * R);
    err = orc_plain_pdf(P, p, cb, cg, 0);
    orc_plain pl = {p, cb, cg};
    orc_levels G;
    if (!err) err = build_levels(P, &G);
    else memset(&G, 0, sizeof G);
    size_t wsz = P->q_cell ? (size_t)P->nb * P->ng * 8 * 2 + P->nb + P->nb * P->ng : 1;
    if (!err) {
#pragma omp parallel
        {
            orc_ray *rays = malloc(sizeof(orc_ray) * R);
            double *work = malloc(sizeof(double) * wsz);
            int myerr = 0;
#pragma omp for schedule(dynamic, 16)
            for (int64_t c = 0; c < (int64_t)nc; ++c) {
                int ci = (int)(c / ((int64_t)P->ny * P->nz));
                int cj = (int)((c / P->nz) % P->ny);
                int ck = (int)(c % P->nz);
                int e = trace_cell(P, &pl, &G, ci, cj, ck, rays, work, yw + c * R, wf + c * R);
                if (e) myerr = e;
            }
#pragma omp critical
            if (myerr && !err) err = myerr;
            free(rays); free(work);
        }
    }
    if (!err) {
        const int fx = P->ny * P->nz, fy = P->nx * P->nz, fz = P->nx * P->ny;
        memset(q, 0, sizeof(double) * 2 * (fx + fy + fz));
        for (size_t c = 0; c < nc; ++c) {
            const int ci = (int)(c / ((size_t)P->ny * P->nz)), cj = (int)((c / P->nz) % P->ny),
                      ck = (int)(c % P->nz);
            const double vc = (P->xf[ci + 1] - P->xf[ci]) * (P->yf[cj + 1] - P->yf[cj]) * (P->zf[ck + 1] - P->zf[ck]);
            for (int r = 0; r < R; ++r) {
                const int f = wf[c * R + r];
                if (f < 0) continue;
                /* the element's area from its in-plane cell widths */
                double area;
                if (f < 2 * fx) {
                    const int e = f % fx, j = e / P->nz, k = e % P->nz;
                    area = (P->yf[j + 1] - P->yf[j]) * (P->zf[k + 1] - P->zf[k]);
                } else if (f < 2 * fx + 2 * fy) {
                    const int e = (f - 2 * fx) % fy, i = e / P->nz, k = e % P->nz;
                    area = (P->xf[i + 1] - P->xf[i]) * (P->zf[k + 1] - P->zf[k]);
                } else {
                    const int e = (f - 2 * fx - 2 * fy) % fz, i = e / P->ny, j = e % P->ny;
                    area = (P->xf[i + 1] - P->xf[i]) * (P->yf[j + 1] - P->yf[j]);
                }
                q[f] += vc * yw[c * R + r] / ((double)R * area);
            }
        }
    }
    free_levels(&G);
    free(p); free(cb); free(cg); free(yw); free(wf);
    return err;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
