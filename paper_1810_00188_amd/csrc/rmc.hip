// rmc.hip -- gfx950 implementation of the C ABI declared in include/rmc.h: the
// emission-based reciprocal Monte Carlo (ERMC) radiative heat source of Silvestri & Pecnik.
//
// Pipeline of one compute (all kernels on the caller's stream, no host round trip):
//   1. k_plain_pdf     T_max spectral pdf and its cumulative sums (Eqs. 13, 16-17), ray
//                      weights per (band, g, octant) bucket (Eq. 14), wall intensities.
//   2. k_records       one 16-byte record per cell (table coordinate of T, mole fractions) in a
//                      bricked layout, read by every (band, g) pair; the march interpolates
//                      kappa and I_n from its pair's tables in LDS at every step (Sec. 2.2).
//   3. k_alloc_count   per tile of cells: histogram of the rays' (n, g, octant) buckets.
//      k_bucket_scan   per bucket: exclusive scan over tiles (no global atomics).
//      k_run_len / k_run_layout: the work list runs region by region (compact groups of tiles),
//                      bucket by bucket inside a region; run starts padded to whole
//                      wavefronts.  k_chunk_map: chunk -> bucket map.
//      k_alloc_scatter per tile: ray work items into their bucket (narrow-band sorting of
//                      Sec. 4.2: a wavefront marches rays of one (n, g, octant)).
//   4. k_march_lane    one lane per ray, Algorithm 1 march, ray value into its slot; rays still
//      k_march_long    marching after long_ray_steps continue in parallel segments.
//   5. k_reduce        per cell: mean and standard error of the R ray values (FP64, or
//                      compensated / plain FP32), natural order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rmc.h"
#include "rmc_device.h"

using namespace rmc;

// Scratch of the allocation-free compute (rmc_compute_divergence_noalloc): per-compute work
// lists, ray slots, histograms and descriptors are carved from this array, which every GPU the
// library runs on holds until the process ends.  Host code reaches it only through the
// per-device address from hipGetSymbolAddress (taken at rmc_create), never by its name.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// ============================================================================ device side
namespace {

constexpr int kMaxLev = 8;      // grid levels of the multigrid march

struct SnapDesc {
    const uint4 *rec;           // [ncpad << rw_log2] cell records (table coordinate, mole fractions), bricked
    int rw_log2;                // 16-byte words per record, log2
    const double *W;            // [nbucket] plain ray weight 4 pi dnu w / (8 p(n,g,o))
    const double *Iw;           // [6][nb] wall intensities, walls x0, x1, y0, y1, z0, z1
    void *Y;                    // ray slots c * R + r: FP32 march {value bits, steps | end << 28} as
                                // one 8-byte record; FP64 march the double values, with
    uint32_t *st;               // [ncells * R] steps | end << 28 (FP64 march only)
    const double *p;            // [nb*ng] plain pdf
    const double *cdf_b;        // [nb]
    const double *cdf_g;        // [nb*ng]
    const double *cpdf;         // per-cell pdf mode: [ncells][nb*ng*8]
    const double *ccdf_b;       // [ncells][nb]
    const double *ccdf_g;       // [ncells][nb*ng]
    const double *ccdf_o;       // [ncells][nb*ng*8]
    const uint32_t *dstrat;     // learned sampling: [ncells * R] drawn stratum (n*ng + g)*8 + o
    double *dprob;              // per-cell pdf or learned sampling: [ncells * R] probability of each ray
    uint32_t *rbkt;             // [ncells * R] bucket (n*ng + g)*8 + o of each ray: written by the
                                // counting pass (learned sampling: the drawn strata themselves)
    uint64_t ncpad;             // cells of the padded, bricked record field
    int nx, ny, nz;
    int nbx, nby, nbz;
    int face_off;               // x faces at face_off, y at +nx+1, z at +nx+ny+2
    uint32_t snap_id;
    int tile_begin, ntiles;
    double Lx, Lz;
    double hx, hz;              // cell widths along x and z when those axes are uniform
    // multigrid march (Sec. 4.3): level L has (nx >> L) x (ny >> L) x (nz >> L) cells with
    // every 2^L-th face; its records follow the same bricked layout
    int nlev;                   // grid levels (1: the DNS grid only)
    int mg_steps;               // steps per level before the next coarser one
    int lev_face[kMaxLev];      // face tables of each level in the staged face array
    uint64_t lev_off[kMaxLev];  // first cell of level L >= 1 in the coarse records
    uint64_t mg_stride;         // cells of all coarse levels
    const uint4 *mg_rec;        // records of the coarse levels
    double epsw[6];             // wall emissivities, walls x0, x1, y0, y1, z0, z1
    int closed;                 // walls on x and z (closed box), else x and z periodic
    int reflect;                // some wall has emissivity below one
    double *wallq;              // wall flux tally (black walls, one grid) or null: x0 [ny][nz], x1,
                                // y0 [nx][nz], y1, z0 [nx][ny], z1
};

// An allocation tile: tile_cells consecutive cells of a snapshot's brick-linear order, and the
// region of the march order it belongs to.  Tiles are numbered region by region.
struct TileInfo {
    int snap;                   // snapshot of the tile
    uint32_t first;             // its first cell in the snapshot's brick-linear order
    uint32_t region;            // its region (numbered over the whole pass)
    uint32_t pad;
};

struct AllocArgs {
    const SnapDesc *snaps;
    const TileInfo *tiles;      // [ntiles]
    int ntiles, tile_cells;
    int nb, ng, nbucket, R;
    uint32_t k0, k1;
    uint32_t *hist;             // [nbucket][ntiles], scanned per bucket over the tiles
    const uint32_t *btotal;     // [nbucket] rays per bucket
    const uint32_t *rtile0;     // [nregion + 1] first tile of each region
    const uint32_t *rstart;     // [nregion][nbucket] start of each (region, bucket) run of the work list
    uint2 *items;               // (i | j<<10 | k<<20, r | k_ord<<8 | snapshot<<16)
    int lds_bricks;             // the tile's bricks are decoded into LDS (else per cell from the index)
    int lds_cdf;                // plain sampling, cdfs staged in LDS by the counting pass: 0 none, 1 bands, 2 both
};

struct Draw {
    int n, g, o;
    double p;
};

// Sampling modes: 0 the T_max pdf, 1 a per-cell pdf (rmc_set_cell_pdf), 2 the learned
// allocation (draws made per cell by k_alloc_draw, read back here).
template <int SM>
__device__ __forceinline__ Draw draw_ray(const SnapDesc &D, int nb, int ng, uint32_t c, uint32_t r,
                                         uint32_t k0, uint32_t k1, int R, const double *cdf_b = nullptr,
                                         const double *cdf_g = nullptr)
{
    if constexpr (SM == 2) {
        const size_t slot = (size_t)c * R + r;
        const uint32_t st = gld(D.dstrat + slot);
        Draw d;
        d.o = (int)(st & 7u);
        d.n = (int)(st >> 3) / ng;
        d.g = (int)(st >> 3) - d.n * ng;
        d.p = gld(D.dprob + slot);
        return d;
    }
    uint32_t w[4];
    philox4x32_10(c, r, 0u, (D.snap_id << 4) | kTagAlloc, k0, k1, w);
    const double u0 = unif_alloc(w[0]), u1 = unif_alloc(w[1]), u2 = unif_alloc(w[2]);
    Draw d;
    if constexpr (SM == 0) {
        // the caller may pass copies staged in LDS; a row of the g cdf in global memory is ranked
        // by independent loads
        d.n = cdf_search(cdf_b ? cdf_b : D.cdf_b, nb, u0);
        d.g = cdf_g ? cdf_search(cdf_g + (size_t)d.n * ng, ng, u1) : cdf_rank(D.cdf_g + (size_t)d.n * ng, ng, u1);
        d.o = (int)floor(8.0 * u2);
        d.p = D.p[d.n * ng + d.g] / 8.0;
    } else {
        const size_t cb = (size_t)c * nb, cg = (size_t)c * nb * ng;
        d.n = cdf_search(D.ccdf_b + cb, nb, u0);
        d.g = cdf_search(D.ccdf_g + cg + (size_t)d.n * ng, ng, u1);
        const size_t so = (cg + (size_t)d.n * ng + d.g) * 8;
        d.o = cdf_search(D.ccdf_o + so, 8, u2);
        d.p = D.cpdf[so + d.o];
    }
    return d;
}

// cell of a tile position: brick-linear index -> (i, j, k), valid if inside the grid
__device__ __forceinline__ bool brick_cell(const SnapDesc &D, uint64_t bc, int &i, int &j, int &k)
{
    const uint64_t brick = bc >> 6;
    const int w = (int)(bc & 63);
    const int bk = (int)(brick % D.nbz);
    const int bj = (int)((brick / D.nbz) % D.nby);
    const int bi = (int)(brick / ((uint64_t)D.nbz * D.nby));
    i = bi * 4 + ((w >> 2) & 1) + (((w >> 5) & 1) << 1);
    j = bj * 4 + ((w >> 1) & 1) + (((w >> 4) & 1) << 1);
    k = bk * 4 + (w & 1) + (((w >> 3) & 1) << 1);
    return bc < D.ncpad && i < D.nx && j < D.ny && k < D.nz;
}

// --------------------------------------------------------------------- field ingest
// block-wide max of non-negative doubles, one atomic per block (on the bit pattern, which
// orders non-negative doubles like the values)
__device__ __forceinline__ void block_max_atomic(double mx, unsigned long long *dst)
{
    __shared__ double wm[16];
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wm[wv] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wm[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, wm[q]);
        atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();
}

// block-wide min of non-negative doubles, one atomic per block
__device__ __forceinline__ void block_min_atomic(double mn, unsigned long long *dst)
{
    __shared__ double wm[16];
    for (int off = 32; off > 0; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off));
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wm[wv] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wm[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmin(m, wm[q]);
        atomicMin(dst, (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();
}

template <class Tin>
__global__ void __launch_bounds__(256) k_ingest_T(const Tin *__restrict__ in, double *__restrict__ out, uint64_t n,
                                                  double T0, double dT, int nT, unsigned long long *maxbits,
                                                  unsigned int *flag)
{
    double mx = 0.0, mn = INFINITY;
    bool bad = false;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const double v = (double)in[q];
        out[q] = v;
        const double u = (v - T0) / dT;
        if (!(u >= 0.0 && u <= (double)(nT - 1))) bad = true;
        else { mx = fmax(mx, v); mn = fmin(mn, v); }
    }
    if (bad) atomicOr(flag, 1u);
    block_max_atomic(mx, maxbits);
    block_min_atomic(mn, maxbits + 2);
}

// Reduction slots of the ingest kernels in the context's `small` buffer (64-bit words):
// mole fractions max [0, 8), min [8, 16), flag 16; temperature max 24, flag 25, min 26.
// Maxima start at 0, minima at a huge double (0x7F7F...), flags at 0.
constexpr int kSmallX = 0, kSmallT = 24, kSmallWords = 27;

__global__ void k_small_init(unsigned long long *small, int x, int t)
{
    const int q = (int)threadIdx.x;
    if (q >= kSmallWords) return;
    const bool in_x = x && q < 17, in_t = t && q >= kSmallT;
    if (!in_x && !in_t) return;
    const bool is_min = (q >= kSmallX + 8 && q < kSmallX + 16) || q == kSmallT + 2;
    small[q] = is_min ? 0x7F7F7F7F7F7F7F7Full : 0ull;
}

template <class Tin>
__global__ void __launch_bounds__(256) k_ingest_X(const Tin *__restrict__ in, double *__restrict__ out, uint64_t nc,
                                                  int ns, unsigned long long *maxbits, unsigned int *flag)
{
    for (int sp = 0; sp < ns; ++sp) {
        double mx = 0.0, mn = INFINITY;
        bool bad = false;
        for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nc;
             q += (uint64_t)gridDim.x * blockDim.x) {
            const double v = (double)in[(size_t)sp * nc + q];
            out[(size_t)sp * nc + q] = v;
            if (!(v >= 0.0 && v < INFINITY)) bad = true;
            else { mx = fmax(mx, v); mn = fmin(mn, v); }
        }
        if (bad) atomicOr(flag, 1u);
        block_max_atomic(mx, maxbits + sp);
        block_min_atomic(mn, maxbits + 8 + sp);
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void k_zero_f64(double *p, uint64_t n)
{
    const uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0.0;
}

__global__ void k_zero_u32(uint32_t *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// ------------------------------------------------------------- spectral pdf (1 thread)
__device__ __forceinline__ double lerp_tab(const double *tab, int nT, double T0, double dT, double T)
{
    const double u = (T - T0) / dT;
    int t = (int)floor(u);
    if (t > nT - 2) t = nT - 2;
    const double f = u - (double)t;
    return tab[t] + f * (tab[t + 1] - tab[t]);
}

struct PdfArgs {
    const double *k64;          // [ns][nb][ng][nT]
    const double *Ib;           // [nb][nT]
    const double *dnu, *wg;
    int nb, ng, ns, nT;
    double T0, dT;
    double Tw[6];               // wall temperatures x0, x1, y0, y1, z0, z1 (x / z: copies of y0
                                // unless the box is closed)
    const double *scal;         // [0]: max cell temperature, [1..ns]: largest mole fractions
    double *e;                  // scratch [nb*ng]
    double *eb;                 // scratch [nb]
    double *p, *cdf_b, *cdf_g, *W, *Iw;
    int *status;
};

// e_{n,g} = pi dnu_n w_g kappa_{n,g}(T_max, xhat) I_n(T_max); p = e / E; cumulative sums in
// index order (Eqs. 13, 16-17 at T_max, Zhang's sampling); W = 4 pi dnu w / (8 p / 8).
// One block: the independent terms in parallel, every running sum by one thread in index
// order (the same operations, in the same order, as the sequential definition).
__global__ void __launch_bounds__(256) k_plain_pdf(PdfArgs A)
{
    const int nb = A.nb, ng = A.ng, npair = nb * ng;
    __shared__ double E_sh;
    double Tmax = A.Tw[2] > A.Tw[3] ? A.Tw[2] : A.Tw[3];
    for (int w = 0; w < 6; ++w)
        if (A.Tw[w] > Tmax) Tmax = A.Tw[w];
    if (A.scal[0] > Tmax) Tmax = A.scal[0];
    for (int pr = threadIdx.x; pr < npair; pr += blockDim.x) {
        const int n = pr / ng, g = pr - (pr / ng) * ng;
        const double In = lerp_tab(A.Ib + (size_t)n * A.nT, A.nT, A.T0, A.dT, Tmax);
        double kap = 0.0;
        for (int sp = 0; sp < A.ns; ++sp) {
            const double ks = lerp_tab(A.k64 + (((size_t)sp * nb + n) * ng + g) * A.nT, A.nT, A.T0, A.dT, Tmax);
            kap += A.scal[1 + sp] * ks;
        }
        A.e[pr] = M_PI * A.dnu[n] * A.wg[g] * kap * In;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < nb; n += blockDim.x) {
        double eb = 0.0;
        for (int g = 0; g < ng; ++g) eb += A.e[n * ng + g];
        A.eb[n] = eb;
        for (int w = 0; w < 6; ++w) A.Iw[w * nb + n] = lerp_tab(A.Ib + (size_t)n * A.nT, A.nT, A.T0, A.dT, A.Tw[w]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double E = 0.0;
        for (int n = 0; n < nb; ++n) E += A.eb[n];
        if (!(E > 0.0)) {
            // nothing emits at T_max (all I_b or kappa zero): every ray value is exactly zero
            // for any positive pdf, so the uniform one is used
            E = 0.0;
            for (int n = 0; n < nb; ++n) {
                A.eb[n] = 0.0;
                for (int g = 0; g < ng; ++g) {
                    A.e[n * ng + g] = 1.0;
                    A.eb[n] += 1.0;
                }
                E += A.eb[n];
            }
        }
        double run = 0.0;
        for (int n = 0; n < nb; ++n) {
            run += A.eb[n];
            A.cdf_b[n] = run / E;
        }
        A.cdf_b[nb - 1] = 1.0;
        E_sh = E;
        *A.status = 0;
    }
    __syncthreads();
    const double E = E_sh;
    for (int n = threadIdx.x; n < nb; n += blockDim.x) {
        double rg = 0.0;
        for (int g = 0; g < ng; ++g) {
            rg += A.e[n * ng + g];
            A.p[n * ng + g] = A.e[n * ng + g] / E;
            A.cdf_g[n * ng + g] = A.eb[n] > 0.0 ? rg / A.eb[n] : (double)(g + 1) / ng;
        }
        A.cdf_g[n * ng + ng - 1] = 1.0;
    }
    __syncthreads();
    for (int pr = threadIdx.x; pr < npair; pr += blockDim.x) {
        const int n = pr / ng, g = pr - (pr / ng) * ng;
        const double prob = A.p[pr] / 8.0;
        const double w = prob > 0.0 ? 4.0 * M_PI * A.dnu[n] * A.wg[g] / (8.0 * prob) : 0.0;
        for (int o = 0; o < 8; ++o) A.W[pr * 8 + o] = w;
    }
}

// Per-cell allocation pdf p_c = (1 - eps) q_c / sum q_c + eps p_plain / 8 and its band,
// g | band and octant | (band, g) cumulative sums, one thread per cell, sequential FP64 in
// index order.
__global__ void k_cell_pdf(const double *__restrict__ q, const double *__restrict__ pplain, uint64_t nc,
                           int nb, int ng, double eps, double *cpdf, double *cb, double *cg, double *co)
{
    const uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int m = nb * ng * 8;
    const double *qc = q + c * m;
    double *pc = cpdf + c * m, *cbc = cb + c * nb, *cgc = cg + c * (size_t)nb * ng, *coc = co + c * m;
    double qs = 0.0;
    for (int i = 0; i < m; ++i) qs += qc[i];
    for (int n = 0; n < nb; ++n)
        for (int g = 0; g < ng; ++g)
            for (int o = 0; o < 8; ++o) {
                const int i = (n * ng + g) * 8 + o;
                pc[i] = (1.0 - eps) * (qc[i] / qs) + eps * (pplain[n * ng + g] / 8.0);
            }
    double tot = 0.0;
    for (int i = 0; i < m; ++i) tot += pc[i];
    double run = 0.0;
    for (int n = 0; n < nb; ++n) {
        double bn = 0.0;
        for (int i = 0; i < ng * 8; ++i) bn += pc[n * ng * 8 + i];
        run += bn;
        cbc[n] = run / tot;
        double rg = 0.0;
        for (int g = 0; g < ng; ++g) {
            double gn = 0.0;
            for (int o = 0; o < 8; ++o) gn += pc[(n * ng + g) * 8 + o];
            rg += gn;
            cgc[n * ng + g] = rg / bn;
            double ro = 0.0;
            for (int o = 0; o < 8; ++o) {
                ro += pc[(n * ng + g) * 8 + o];
                coc[(n * ng + g) * 8 + o] = ro / gn;
            }
            coc[(n * ng + g) * 8 + 7] = 1.0;
        }
        cgc[n * ng + ng - 1] = 1.0;
    }
    cbc[nb - 1] = 1.0;
    for (int i = 0; i < m; ++i) pc[i] /= tot;
}

// ------------------------------------------------------------------ cell records
// rec[brick(i,j,k)] = {u = (T_c - T0) / dT (FP64), x_s(c) in march precision}: the table
// coordinate of the linear interpolation in T (Sec. 2.2) and the mole fractions of the mixture,
// from which the march interpolates kappa_{n,g} and I_n of any (band, g) pair.  Padding cells
// hold zeros (never read).
template <class Real>
__global__ void __launch_bounds__(256) k_records(const double *__restrict__ T, const double *__restrict__ X, int ns,
                                                 uint64_t nc, double T0, double dT, SnapDesc D,
                                                 uint4 *__restrict__ rec)
{
    const uint64_t bc = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (bc >= D.ncpad) return;
    int i, j, k;
    const bool valid = brick_cell(D, bc, i, j, k);
    const int rw = 1 << D.rw_log2;
    uint32_t w[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) w[q] = 0u;
    if (valid) {
        const uint64_t c = ((uint64_t)i * D.ny + j) * D.nz + k;
        const double u = (T[c] - T0) / dT;
        w[0] = (uint32_t)__double2loint(u);
        w[1] = (uint32_t)__double2hiint(u);
#pragma unroll
        for (int sp = 0; sp < 8; ++sp) {
            if (sp >= ns) break;
            const double x = X[(size_t)sp * nc + c];
            if constexpr (sizeof(Real) == 4) {
                w[2 + sp] = __float_as_uint((float)x);
            } else {
                w[2 + 2 * sp] = (uint32_t)__double2loint(x);
                w[3 + 2 * sp] = (uint32_t)__double2hiint(x);
            }
        }
    }
    uint4 *out = rec + (bc << D.rw_log2);
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < rw) out[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// Fields of the next coarser grid (multigrid march, Sec. 4.3): each coarse cell takes the
// volume-weighted mean temperature and mole fractions of the 2 x 2 x 2 cells of the level
// below (nx x ny x nz cells with faces xf, yf, zf), natural order.
__global__ void __launch_bounds__(256) k_coarsen(const double *__restrict__ T, const double *__restrict__ X, int ns,
                                                 int nx, int ny, int nz, const double *__restrict__ xf,
                                                 const double *__restrict__ yf, const double *__restrict__ zf,
                                                 double *__restrict__ Tc, double *__restrict__ Xc)
{
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const uint64_t ncc = (uint64_t)cx * cy * cz, nc = (uint64_t)nx * ny * nz;
    const uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (q >= ncc) return;
    const int K = (int)(q % cz), J = (int)((q / cz) % cy), I = (int)(q / ((uint64_t)cz * cy));
    double vs = 0.0, ts = 0.0, xs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) {
                const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + e;
                const double v = (xf[i + 1] - xf[i]) * (yf[j + 1] - yf[j]) * (zf[k + 1] - zf[k]);
                const uint64_t c = ((uint64_t)i * ny + j) * nz + k;
                vs += v;
                ts += v * T[c];
                for (int sp = 0; sp < ns; ++sp) xs[sp] += v * X[(size_t)sp * nc + c];
            }
    Tc[q] = ts / vs;
    for (int sp = 0; sp < ns; ++sp) Xc[(size_t)sp * ncc + q] = xs[sp] / vs;
}

// ------------------------------------------------------------- allocation and buckets
// Rays of one tile: cells [tile_begin.., +tile_cells) of the brick-linear order, all R rays
// of each cell in one pass of the block (cells_per_pass = blockDim / R).
constexpr int kAllocThreads = 1024;   // threads per tile: R rays of 1024 / R cells per pass

// Workgroup barrier that orders LDS accesses only: global loads and stores in flight stay in
// flight (__syncthreads waits for them too), for loops whose barriers guard LDS data alone.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The bricks of a tile (tile_cells is a multiple of 64: whole bricks), decoded once into LDS as
// bi | bj << 10 | bk << 20, or ~0 past the last brick of the snapshot.
__device__ __forceinline__ void tile_bricks(const SnapDesc &D, uint64_t first, int tile_cells, uint32_t *bt)
{
    const uint32_t nbt = (uint32_t)tile_cells >> 6, b0 = (uint32_t)(first >> 6);
    const uint32_t nbricks = (uint32_t)(D.ncpad >> 6);
    for (uint32_t q = threadIdx.x; q < nbt; q += blockDim.x) {
        const uint32_t b = b0 + q;
        uint32_t v = 0xFFFFFFFFu;
        if (b < nbricks) {
            const uint32_t bk = b % (uint32_t)D.nbz, t = b / (uint32_t)D.nbz;
            v = (t / (uint32_t)D.nby) | ((t % (uint32_t)D.nby) << 10) | (bk << 20);
        }
        bt[q] = v;
    }
}

// Cell (i, j, k) at position p of the tile (the same order as brick_cell); false outside the grid.
__device__ __forceinline__ bool tile_cell(const SnapDesc &D, const uint32_t *bt, int p, int &i, int &j, int &k)
{
    const uint32_t v = bt[p >> 6];
    const int w = p & 63;
    i = (int)(v & 1023u) * 4 + ((w >> 2) & 1) + (((w >> 5) & 1) << 1);
    j = (int)((v >> 10) & 1023u) * 4 + ((w >> 1) & 1) + (((w >> 4) & 1) << 1);
    k = (int)(v >> 20) * 4 + (w & 1) + (((w >> 3) & 1) << 1);
    return v != 0xFFFFFFFFu && i < D.nx && j < D.ny && k < D.nz;
}

// LDS of k_alloc_count: the plain cdfs staged (cdf 1: the band cdf, nb doubles; 2: also the g
// cdfs, nb*ng), then nbucket counters, then the tile's bricks (if decoded there).
inline size_t alloc_count_lds(int cdf, bool bricks, int nb, int ng, int nbucket, int tile_cells)
{
    return sizeof(double) * (cdf == 2 ? nb + nb * ng : cdf == 1 ? nb : 0) +
           sizeof(uint32_t) * (nbucket + (bricks ? tile_cells / 64 : 0));
}

// Cell at position p of the tile, from the decoded bricks or from the brick-linear index.
__device__ __forceinline__ bool alloc_cell(const SnapDesc &D, const uint32_t *bt, uint64_t first, int p, int &i,
                                           int &j, int &k)
{
    return bt ? tile_cell(D, bt, p, i, j, k) : brick_cell(D, first + p, i, j, k);
}

template <int SM>
__global__ void __launch_bounds__(kAllocThreads) k_alloc_count(AllocArgs A)
{
    extern __shared__ double lds_d[];
    const int cdf = SM == 0 ? A.lds_cdf : 0;
    const int ncdf = cdf == 2 ? A.nb + A.nb * A.ng : cdf == 1 ? A.nb : 0;
    uint32_t *lh = reinterpret_cast<uint32_t *>(lds_d + ncdf);   // [nbucket]
    uint32_t *bt = A.lds_bricks ? lh + A.nbucket : nullptr;        // [tile_cells / 64]
    const int tile = blockIdx.x;
    const TileInfo TI = A.tiles[tile];
    const SnapDesc D = A.snaps[TI.snap];   // a copy: its fields stay in registers across the stores
    const uint64_t first = TI.first;
    for (int b = threadIdx.x; b < A.nbucket; b += blockDim.x) lh[b] = 0;
    if (cdf) {
        for (int q = threadIdx.x; q < A.nb; q += blockDim.x) lds_d[q] = D.cdf_b[q];
        if (cdf == 2)
            for (int q = threadIdx.x; q < A.nb * A.ng; q += blockDim.x) lds_d[A.nb + q] = D.cdf_g[q];
    }
    if (bt) tile_bricks(D, first, A.tile_cells, bt);
    __syncthreads();
    const int cpp = blockDim.x / A.R;
    const int cq = threadIdx.x / A.R, r = threadIdx.x - cq * A.R;
    for (int base = 0; base < A.tile_cells; base += cpp) {
        int i, j, k;
        if (cq < cpp && base + cq < A.tile_cells && alloc_cell(D, bt, first, base + cq, i, j, k)) {
            const uint32_t c = (uint32_t)(((uint64_t)i * D.ny + j) * D.nz + k);
            const Draw d = draw_ray<SM>(D, A.nb, A.ng, c, (uint32_t)r, A.k0, A.k1, A.R, cdf ? lds_d : nullptr,
                                        cdf == 2 ? lds_d + A.nb : nullptr);
            const uint32_t bucket = (uint32_t)((d.n * A.ng + d.g) * 8 + d.o);
            atomicAdd(&lh[bucket], 1u);
            const size_t slot = (size_t)c * A.R + r;
            if constexpr (SM != 2) gst(D.rbkt + slot, bucket);   // learned sampling: rbkt already holds it
            if constexpr (SM == 1) gst(D.dprob + slot, d.p);     // the march's weight
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < A.nbucket; b += blockDim.x)
        A.hist[(size_t)b * A.ntiles + tile] = lh[b];
}

// per bucket: exclusive scan of the tile counts in place, total into bucket_total
__global__ void __launch_bounds__(64) k_bucket_scan(uint32_t *hist, int ntiles, uint32_t *bucket_total)
{
    const int b = blockIdx.x;
    uint32_t *h = hist + (size_t)b * ntiles;
    uint32_t carry = 0;
    const int lane = threadIdx.x;
    for (int base = 0; base < ntiles; base += 64) {
        const uint32_t v = base + lane < ntiles ? h[base + lane] : 0u;
        uint32_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (base + lane < ntiles) h[base + lane] = carry + x - v;
        carry += __shfl(x, 63);
    }
    if (lane == 0) bucket_total[b] = carry;
}

// Scanned count of bucket b before tile t (t = ntiles: the bucket's total).
__device__ __forceinline__ uint32_t hist_before(const uint32_t *hist, const uint32_t *total, int ntiles, int b, uint32_t t)
{
    return t < (uint32_t)ntiles ? hist[(size_t)b * ntiles + t] : total[b];
}

// Rays of run e = (region, bucket) of the work list, padded to whole wavefronts (one wavefront
// never mixes buckets).
__global__ void k_run_len(const uint32_t *hist, const uint32_t *total, int ntiles, const uint32_t *rtile0,
                          int nbucket, uint64_t nrun, uint32_t *run_len)
{
    const uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (e >= nrun) return;
    const uint32_t g = (uint32_t)(e / nbucket), b = (uint32_t)(e % nbucket);
    const uint32_t n = hist_before(hist, total, ntiles, b, rtile0[g + 1]) - hist_before(hist, total, ntiles, b, rtile0[g]);
    run_len[e] = (n + 63u) & ~63u;
}

// Block-wide exclusive scan of one value per thread (1024 threads); returns the thread's
// exclusive prefix and the block total in *total.
__device__ __forceinline__ uint32_t block_scan_1024(uint32_t v, uint32_t *part, uint32_t *total)
{
    const int tid = threadIdx.x;
    part[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t u = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += u;
        __syncthreads();
    }
    const uint32_t incl = part[tid];
    *total = part[1023];
    __syncthreads();
    return incl - v;
}

// Padded rays of each region (one workgroup per region).
__global__ void __launch_bounds__(1024) k_run_region_sum(const uint32_t *run_len, int nbucket, uint32_t *region_len)
{
    __shared__ uint32_t part[1024];
    const uint32_t *rl = run_len + (size_t)blockIdx.x * nbucket;
    uint32_t sum = 0;
    for (int b = threadIdx.x; b < nbucket; b += 1024) sum += rl[b];
    uint32_t total;
    block_scan_1024(sum, part, &total);
    if (threadIdx.x == 0) region_len[blockIdx.x] = total;
}

// Run starts: regions in turn, inside a region the buckets in the given order (longest
// expected rays first); exclusive scan of the padded lengths (one workgroup per region, after
// the regions before it), total chunks.
__global__ void __launch_bounds__(1024) k_run_layout(const uint32_t *run_len, const uint32_t *region_len,
                                                      const uint32_t *order, int nbucket, int nregion, uint32_t *rstart,
                                                      uint32_t *nchunks)
{
    __shared__ uint32_t part[1024];
    const int g = blockIdx.x, tid = threadIdx.x;
    uint32_t base = 0;   // padded rays of the regions before this one
    for (int q = tid; q < g; q += 1024) base += region_len[q];
    uint32_t before;
    block_scan_1024(base, part, &before);
    base = before;
    const uint32_t *rl = run_len + (size_t)g * nbucket;
    uint32_t *rs = rstart + (size_t)g * nbucket;
    const int per = (nbucket + 1023) / 1024;
    uint32_t s = 0;
    for (int x = tid * per; x < min(nbucket, (tid + 1) * per); ++x) s += rl[order[x]];
    uint32_t total;
    uint32_t run = base + block_scan_1024(s, part, &total);
    for (int x = tid * per; x < min(nbucket, (tid + 1) * per); ++x) {
        const uint32_t b = order[x];
        rs[b] = run;
        run += rl[b];
    }
    if (g == nregion - 1 && tid == 0) {
        rstart[(size_t)nregion * nbucket] = base + total;
        *nchunks = (base + total) / 64u;
    }
}

// chunk -> bucket map and invalid markers on the padding of each run
__global__ void k_chunk_map(const uint32_t *hist, const uint32_t *total, int ntiles, const uint32_t *rtile0,
                            const uint32_t *rstart, int nbucket, uint64_t nrun, uint32_t *chunk_bucket, uint2 *items)
{
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.y + threadIdx.y;
    if (r >= nrun) return;
    const uint32_t g = (uint32_t)(r / nbucket), b = (uint32_t)(r % nbucket);
    const uint32_t n = hist_before(hist, total, ntiles, b, rtile0[g + 1]) - hist_before(hist, total, ntiles, b, rtile0[g]);
    const uint32_t s = rstart[r], e = s + ((n + 63u) & ~63u), used = s + n;
    for (uint32_t q = s / 64 + threadIdx.x; q < e / 64; q += blockDim.x) chunk_bucket[q] = (uint32_t)b;
    for (uint32_t q = used + threadIdx.x; q < e; q += blockDim.x) items[q] = make_uint2(0u, kInvalidItem);
}

// LDS of k_alloc_scatter: nbucket positions, the bucket of each thread, the tile's bricks (if
// decoded there).
inline size_t alloc_scatter_lds(bool bricks, int nbucket, int threads, int tile_cells)
{
    return sizeof(uint32_t) * (nbucket + threads + (bricks ? tile_cells / 64 : 0));
}

// Rank of a ray among the earlier rays of its cell drawn into the same bucket: threads s0 ..
// s0 + r - 1 hold those rays' buckets in sb.  Four at a time when s0 is a multiple of 4.
__device__ __forceinline__ uint32_t same_bucket_before(const uint32_t *sb, int s0, int r, uint32_t bucket,
                                                       bool by4)
{
    uint32_t kord = 0;
    int q = 0;
    if (by4) {
        const uint4 *sb4 = reinterpret_cast<const uint4 *>(sb + s0);
        for (; q + 4 <= r; q += 4) {
            const uint4 v = sb4[q >> 2];
            kord += (v.x == bucket ? 1u : 0u) + (v.y == bucket ? 1u : 0u) + (v.z == bucket ? 1u : 0u) +
                    (v.w == bucket ? 1u : 0u);
        }
    }
    for (; q < r; ++q) kord += sb[s0 + q] == bucket ? 1u : 0u;
    return kord;
}

// The same rank when a cell's R rays are R consecutive lanes of one wavefront (R divides 64):
// the live lanes of the cell below this one whose bucket agrees with this lane's in each of its
// nbits bits (one ballot per bit, no LDS).  Every lane of the wavefront calls it.
__device__ __forceinline__ uint32_t same_bucket_in_wave(uint32_t bucket, bool live, int r, int nbits)
{
    uint64_t m = __ballot(live);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = ((bucket >> b) & 1u) != 0u;
        const uint64_t ones = __ballot(bit);
        m &= bit ? ones : ~ones;
    }
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t below = (1ull << lane) - 1ull;   // the lanes under this one
    const uint64_t cell = ~0ull << (lane - r);      // from the cell's first lane on
    return (uint32_t)__popcll(m & below & cell);
}

template <int SM>
__global__ void __launch_bounds__(kAllocThreads) k_alloc_scatter(AllocArgs A)
{
    extern __shared__ uint32_t lb[];   // [nbucket] next free position, [blockDim] bucket of each thread, bricks
    uint32_t *sb = lb + A.nbucket, *bt = A.lds_bricks ? sb + blockDim.x : nullptr;
    const int tile = blockIdx.x;
    const TileInfo TI = A.tiles[tile];
    const int s = TI.snap;
    const SnapDesc D = A.snaps[s];   // a copy: its fields stay in registers across the item stores
    const uint64_t first = TI.first;
    const uint32_t t0 = A.rtile0[TI.region];   // the region's first tile
    for (int b = threadIdx.x; b < A.nbucket; b += blockDim.x)
        lb[b] = A.rstart[(size_t)TI.region * A.nbucket + b] + A.hist[(size_t)b * A.ntiles + tile] -
                A.hist[(size_t)b * A.ntiles + t0];
    if (bt) tile_bricks(D, first, A.tile_cells, bt);
    __syncthreads();
    const int cpp = blockDim.x / A.R;
    const int cq = threadIdx.x / A.R, r = threadIdx.x - cq * A.R;
    const bool by4 = (A.R & 3) == 0 && (A.nbucket & 3) == 0;   // sb + cq * R is 16-byte aligned
    // A pass covers 1024 / R cells, a ray per thread.  The buckets (drawn by the counting pass)
    // of kScatterAhead passes are read at once, so that one load latency is exposed per group
    // of passes rather than per pass (the barriers order LDS only).  Per pass the thread keeps
    // its cell packed as i | j << 10 | k << 20 and its bucket (0xFFFFFFFF: no ray).
    constexpr int kScatterAhead = 8;
    const bool wave_rank = 64 % A.R == 0;
    const int nbits = 32 - __clz(max(A.nbucket - 1, 1));
    for (int g = 0; g < A.tile_cells; g += kScatterAhead * cpp) {
        uint32_t cell[kScatterAhead], bk[kScatterAhead];
#pragma unroll
        for (int u = 0; u < kScatterAhead; ++u) {
            const int p = g + u * cpp + cq;
            int i = 0, j = 0, k = 0;
            bk[u] = 0xFFFFFFFFu;
            if (cq < cpp && p < A.tile_cells && alloc_cell(D, bt, first, p, i, j, k))
                bk[u] = gld(D.rbkt + (size_t)(((uint32_t)i * D.ny + j) * D.nz + k) * A.R + r);   // cells < 2^30
            cell[u] = (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20);
        }
#pragma unroll
        for (int u = 0; u < kScatterAhead; ++u) {
            if (g + u * cpp >= A.tile_cells) break;   // uniform over the workgroup
            const uint32_t bucket = bk[u];
            // the ray's ordinal among its cell's rays in the same bucket: with the cell and the
            // bucket it keys the ray's direction stream, which the march draws
            uint32_t kord = 0;
            if (wave_rank) kord = same_bucket_in_wave(bucket, bucket != 0xFFFFFFFFu, r, nbits);
            else sb[threadIdx.x] = bucket;
            lds_barrier();   // the barriers guard sb and lb; no thread reads another's items
            if (bucket != 0xFFFFFFFFu) {
                if (!wave_rank) kord = same_bucket_before(sb, threadIdx.x - r, r, bucket, by4);
                const uint32_t pos = atomicAdd(&lb[bucket], 1u);
                A.items[pos] = make_uint2(cell[u], (uint32_t)r | (kord << 8) | ((uint32_t)s << 16));
            }
            lds_barrier();
        }
    }
}

// ------------------------------------------------------ rays sorted by expected length
// Classes of expected ray length (length_sort 1): six per octave of the estimated step
// count, 0 .. kLenClasses - 1.  The estimate follows the straight path from the cell centre for
// L = min(distance to the y wall it heads for, ln(1/tol) / kappa_ref) and counts its face
// crossings: L |d_x| nx / Lx + L |d_z| nz / Lz along the uniform periodic axes, and along y the
// faces between the centre and the end point (bisection in the face table, exact on a stretched
// grid).  kappa_ref is the pair's kappa at a mid temperature and mole fraction of the field.  It
// only orders work; no result depends on it.
constexpr int kLenClasses = 64;

__device__ __forceinline__ uint32_t bucket_len_class(const SnapDesc &D, const double *yf, float kref,
                                                     float log_inv_tol, int j, uint32_t o, uint32_t w0, uint32_t w1)
{
    const float mu = 1.0f - 2.0f * unif_dir<float>(w0);
    const float phi = 6.28318530718f * unif_dir<float>(w1);
    const float s = sqrtf((1.0f - mu) * (1.0f + mu));
    float sn, cs;
    __sincosf(phi, &sn, &cs);
    const float ax = fabsf(s * cs), ay = fmaxf(fabsf(mu), 1e-12f), az = fabsf(s * sn);
    const double yc = 0.5 * (yf[j] + yf[j + 1]);
    const bool down = (o & 2u) != 0u;
    const float lw = (float)(down ? yc - yf[0] : yf[D.ny] - yc) / ay;
    const float L = kref > 0.0f ? fminf(lw, log_inv_tol / kref) : lw;
    const double ye = down ? yc - (double)(L * ay) : yc + (double)(L * ay);
    int lo = 0, hi = D.ny + 1;   // faces at or below ye
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (yf[mid] <= ye) lo = mid + 1;
        else hi = mid;
    }
    const int nyc = abs((lo - 1) - j);
    const float E = 1.0f + L * (ax * (float)((double)D.nx / D.Lx) + az * (float)((double)D.nz / D.Lz)) + (float)nyc;
    const int c = (int)floorf(6.0f * __log2f(fminf(E, 1e9f)));
    return (uint32_t)(c < 0 ? 0 : (c >= kLenClasses ? kLenClasses - 1 : c));
}

// -------------------------------------------------------------------------- march
// Ray slot write: one 8-byte store per ray in the FP32 march (a ray's slot is a scattered
// address, so two 4-byte stores would cost two partial-line writes).
template <class Real> __device__ __forceinline__ void store_slot(const SnapDesc &D, size_t slot, double y, uint32_t sw)
{
    if constexpr (sizeof(Real) == 4) {
        reinterpret_cast<uint2 *>(D.Y)[slot] = make_uint2(__float_as_uint((float)y), sw);
    } else {
        reinterpret_cast<double *>(D.Y)[slot] = y;
        D.st[slot] = sw;
    }
}

template <class Real> struct MarchArgs {
    const SnapDesc *snaps;
    const double *faces;        // all snapshots' face tables, staged into LDS
    int nfaces;
    const uint2 *items;
    const uint32_t *chunk_bucket;
    const uint32_t *nchunks;
    const double *dnu, *wg;     // per-ray weights in per-cell pdf mode
    int nb, ng, R;
    uint32_t k0, k1;
    Real tol;
    int max_steps;
    int cap;                    // steps a ray takes in the lane kernel before it is handed to k_march_long
    const float *kmin;          // per (n, g): lower bound of kappa over the field (segmenting range)
    const float *kref;          // per (n, g): reference kappa of the expected-length classes
    struct ContRec *cont;       // continuation records of capped rays
    uint32_t *cont_count;
    uint32_t cont_cap;
    unsigned long long *long_steps;   // steps taken by k_march_long in this compute
    int span_log2;              // log2 of the run of consecutive chunks an XCD takes in turn
    float log_inv_tol;          // ln(1 / tol), for the expected-length estimate
    int long_form;              // k_march_long: 0 by the count of long rays, 1 workgroups, 2 wavefronts
    const double *Ib;           // I_n at the table nodes [nb][nT]
    const float *k32;           // k^s_{n,g} at the table nodes [ns][nb * ng][nT] (FP32-exact values)
    int nT, ns;
    int tab_off;                // LDS: first double of the table slots, after the face tables
    int slot_dbl;               // LDS: doubles per table slot
};

// Doubles of an LDS table slot: I_n at the nT nodes, then ns x nT FP32 k values (16-byte
// multiple).
inline int table_slot_doubles(int nT, int ns) { return (nT + (ns * nT + 1) / 2 + 1) & ~1; }

// Dynamic LDS of the march kernels: the face tables, then four table slots.
inline size_t march_lds_bytes(int nfaces, int nT, int ns)
{
    return sizeof(double) * ((size_t)((nfaces + 1) & ~1) + 4 * (size_t)table_slot_doubles(nT, ns));
}
// what the march kernels' own arrays take besides (the length-sorting variant's is the largest)
constexpr size_t kMarchStaticLds = 12 * 1024;

// Tables of (band, g) pair `pair` into an LDS slot: I_n at the nodes (FP64), then k^s_{n,g}
// at the nodes (FP32) species after species; filled by `nt` threads from thread t0 on.
template <class Real>
__device__ __forceinline__ void stage_tables(double *slot, const MarchArgs<Real> &A, int pair, int t0, int nt)
{
    const int n = pair / A.ng, npairs = A.nb * A.ng;
    for (int q = t0; q < A.nT; q += nt) slot[q] = gld(A.Ib + (size_t)n * A.nT + q);
    float *ks = reinterpret_cast<float *>(slot + A.nT);
    for (int sp = 0; sp < A.ns; ++sp)
        for (int q = t0; q < A.nT; q += nt) ks[sp * A.nT + q] = gld(A.k32 + ((size_t)sp * npairs + pair) * A.nT + q);
}

template <class Real>
__device__ __forceinline__ Props<Real> slot_props(const double *slot, const MarchArgs<Real> &A, const uint4 *rec,
                                                  int rw_log2)
{
    Props<Real> P;
    P.rec = rec;
    P.ib = slot;
    P.k = reinterpret_cast<const float *>(slot + A.nT);
    P.kstride = A.nT;
    P.ns = A.ns;
    P.tmax = A.nT - 2;
    P.rw_log2 = rw_log2;
    return P;
}

// Table slots of the four wavefronts of a workgroup (s_pair[w]: the pair of wavefront w, -1
// without work): wavefront w uses the slot of the first wavefront with the same pair (buckets
// are contiguous in chunk order, so the four usually share one), and all threads stage the
// distinct ones.  Returns the slot of wavefront wib; the caller synchronises before reading.
template <class Real>
__device__ __forceinline__ int stage_wave_tables(double *tabs, const MarchArgs<Real> &A, const int *s_pair, int wib)
{
    int mine = wib;
    for (int w = 0; w < 4; ++w) {
        const int pw = s_pair[w];
        int first = w;
        for (int v = 0; v < w; ++v)
            if (s_pair[v] == pw) { first = v; break; }
        if (pw >= 0 && first == w) stage_tables(tabs + w * A.slot_dbl, A, pw, (int)threadIdx.x, (int)blockDim.x);
        if (w == wib) mine = first;
    }
    return mine;
}

// Workgroups of a launch are dealt to the XCDs in turn (workgroup b runs on XCD b mod 8) and
// each XCD starts its workgroups in order.  Wavefront `wib` of workgroup b = 8 k + x takes
// position p = 4 k + wib in XCD x's sequence, which walks the runs x, x + 8, x + 16, ... of
// 2^span_log2 consecutive chunks: the waves in flight on one XCD then work on neighbouring
// chunks (one (n, g) pair, nearby cells of one region), whose cell records its L2 keeps.  A run
// of 4 chunks gives the plain order chunk = 4 b + wib.
constexpr int kXcds = 8;

__device__ __forceinline__ uint32_t xcd_chunk(uint32_t block, uint32_t wib, int span_log2)
{
    const uint32_t pos = (block / kXcds) * 4 + wib;
    return ((block % kXcds + kXcds * (pos >> span_log2)) << span_log2) | (pos & ((1u << span_log2) - 1));
}

// Workgroups (of 4 wavefronts) a launch needs so that every chunk below max_chunks has a slot.
inline uint64_t xcd_blocks(uint64_t max_chunks, int span_log2)
{
    const uint64_t span = 1ull << span_log2;
    const uint64_t runs = (max_chunks + span - 1) / span;
    return (uint64_t)kXcds * ((runs + kXcds - 1) / kXcds) * (span / 4);
}

// State of a ray handed from the lane kernel to k_march_long after `steps` steps.
struct ContRec {
    uint32_t q;                 // work item index
    int lev;                    // grid level the ray is on (multigrid march; 0 otherwise)
    int i, j, k, steps;         // cell of the next step (on that level)
    int sgn;                    // direction sign bits (y flips at reflecting walls)
    double tau, acc;
    double t, tx, ty, tz;       // current parameter, next-face parameters
    double oy;                  // origin y, mirrored at every reflection
};

template <class Real, bool INC_XZ>
__device__ __forceinline__ ContRec cont_rec(uint32_t q, int lev, const Ray<Real, INC_XZ> &R)
{
    ContRec rc;
    rc.q = q;
    rc.lev = lev;
    rc.i = R.i; rc.j = R.j; rc.k = R.k; rc.steps = R.steps;
    rc.sgn = R.sgn;
    rc.oy = R.oy;
    rc.tau = R.tau; rc.acc = R.acc;
    rc.t = R.t; rc.tx = R.tx; rc.ty = R.ty; rc.tz = R.tz;
    return rc;
}

__device__ __forceinline__ RayGeo ray_geo(const SnapDesc &D, const double *sf)
{
    RayGeo G;
    G.xf = sf + D.face_off;
    G.yf = G.xf + D.nx + 1;
    G.zf = G.yf + D.ny + 1;
    G.nx = D.nx; G.ny = D.ny; G.nz = D.nz;
    G.bsx = D.nby * D.nbz * 64;
    G.bsy = D.nbz * 64;
    G.Lx = D.Lx;
    G.Lz = D.Lz;
    G.closed = D.closed != 0;
    G.reflect = D.reflect != 0;
    return G;
}

// Walls as seen by the rays of band n.
__device__ __forceinline__ Walls walls_of(const SnapDesc &D, int n, int nb)
{
    Walls W;
    W.I = D.Iw + n;
    W.stride = nb;
    W.eps = D.epsw;
    return W;
}

// Geometry of grid level L (faces staged per level; level 0 is ray_geo's).
__device__ __forceinline__ RayGeo ray_geo_level(const SnapDesc &D, const double *sf, int L)
{
    RayGeo G;
    G.nx = D.nx >> L; G.ny = D.ny >> L; G.nz = D.nz >> L;
    G.xf = sf + D.lev_face[L];
    G.yf = G.xf + G.nx + 1;
    G.zf = G.yf + G.ny + 1;
    const int nby = (G.ny + 3) >> 2, nbz = (G.nz + 3) >> 2;
    G.bsx = nby * nbz * 64;
    G.bsy = nbz * 64;
    G.Lx = D.Lx;
    G.Lz = D.Lz;
    G.closed = D.closed != 0;
    G.reflect = D.reflect != 0;
    return G;
}

// The ray's properties on grid level L: the level's records, the same tables.
template <class Real> __device__ __forceinline__ Props<Real> level_props(const SnapDesc &D, int L, Props<Real> P)
{
    P.rec = L == 0 ? D.rec : D.mg_rec + (D.lev_off[L] << D.rw_log2);
    return P;
}

// Multigrid march (Sec. 4.3): mg_steps steps on each grid, then the ray goes on from its
// current point in the coarser cell that holds its cell, and runs to depletion on the last
// grid.  Source kappa and intensity stay those of the DNS cell (k0, I0 on entry).  On the
// last grid the ray stops after last_cap steps in all (returns false; R then holds its state
// on that grid), else returns true when finished.
template <class Real, bool INC_XZ>
__device__ __forceinline__ bool march_levels(Ray<Real, INC_XZ> &R, const SnapDesc &D, const double *sf,
                                             const Props<Real> &P0, int n, int nb, Real tol, int max_steps, Real k0,
                                             double I0, int last_cap)
{
    RayGeo G = ray_geo(D, sf);
    Props<Real> P = P0;
    for (int L = 0;; ++L) {
        const bool last = L + 1 >= D.nlev;
        const int cap = last ? last_cap : D.mg_steps * (L + 1);
        if (ray_march(R, G, P, walls_of(D, n, nb), tol, max_steps, k0, I0, cap)) return true;
        if (last) return false;
        G = ray_geo_level(D, sf, L + 1);
        ray_descend(R, G);
        P = level_props(D, L + 1, P0);
        prop_load(P, R.px + R.py + R.pz, k0, I0);
    }
}

// Wall flux (black walls, one grid): a ray that ended on a black wall adds its wall term
// w kappa_src tau_w (I_src - I_w), times its source cell's volume over R and over the area of
// the wall face element it reached, to that element: the net radiative flux the wall receives
// from the gas [W m^-2].  Face indices outside the grid (a ray through an edge) are clamped.
// FP64 atomics: the sums are reproducible to rounding, not bitwise.
template <class Real, bool INC_XZ>
__device__ __forceinline__ void tally_wall(const SnapDesc &D, const RayGeo &G, const Ray<Real, INC_XZ> &R, int n,
                                           int nb, int nrays, double wk, uint32_t c)
{
    const int w = wall_of_end(R.end);
    if (w < 0) return;
    const int ck = (int)(c % (uint32_t)G.nz), cj = (int)((c / (uint32_t)G.nz) % (uint32_t)G.ny),
              ci = (int)(c / ((uint32_t)G.nz * (uint32_t)G.ny));   // the source cell (natural index)
    const double Iw = gld(D.Iw + (size_t)w * nb + n);
    const double yw = wk * ((R.tau * 1.0) * (R.Isrc - Iw));
    const int i = min(max(R.i, 0), G.nx - 1), j = min(max(R.j, 0), G.ny - 1), k = min(max(R.k, 0), G.nz - 1);
    const double dx = G.xf[i + 1] - G.xf[i], dy = G.yf[j + 1] - G.yf[j], dz = G.zf[k + 1] - G.zf[k];
    const double vc = (G.xf[ci + 1] - G.xf[ci]) * (G.yf[cj + 1] - G.yf[cj]) * (G.zf[ck + 1] - G.zf[ck]);
    const size_t fx = (size_t)G.ny * G.nz, fy = (size_t)G.nx * G.nz, fz = (size_t)G.nx * G.ny;
    size_t off;
    double area;
    if (w < 2) { off = w * fx + (size_t)j * G.nz + k; area = dy * dz; }
    else if (w < 4) { off = 2 * fx + (w - 2) * fy + (size_t)i * G.nz + k; area = dx * dz; }
    else { off = 2 * fx + 2 * fy + (w - 4) * fz + (size_t)i * G.ny + j; area = dx * dy; }
    atomicAdd(D.wallq + off, vc * yw / ((double)nrays * area));
}

// Direction of the ray of work item it (cell (i, j, k) of snapshot D, ordinal k_ord) in bucket
// (pair, octant o): its Philox stream, keyed by (cell, band, g, octant, ordinal), inverted as in
// Eq. 9 inside the octant.
__device__ __forceinline__ void item_dir_words(uint2 it, const SnapDesc &D, int pair, int ng, int o, uint32_t k0,
                                               uint32_t k1, uint32_t &w0, uint32_t &w1)
{
    const uint32_t i = it.x & 1023u, j = (it.x >> 10) & 1023u, k = (it.x >> 20) & 1023u;
    const uint32_t c = (uint32_t)(((uint64_t)i * D.ny + j) * D.nz + k);
    const uint32_t n = (uint32_t)(pair / ng), g = (uint32_t)pair - n * (uint32_t)ng;
    uint32_t v[4];
    philox4x32_10(c, (n << 16) | (g << 8) | (uint32_t)o, (it.y >> 8) & 255u, (D.snap_id << 4) | kTagDir, k0, k1, v);
    w0 = v[0];
    w1 = v[1];
}

__device__ __forceinline__ void item_direction(uint2 it, const SnapDesc &D, int pair, int ng, int o, uint32_t k0,
                                               uint32_t k1, double &dx, double &dy, double &dz)
{
    uint32_t w0, w1;
    item_dir_words(it, D, pair, ng, o, k0, k1, w0, w1);
    octant_direction(w0, w1, o, dx, dy, dz);
}

// One ray per lane, no refill: every wavefront marches 64 work items of one bucket and
// retires when its longest ray ends; the hardware scheduler balances the many short-lived
// wavefronts.  With SORT, the workgroup first reorders the 256 items of its four chunks by
// expected-length class (counting sort in LDS on (bucket segment, class)), so that a
// wavefront's rays end at similar times while its sources stay within four neighbouring
// chunks; items never leave the chunks of their bucket.
// PDF: the ray's probability is per ray (dprob), not per bucket (W).
template <class Real, bool PDF, bool INC_XZ, bool MULTI, bool SORT>
__global__ void __launch_bounds__(256) k_march_lane(MarchArgs<Real> A)
{
    extern __shared__ double sf[];
    for (int q = threadIdx.x; q < A.nfaces; q += blockDim.x) sf[q] = A.faces[q];
    const int wib = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const uint32_t nch = __builtin_amdgcn_readfirstlane(*A.nchunks);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(xcd_chunk(blockIdx.x, (uint32_t)wib, A.span_log2));
    const bool wvalid = wave < nch;
    const uint32_t b = wvalid ? __builtin_amdgcn_readfirstlane(gld(A.chunk_bucket + wave)) : 0xFFFFFFFFu;
    const int o = (int)(b & 7), pair = (int)(b >> 3);
    __shared__ int s_pair[4];
    if (lane == 0) s_pair[wib] = wvalid ? pair : -1;
    __syncthreads();
    const double *tab = sf + A.tab_off + stage_wave_tables(sf + A.tab_off, A, s_pair, wib) * A.slot_dbl;
    __syncthreads();
    uint2 it;
    uint32_t q;                 // position of the item in the work list
    if constexpr (!SORT) {
        if (!wvalid) return;
        q = wave * 64u + (uint32_t)lane;
        it = gld(A.items + q);
        if (it.y == kInvalidItem) return;
    } else {
        // the workgroup's 256 items by (segment, length class): a counting sort in LDS; a
        // segment is a run of its wavefronts with one bucket, so items never leave their bucket
        __shared__ uint2 s_it[256];
        __shared__ uint32_t s_cnt[4 * kLenClasses];
        __shared__ uint32_t s_src[256];
        __shared__ uint32_t s_bk[4];
        for (int q2 = threadIdx.x; q2 < 4 * kLenClasses; q2 += blockDim.x) s_cnt[q2] = 0u;
        const uint2 it0 = wvalid ? gld(A.items + wave * 64u + (uint32_t)lane) : make_uint2(0u, kInvalidItem);
        s_it[threadIdx.x] = it0;
        if (lane == 0) s_bk[wib] = b;
        __syncthreads();
        uint32_t seg = 0;
        for (int w = 1; w <= wib; ++w) seg += s_bk[w] != s_bk[w - 1] ? 1u : 0u;
        uint32_t cls = kLenClasses - 1;   // padding last in its segment
        if (it0.y != kInvalidItem) {
            const SnapDesc &D0 = A.snaps[MULTI ? (int)((it0.y >> 16) & 0x7FFF) : 0];
            uint32_t w0, w1;
            item_dir_words(it0, D0, pair, A.ng, o, A.k0, A.k1, w0, w1);
            const uint32_t c = bucket_len_class(D0, sf + D0.face_off + D0.nx + 1, gld(A.kref + pair), A.log_inv_tol,
                                                (int)((it0.x >> 10) & 1023), (uint32_t)o, w0, w1);
            cls = min(c, (uint32_t)kLenClasses - 2);
        }
        const uint32_t bin = seg * kLenClasses + cls;
        const uint32_t rank = atomicAdd(&s_cnt[bin], 1u);
        __syncthreads();
        if (threadIdx.x < 64) {   // exclusive scan of the 256 bins, four per lane
            const uint32_t c0 = s_cnt[4 * threadIdx.x], c1 = s_cnt[4 * threadIdx.x + 1],
                           c2 = s_cnt[4 * threadIdx.x + 2], c3 = s_cnt[4 * threadIdx.x + 3];
            const uint32_t sum = c0 + c1 + c2 + c3;
            uint32_t x = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off);
                if ((int)threadIdx.x >= off) x += y;
            }
            const uint32_t base = x - sum;
            s_cnt[4 * threadIdx.x] = base;
            s_cnt[4 * threadIdx.x + 1] = base + c0;
            s_cnt[4 * threadIdx.x + 2] = base + c0 + c1;
            s_cnt[4 * threadIdx.x + 3] = base + c0 + c1 + c2;
        }
        __syncthreads();
        s_src[s_cnt[bin] + rank] = threadIdx.x;
        __syncthreads();
        const uint32_t src = s_src[threadIdx.x];
        if (!wvalid) return;
        it = s_it[src];
        if (it.y == kInvalidItem) return;
        q = xcd_chunk(blockIdx.x, src >> 6, A.span_log2) * 64u + (src & 63u);
    }
    const int s = MULTI ? (int)((it.y >> 16) & 0x7FFF) : 0;
    const SnapDesc &D = A.snaps[s];
    double dx, dy, dz;
    item_direction(it, D, pair, A.ng, o, A.k0, A.k1, dx, dy, dz);
    const RayGeo G = ray_geo(D, sf);
    XzUniform U;
    U.hx = D.hx;
    U.hz = D.hz;
    const int i = (int)(it.x & 1023), j = (int)((it.x >> 10) & 1023), k = (int)((it.x >> 20) & 1023);
    const int r = (int)(it.y & 255);
    const int n = pair / A.ng;
    const Props<Real> P = slot_props(tab, A, D.rec, D.rw_log2);
    const uint32_t c = (uint32_t)(((uint64_t)i * D.ny + j) * D.nz + k);
    Ray<Real, INC_XZ> R;
    Real kap_src;
    double Isrc;
    ray_init(R, G, U, P, i, j, k, dx, dy, dz, kap_src, Isrc);
    if (!ray_march(R, G, P, walls_of(D, n, A.nb), A.tol, A.max_steps, kap_src, Isrc, A.cap)) {
        // long ray: hand its state to k_march_long (or, if the list is full, finish it here)
        const uint32_t idx = atomicAdd(A.cont_count, 1u);
        if (idx < A.cont_cap) {
            A.cont[idx] = cont_rec(q, 0, R);
            return;
        }
        Real kc;
        double Ic;
        prop_load(P, R.px + R.py + R.pz, kc, Ic);
        ray_march(R, G, P, walls_of(D, n, A.nb), A.tol, A.max_steps, kc, Ic, A.max_steps);
    }
    const size_t slot = (size_t)c * A.R + r;
    double w;
    if constexpr (!PDF) {
        w = gld(D.W + b);
    } else {
        const double p = gld(D.dprob + slot);
        w = 4.0 * M_PI * A.dnu[n] * A.wg[pair - n * A.ng] / (8.0 * p);
    }
    store_slot<Real>(D, slot, w * (double)kap_src * (double)R.acc, (uint32_t)R.steps | ((uint32_t)R.end << 28));
    if (D.wallq) tally_wall(D, G, R, n, A.nb, A.R, w * (double)kap_src, c);
}

// Multigrid march: one ray per lane as in k_march_lane (no length sort).  A ray still marching
// after `cap` steps on the last grid is handed to k_march_long, which continues it there.
template <class Real, bool PDF, bool INC_XZ, bool MULTI>
__global__ void __launch_bounds__(256) k_march_mg(MarchArgs<Real> A)
{
    extern __shared__ double sf[];
    for (int q = threadIdx.x; q < A.nfaces; q += blockDim.x) sf[q] = A.faces[q];
    const int wib = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const uint32_t nch = __builtin_amdgcn_readfirstlane(*A.nchunks);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(xcd_chunk(blockIdx.x, (uint32_t)wib, A.span_log2));
    const bool wvalid = wave < nch;
    const uint32_t b = wvalid ? __builtin_amdgcn_readfirstlane(gld(A.chunk_bucket + wave)) : 0xFFFFFFFFu;
    const int o = (int)(b & 7), pair = (int)(b >> 3);
    __shared__ int s_pair[4];
    if (lane == 0) s_pair[wib] = wvalid ? pair : -1;
    __syncthreads();
    const double *tab = sf + A.tab_off + stage_wave_tables(sf + A.tab_off, A, s_pair, wib) * A.slot_dbl;
    __syncthreads();
    if (!wvalid) return;
    const uint32_t q = wave * 64u + (uint32_t)lane;
    const uint2 it = gld(A.items + q);
    if (it.y == kInvalidItem) return;
    const int s = MULTI ? (int)((it.y >> 16) & 0x7FFF) : 0;
    const SnapDesc &D = A.snaps[s];
    double dx, dy, dz;
    item_direction(it, D, pair, A.ng, o, A.k0, A.k1, dx, dy, dz);
    const RayGeo G = ray_geo(D, sf);
    XzUniform U;
    U.hx = D.hx;
    U.hz = D.hz;
    const int i = (int)(it.x & 1023), j = (int)((it.x >> 10) & 1023), k = (int)((it.x >> 20) & 1023);
    const int r = (int)(it.y & 255);
    const int n = pair / A.ng;
    const Props<Real> P = slot_props(tab, A, D.rec, D.rw_log2);
    const uint32_t c = (uint32_t)(((uint64_t)i * D.ny + j) * D.nz + k);
    Ray<Real, INC_XZ> R;
    Real kap_src;
    double Isrc;
    ray_init(R, G, U, P, i, j, k, dx, dy, dz, kap_src, Isrc);
    const int last_cap = (int)min((long)A.cap + (long)D.mg_steps * (D.nlev - 1), (long)A.max_steps);
    if (!march_levels(R, D, sf, P, n, A.nb, A.tol, A.max_steps, kap_src, Isrc, last_cap)) {
        const uint32_t idx = atomicAdd(A.cont_count, 1u);
        if (idx < A.cont_cap) {
            A.cont[idx] = cont_rec(q, D.nlev - 1, R);
            return;
        }
        const RayGeo GL = ray_geo_level(D, sf, D.nlev - 1);
        const Props<Real> PL = level_props(D, D.nlev - 1, P);
        Real kc;
        double Ic;
        prop_load(PL, R.px + R.py + R.pz, kc, Ic);
        ray_march(R, GL, PL, walls_of(D, n, A.nb), A.tol, A.max_steps, kc, Ic, A.max_steps);
    }
    const size_t slot = (size_t)c * A.R + r;
    double w;
    if constexpr (!PDF) {
        w = gld(D.W + b);
    } else {
        const double p = gld(D.dprob + slot);
        w = 4.0 * M_PI * A.dnu[n] * A.wg[pair - n * A.ng] / (8.0 * p);
    }
    store_slot<Real>(D, slot, w * (double)kap_src * (double)R.acc, (uint32_t)R.steps | ((uint32_t)R.end << 28));
}

// Long rays (FP32 march, uniform periodic x and z): one workgroup per ray handed over by the
// lane kernel.  The path is continued in rounds.  A round covers the parameter range up to
// tend (the wall, the distance at which even the smallest kappa of the field would bring tau
// to tol, 1.25 times the distance the optical depth seen so far predicts, and the step cap,
// whichever is first) and splits it at the crossings of the axis (x or z) the ray advances
// fastest along into 256 segments, one per thread.  Each thread marches its segment with tau = 1
// (same geometry and absorption as the sequential march); a prefix product of the segment
// transmissivities gives every segment's incoming tau.  The first segment in which the ray
// stops (tau <= tol, the wall, or the step cap) is re-marched sequentially with its true
// incoming tau and step count, and the ray value is
//   acc = acc_before + sum_{l < l*} tau_in(l) acc_l + acc(l*).
// A stopping segment of more than kSplitCross crossings is not re-marched by its one thread:
// the contributions before it are added and the next round starts from its start state, with
// its incoming tau and step count, and ends where it ended, so that this round splits it again
// and the sequential re-march covers a few crossings only.
// Products and sums over the segments run in a fixed order (within each wavefront, then over
// the four wavefronts), so results do not depend on timing.
// When no segment stops, the contributions are added and the next round starts where the
// last segment ended.  Reflecting y walls keep the crossings of x and z evenly spaced: the
// range is then bounded by the black wall a ray reaches within two wall-to-wall traversals,
// or by the wall losses added to the smallest kappa, and a segment's start state replays the
// reflections before it with the sequential march's own arithmetic (mirrored origin, flipped
// direction), so that every segment starts where the sequential march would be.
constexpr int kLongSeg = 256;   // segments per round: the threads of one workgroup
constexpr int kSplitCross = 4;  // longest stopping segment (in crossings) re-marched sequentially

// State at the end of the last segment of a round, passed on through LDS.
struct LongTail {
    double tau, t, tx, ty, tz, oy;
    int steps, i, j, k, sgn;
};

// Orders a wavefront's LDS accesses before and after (its lanes write, then read, a slot).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool PDF, bool MULTI, bool WG>
__device__ __forceinline__ void long_rays(const MarchArgs<float> &A, double *sf, uint32_t nrec)
{
    constexpr int NSEG = WG ? kLongSeg : 64;
    __shared__ double s_tau[4], s_acc[4];
    __shared__ int s_steps[4], s_first[4], s_span;
    __shared__ double s_tcap;
    __shared__ LongTail s_tail;
    const int lane = (int)(threadIdx.x & 63), wid = (int)(threadIdx.x >> 6);
    const int seg = WG ? (int)threadIdx.x : lane;
    const uint32_t first = WG ? blockIdx.x
                              : __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t stride = WG ? gridDim.x : gridDim.x * (blockDim.x >> 6);
    for (uint32_t rec = first; rec < nrec; rec += stride) {
        const ContRec rc = A.cont[rec];
        const uint2 it = gld(A.items + rc.q);
        const uint32_t b = gld(A.chunk_bucket + (rc.q >> 6));
        const int s = MULTI ? (int)((it.y >> 16) & 0x7FFF) : 0;
        const SnapDesc &D = A.snaps[s];
        const RayGeo G0 = ray_geo(D, sf);
        XzUniform U;
        U.hx = D.hx;
        U.hz = D.hz;
        const int ci = (int)(it.x & 1023), cj = (int)((it.x >> 10) & 1023), ck = (int)((it.x >> 20) & 1023);
        const int r = (int)(it.y & 255);
        const int o = (int)(b & 7), pair = (int)(b >> 3);
        const int n = pair / A.ng;
        // the ray's tables: a slot per workgroup (one ray) or per wavefront (one ray each)
        double *slot = sf + A.tab_off + (WG ? 0 : wid) * A.slot_dbl;
        if constexpr (WG) {
            stage_tables(slot, A, pair, (int)threadIdx.x, (int)blockDim.x);
            __syncthreads();
        } else {
            wave_lds_sync();   // the previous ray's reads of the slot are done
            stage_tables(slot, A, pair, lane, 64);
            wave_lds_sync();
        }
        const Props<float> P0 = slot_props(slot, A, D.rec, D.rw_log2);
        Props<float> P = P0;
        const uint32_t c = (uint32_t)(((uint64_t)ci * D.ny + cj) * D.nz + ck);
        double dx, dy, dz;
        item_direction(it, D, pair, A.ng, o, A.k0, A.k1, dx, dy, dz);
        Ray<float, true> R;
        float kap_src;
        double Isrc;
        ray_init(R, G0, U, P0, ci, cj, ck, dx, dy, dz, kap_src, Isrc);
        // continue on the ray's grid level (multigrid): its geometry, records and increments
        const RayGeo G = rc.lev ? ray_geo_level(D, sf, rc.lev) : G0;
        if (rc.lev) {
            P = level_props(D, rc.lev, P0);
            const double sc = (double)(1 << rc.lev);
            U.hx *= sc;
            U.hz *= sc;
            R.dtx *= sc;
            R.dtz *= sc;
            R.wx = R.stx > 0 ? 0 : G.nx - 1;
            R.wz = R.stz > 0 ? 0 : G.nz - 1;
        }
        const bool ax = fabs(dx) >= fabs(dz);            // the crossing axis
        const double dta = ax ? R.dtx : R.dtz;
        const double tw = (((dy > 0.0) ? G.yf[G.ny] : G.yf[0]) - R.oy) * R.ry;   // the wall
        const float km = gld(A.kmin + pair);
        // reflecting y walls: the ray reaches a black wall within two wall-to-wall traversals,
        // and every traversal leaves at most the factor sqrt((1 - eps0) (1 - eps1)) of tau
        const double ry0 = R.ry;
        const int sgn0 = R.sgn;
        double tblack = INFINITY, kwall = 0.0;
        if (G.reflect) {
            const double e0 = gld(D.epsw + kWallY0), e1 = gld(D.epsw + kWallY1);
            const double H = G.yf[G.ny] - G.yf[0];
            if (e0 == 1.0 || e1 == 1.0) tblack = 2.0 * H * fabs(ry0);
            else if (e0 > 0.0 || e1 > 0.0) kwall = -log((1.0 - e0) * (1.0 - e1)) * fabs(dy) / (2.0 * H);
        }
        // workgroup-uniform state of the ray at the start of a round
        int si = rc.i, sj = rc.j, sk = rc.k, ssteps = rc.steps, ssgn = rc.sgn;
        double st = rc.t, stx = rc.tx, sty = rc.ty, stz = rc.tz, stau = rc.tau, sacc = rc.acc, soy = rc.oy;
        double tcap = INFINITY;   // end of the stopping segment a round splits again
        while (true) {
            double tend = G.reflect ? st + tblack : tw;
            const double od = log(stau / (double)A.tol);  // optical depth left (> 0: the ray goes on)
            if (!G.reflect) {
                if (km > 0.0f) tend = fmin(tend, st + od / (double)km);
            } else if ((double)km + kwall > 0.0) {
                tend = fmin(tend, st + od / ((double)km + kwall));
            }
            const double kobs = st > 0.0 ? -log(stau) / st : 0.0;
            if (kobs > 0.0) tend = fmin(tend, st + 1.25 * od / kobs);
            const double ta0 = ax ? stx : stz;
            tend = fmin(tend, ta0 + (double)(A.max_steps - ssteps) * dta);   // every crossing is a step
            tend = fmin(tend, tcap);
            tcap = INFINITY;
            const long M = ta0 < tend ? (long)floor((tend - ta0) / dta) + 1 : 0;
            const long B0 = (M * seg) / NSEG, B1 = (M * (seg + 1)) / NSEG;
            const bool empty = seg < NSEG - 1 && B1 == B0;
            R.tau = 1.0;
            R.acc = 0.0;
            R.steps = 0;
            R.end = kEndTol;
            if (B0 == 0) {
                R.i = si; R.j = sj; R.k = sk;
                R.t = st; R.tx = stx; R.ty = sty; R.tz = stz;
                R.oy = soy;
                R.sgn = ssgn;
                R.ry = ((ssgn ^ sgn0) & 2) ? -ry0 : ry0;
            } else {
                const long m0 = B0 - 1;                   // the crossing the segment starts on
                const double ts = ta0 + (double)m0 * dta;
                R.t = ts;
                // the y reflections before ts, replayed with the sequential march's arithmetic
                double oyk = soy;
                int sgk = ssgn;
                if (G.reflect)
                    for (int guard = 0; guard < (1 << 24); ++guard) {
                        const int side = (sgk & 2) ? 0 : 1;
                        const double yw = G.yf[side ? G.ny : 0];
                        const double th = (yw - oyk) * (((sgk ^ sgn0) & 2) ? -ry0 : ry0);
                        if (!(th <= ts)) break;
                        oyk = 2.0 * yw - oyk;
                        sgk ^= 2;
                    }
                R.oy = oyk;
                R.sgn = (R.sgn & ~2) | (sgk & 2);
                R.ry = ((sgk ^ sgn0) & 2) ? -ry0 : ry0;
                const double dyk = ((sgk ^ sgn0) & 2) ? -dy : dy;
                if (ax) {
                    int ii = (int)(((long)si + ((R.sgn & 1) ? -(m0 + 1) : (m0 + 1))) % G.nx);
                    R.i = ii < 0 ? ii + G.nx : ii;
                    R.tx = ta0 + (double)(m0 + 1) * dta;
                    const double z = R.oz + ts * dz - G.zf[0];
                    const double u = z / U.hz;
                    long kb = (R.sgn & 4) ? (long)ceil(u) - 1 : (long)floor(u);
                    R.tz = (G.zf[0] + (double)(kb + ((R.sgn & 4) ? 0 : 1)) * U.hz - R.oz) * R.rz;
                    int kk = (int)(kb % G.nz);
                    R.k = kk < 0 ? kk + G.nz : kk;
                } else {
                    int kk = (int)(((long)sk + ((R.sgn & 4) ? -(m0 + 1) : (m0 + 1))) % G.nz);
                    R.k = kk < 0 ? kk + G.nz : kk;
                    R.tz = ta0 + (double)(m0 + 1) * dta;
                    const double x = R.ox + ts * dx - G.xf[0];
                    const double u = x / U.hx;
                    long ib = (R.sgn & 1) ? (long)ceil(u) - 1 : (long)floor(u);
                    R.tx = (G.xf[0] + (double)(ib + ((R.sgn & 1) ? 0 : 1)) * U.hx - R.ox) * R.rx;
                    int ii = (int)(ib % G.nx);
                    R.i = ii < 0 ? ii + G.nx : ii;
                }
                const double y = R.oy + ts * dyk;
                int lo = 0, hi = G.ny - 1;                // cell containing y, entered in direction dyk
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    const bool below = (dyk > 0.0) ? (G.yf[mid] <= y) : (G.yf[mid] < y);
                    if (below) lo = mid; else hi = mid - 1;
                }
                R.j = lo;
                R.ty = (G.yf[lo + ((R.sgn & 2) ? 0 : 1)] - R.oy) * R.ry;
            }
            R.px = brick_x(R.i, G.bsx); R.py = brick_y(R.j, G.bsy); R.pz = brick_z(R.k);
            const int start_i = R.i, start_j = R.j, start_k = R.k, start_sgn = R.sgn;
            const double start_t = R.t, start_tx = R.tx, start_ty = R.ty, start_tz = R.tz;
            const double start_oy = R.oy, start_ry = R.ry;
            // local march of the segment with tau = 1: segments but the last end on their last
            // crossing, the last at tend
            bool wall_end = false;
            if (!empty) {
                long next = B0;
                float kc;
                double Ic;
                prop_load(P, R.px + R.py + R.pz, kc, Ic);
                while (true) {
                    const double te = R.tx < R.ty ? (R.tz < R.tx ? R.tz : R.tx) : (R.tz < R.ty ? R.tz : R.ty);
                    const bool cross = (ax ? R.tx : R.tz) == te;
                    double ds;
                    int wall;
                    const int cell = ray_advance(R, G, ds, wall);
                    const uint4 vn = prop_fetch(P, cell);
                    const float x = kc * (float)ds;
                    float a, e;
                    absorb_f32(x, a, e);
                    R.acc += (double)((float)R.tau * a * (float)(Isrc - Ic));
                    R.tau *= x < 0.25f ? 1.0 - (double)a : (double)e;
                    ++R.steps;
                    if (wall) {   // y walls only on this path (x and z periodic); reflection done
                        for (int w = kWallY0; w <= kWallY1; ++w) {
                            if (!((wall >> w) & 1)) continue;
                            const double ew = gld(D.epsw + w);
                            R.acc += R.tau * ew * (Isrc - gld(D.Iw + (size_t)w * A.nb + n));
                            R.tau *= 1.0 - ew;
                            if (ew == 1.0) {
                                R.end = wall_end_code(w);
                                wall_end = true;
                                break;
                            }
                        }
                        if (wall_end) break;
                    }
                    if (!(R.tau > (double)A.tol)) break;
                    if (seg < NSEG - 1 ? (cross && ++next == B1) : (R.t >= tend)) break;
                    if (R.steps >= A.max_steps) break;
                    prop_eval(P, vn, cell, kc, Ic);
                }
            }
            // incoming tau and steps of every segment: inclusive prefix product and sum within
            // each wavefront, then (a workgroup per ray) the totals of the wavefronts before
            double pin = R.tau;
            int sin_ = R.steps;
            for (int off = 1; off < 64; off <<= 1) {
                const double pv = __shfl_up(pin, off);
                const int sv = __shfl_up(sin_, off);
                if (lane >= off) { pin *= pv; sin_ += sv; }
            }
            double before = 1.0;
            int sbefore = 0;
            if constexpr (WG) {
                if (lane == 63) { s_tau[wid] = pin; s_steps[wid] = sin_; }
                __syncthreads();
                for (int w = 0; w < wid; ++w) { before *= s_tau[w]; sbefore += s_steps[w]; }
            }
            double tau_in = __shfl_up(pin, 1);
            int steps_in = __shfl_up(sin_, 1);
            if (lane == 0) { tau_in = 1.0; steps_in = 0; }
            tau_in = stau * (before * tau_in);
            steps_in += ssteps + sbefore;
            const bool stops = !empty && (wall_end || !(tau_in * R.tau > (double)A.tol) ||
                                          steps_in + R.steps >= A.max_steps);
            const uint64_t sm = __ballot(stops);
            int lstar;
            if constexpr (WG) {
                if (lane == 0) s_first[wid] = sm ? wid * 64 + __ffsll((long long)sm) - 1 : NSEG;
                __syncthreads();
                lstar = min(min(s_first[0], s_first[1]), min(s_first[2], s_first[3]));
            } else {
                lstar = sm ? __ffsll((long long)sm) - 1 : NSEG;
            }
            if (lstar == NSEG) {
                // nothing stopped: add the contributions, continue from the end of the last segment
                double contrib = tau_in * R.acc;
                for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
                if constexpr (WG) {
                    if (lane == 0) s_acc[wid] = contrib;
                    if (seg == NSEG - 1) {
                        s_tail.tau = tau_in * R.tau;
                        s_tail.steps = steps_in + R.steps;
                        s_tail.i = R.i; s_tail.j = R.j; s_tail.k = R.k;
                        s_tail.t = R.t; s_tail.tx = R.tx; s_tail.ty = R.ty; s_tail.tz = R.tz;
                        s_tail.oy = R.oy;
                        s_tail.sgn = R.sgn;
                    }
                    __syncthreads();
                    sacc += ((s_acc[0] + s_acc[1]) + s_acc[2]) + s_acc[3];
                    stau = s_tail.tau;
                    ssteps = s_tail.steps;
                    si = s_tail.i; sj = s_tail.j; sk = s_tail.k;
                    st = s_tail.t; stx = s_tail.tx; sty = s_tail.ty; stz = s_tail.tz;
                    soy = s_tail.oy;
                    ssgn = s_tail.sgn;
                    __syncthreads();   // the LDS values are read before the next round writes them
                } else {
                    sacc += contrib;
                    stau = __shfl(tau_in * R.tau, 63);
                    ssteps = __shfl(steps_in + R.steps, 63);
                    si = __shfl(R.i, 63); sj = __shfl(R.j, 63); sk = __shfl(R.k, 63);
                    st = __shfl(R.t, 63); stx = __shfl(R.tx, 63); sty = __shfl(R.ty, 63); stz = __shfl(R.tz, 63);
                    soy = __shfl(R.oy, 63);
                    ssgn = __shfl(R.sgn, 63);
                }
                continue;
            }
            // the stopping segment's crossings; a long one is split again in the next round
            int span;
            if constexpr (WG) {
                if (seg == lstar) {
                    s_span = (int)(B1 - B0);
                    s_tcap = seg < NSEG - 1 ? ta0 + (double)(B1 - 1) * dta : tend;
                    s_tail.tau = tau_in;
                    s_tail.steps = steps_in;
                    s_tail.i = start_i; s_tail.j = start_j; s_tail.k = start_k;
                    s_tail.t = start_t; s_tail.tx = start_tx; s_tail.ty = start_ty; s_tail.tz = start_tz;
                    s_tail.oy = start_oy;
                    s_tail.sgn = start_sgn;
                }
                __syncthreads();
                span = s_span;
            } else {
                span = __shfl((int)(B1 - B0), lstar);
            }
            if (span > kSplitCross) {
                double part = (seg < lstar) ? tau_in * R.acc : 0.0;
                for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
                if constexpr (WG) {
                    if (lane == 0) s_acc[wid] = part;
                    __syncthreads();
                    sacc += ((s_acc[0] + s_acc[1]) + s_acc[2]) + s_acc[3];
                    stau = s_tail.tau;
                    ssteps = s_tail.steps;
                    si = s_tail.i; sj = s_tail.j; sk = s_tail.k;
                    st = s_tail.t; stx = s_tail.tx; sty = s_tail.ty; stz = s_tail.tz;
                    soy = s_tail.oy;
                    ssgn = s_tail.sgn;
                    tcap = s_tcap;
                    __syncthreads();   // the LDS values are read before the next round writes them
                } else {
                    sacc += part;
                    stau = __shfl(tau_in, lstar);
                    ssteps = __shfl(steps_in, lstar);
                    si = __shfl(start_i, lstar); sj = __shfl(start_j, lstar); sk = __shfl(start_k, lstar);
                    st = __shfl(start_t, lstar); stx = __shfl(start_tx, lstar); sty = __shfl(start_ty, lstar);
                    stz = __shfl(start_tz, lstar);
                    soy = __shfl(start_oy, lstar);
                    ssgn = __shfl(start_sgn, lstar);
                    tcap = __shfl(seg < NSEG - 1 ? ta0 + (double)(B1 - 1) * dta : tend, lstar);
                }
                continue;
            }
            double contrib = (seg < lstar) ? tau_in * R.acc : 0.0;
            if (seg == lstar) {
                // re-march the stopping segment with its true incoming tau and step count
                R.i = start_i; R.j = start_j; R.k = start_k;
                R.t = start_t; R.tx = start_tx; R.ty = start_ty; R.tz = start_tz;
                R.oy = start_oy; R.ry = start_ry; R.sgn = start_sgn;
                R.px = brick_x(R.i, G.bsx); R.py = brick_y(R.j, G.bsy); R.pz = brick_z(R.k);
                R.tau = tau_in;
                R.acc = 0.0;
                R.steps = steps_in;
                R.end = kEndTol;
                float kc;
                double Ic;
                prop_load(P, R.px + R.py + R.pz, kc, Ic);
                ray_march(R, G, P, walls_of(D, n, A.nb), A.tol, A.max_steps, kc, Ic, A.max_steps);
                contrib = R.acc;
            }
            // fixed-order sum of the contributions over the wavefront (and the workgroup)
            for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
            double total = contrib;
            if constexpr (WG) {
                if (lane == 0) s_acc[wid] = contrib;
                __syncthreads();
                total = ((s_acc[0] + s_acc[1]) + s_acc[2]) + s_acc[3];
            }
            if (seg == lstar) {
                const size_t slot = (size_t)c * A.R + r;
                double w;
                if constexpr (!PDF) {
                    w = gld(D.W + b);
                } else {
                    const double p = gld(D.dprob + slot);
                    w = 4.0 * M_PI * A.dnu[n] * A.wg[pair - n * A.ng] / (8.0 * p);
                }
                const double acc = sacc + total;
                store_slot<float>(D, slot, w * (double)kap_src * acc, (uint32_t)R.steps | ((uint32_t)R.end << 28));
                atomicAdd(A.long_steps, (unsigned long long)(R.steps - rc.steps));
                if (D.wallq) tally_wall(D, G, R, n, A.nb, A.R, w * (double)kap_src, c);
            }
            if constexpr (WG) __syncthreads();   // the LDS values are read before the next ray writes them
            break;
        }
    }
}

// Few long rays (black walls: the rare grazing ones) are latency-bound: a workgroup and 256
// segments each.  Many (reflecting walls, large grids at high R) are throughput-bound: a
// wavefront and 64 segments each.  The count is known on the device only; the branch is
// uniform over the launch.
constexpr uint32_t kLongWgMax = 8192;

template <bool PDF, bool MULTI>
__global__ void __launch_bounds__(256) k_march_long(MarchArgs<float> A)
{
    extern __shared__ double sf[];
    for (int q = threadIdx.x; q < A.nfaces; q += blockDim.x) sf[q] = A.faces[q];
    __syncthreads();
    const uint32_t nrec = min(__builtin_amdgcn_readfirstlane(*A.cont_count), A.cont_cap);
    if (A.long_form == 1 || (A.long_form == 0 && nrec <= kLongWgMax)) long_rays<PDF, MULTI, true>(A, sf, nrec);
    else long_rays<PDF, MULTI, false>(A, sf, nrec);
}

#include "learn_kernels.inc"

// ------------------------------------------------------------------------ gather probe
// The memory side of the march alone, for the denominator of its roofline: every lane walks a
// straight ray of `steps` cells and reads per step the record of its cell (the first 16-byte
// word) from the field of the last compute, with the march's launch order (XCD-aware chunks;
// the chunks of one (n, g) pair in a row, each starting in the tile region its position in the
// pair's share points to, lanes at cells of one 256-cell tile) -- without the physics and the
// table lookups.  Unit cells, x and z periodic, y reflected at the walls; directions from a
// hash.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x)
{
    x ^= x >> 16; x *= 0x7FEB352Du; x ^= x >> 15; x *= 0x846CA68Bu; x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) k_gather_probe(SnapDesc D, int npairs, int steps, uint32_t nchunks,
                                                      int span_log2, double *__restrict__ out)
{
    const int wib = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const uint32_t chunk = __builtin_amdgcn_readfirstlane(xcd_chunk(blockIdx.x, (uint32_t)wib, span_log2));
    if (chunk >= nchunks) return;
    const int pair = (int)((uint64_t)chunk * npairs / nchunks);
    const uint64_t c0 = ((uint64_t)pair * nchunks + npairs - 1) / npairs;      // first chunk of the pair
    const uint64_t c1 = ((uint64_t)(pair + 1) * nchunks + npairs - 1) / npairs;
    const uint64_t tiles = (D.ncpad + 255) / 256;
    const uint64_t tile = (chunk - c0) * tiles / (c1 > c0 ? c1 - c0 : 1);
    const uint32_t h0 = probe_hash(chunk * 64u + (uint32_t)lane);
    int i, j, k;
    if (!brick_cell(D, min(tile * 256 + (h0 & 255u), D.ncpad - 1), i, j, k)) {
        i = min(i, D.nx - 1); j = min(j, D.ny - 1); k = min(k, D.nz - 1);
    }
    const uint32_t h1 = probe_hash(h0 ^ 0x9E3779B9u), h2 = probe_hash(h1 + 0x632BE5ABu);
    const float dx = (float)(h0 >> 8) * 0x1p-24f - 0.5f, dy = (float)(h1 >> 8) * 0x1p-24f - 0.5f,
                dz = (float)(h2 >> 8) * 0x1p-24f - 0.5f;
    const float ax = 1.0f / fmaxf(fabsf(dx), 1e-6f), ay = 1.0f / fmaxf(fabsf(dy), 1e-6f),
                az = 1.0f / fmaxf(fabsf(dz), 1e-6f);
    int sx = dx > 0.0f ? 1 : -1, sy = dy > 0.0f ? 1 : -1, sz = dz > 0.0f ? 1 : -1;
    float tx = 0.5f * ax, ty = 0.5f * ay, tz = 0.5f * az;
    const int bsx = D.nby * D.nbz * 64, bsy = D.nbz * 64;
    double acc = 0.0;
    for (int st = 0; st < steps; ++st) {
        const int cell = brick_x(i, bsx) + brick_y(j, bsy) + brick_z(k);
        const uint4 v = gld(D.rec + ((size_t)(uint32_t)cell << D.rw_log2));
        acc += __hiloint2double((int)v.y, (int)v.x) * (double)__uint_as_float(v.z);
        if (tx <= ty && tx <= tz) {
            i += sx;
            i = i == D.nx ? 0 : (i < 0 ? D.nx - 1 : i);
            tx += ax;
        } else if (ty <= tz) {
            j += sy;
            if (j < 0 || j >= D.ny) { j -= sy; sy = -sy; }
            ty += ay;
        } else {
            k += sz;
            k = k == D.nz ? 0 : (k < 0 ? D.nz - 1 : k);
            tz += az;
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) out[chunk] = acc;
}

// --------------------------------------------------------------------------- trace
template <class Real> struct TraceArgs {
    const SnapDesc *snaps;
    const double *faces;
    int nfaces;
    const int64_t *cells;
    int ncell;
    const double *dnu, *wg;
    int nb, ng, R;
    uint32_t k0, k1;
    Real tol;
    int max_steps;
    rmc_ray_record *out;
    const double *Ib;           // I_n at the table nodes [nb][nT]
    const float *k32;           // k^s_{n,g} at the table nodes [ns][nb * ng][nT]
    int nT, ns;
};

// All R rays of listed cells, drawn and marched with the same device functions as the
// production path; one thread per ray (ordinal k recomputed from the earlier draws).
template <class Real, int SM, bool INC_XZ>
__global__ void __launch_bounds__(256) k_trace(TraceArgs<Real> A)
{
    extern __shared__ double sf[];
    for (int q = threadIdx.x; q < A.nfaces; q += blockDim.x) sf[q] = A.faces[q];
    __syncthreads();
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)A.ncell * A.R) return;
    const int q = (int)(idx / A.R), r = (int)(idx - (int64_t)q * A.R);
    const SnapDesc &D = A.snaps[0];
    const int64_t c64 = A.cells[q];
    const uint32_t c = (uint32_t)c64;
    const int i = (int)(c64 / ((int64_t)D.ny * D.nz));
    const int j = (int)((c64 / D.nz) % D.ny);
    const int k = (int)(c64 % D.nz);
    const Draw d = draw_ray<SM>(D, A.nb, A.ng, c, (uint32_t)r, A.k0, A.k1, A.R);
    uint32_t kord = 0;
    for (int r2 = 0; r2 < r; ++r2) {
        const Draw e = draw_ray<SM>(D, A.nb, A.ng, c, (uint32_t)r2, A.k0, A.k1, A.R);
        kord += (e.n == d.n && e.g == d.g && e.o == d.o) ? 1u : 0u;
    }
    const int pair = d.n * A.ng + d.g;
    Props<Real> P;              // every thread its own pair: the tables are read from global memory
    P.rec = D.rec;
    P.ib = A.Ib + (size_t)d.n * A.nT;
    P.k = A.k32 + (size_t)pair * A.nT;
    P.kstride = A.nb * A.ng * A.nT;
    P.ns = A.ns;
    P.tmax = A.nT - 2;
    P.rw_log2 = D.rw_log2;
    uint32_t v[4];
    philox4x32_10(c, ((uint32_t)d.n << 16) | ((uint32_t)d.g << 8) | (uint32_t)d.o, kord,
                  (D.snap_id << 4) | kTagDir, A.k0, A.k1, v);
    double dx, dy, dz;
    octant_direction(v[0], v[1], d.o, dx, dy, dz);
    const RayGeo G = ray_geo(D, sf);
    XzUniform U;
    U.hx = D.hx;
    U.hz = D.hz;
    Ray<Real, INC_XZ> R;
    Real kap_src;
    double Isrc;
    ray_init(R, G, U, P, i, j, k, dx, dy, dz, kap_src, Isrc);
    if (D.nlev > 1) march_levels(R, D, sf, P, d.n, A.nb, A.tol, A.max_steps, kap_src, Isrc, A.max_steps);
    else ray_march(R, G, P, walls_of(D, d.n, A.nb), A.tol, A.max_steps, kap_src, Isrc, A.max_steps);
    const double w = 4.0 * M_PI * A.dnu[d.n] * A.wg[d.g] / (8.0 * d.p);
    rmc_ray_record rec;
    rec.Y = w * (double)kap_src * (double)R.acc;
    rec.p = d.p;
    rec.n = d.n; rec.g = d.g; rec.o = d.o; rec.k = (int32_t)kord;
    rec.steps = R.steps;
    rec.end = R.end;
    A.out[idx] = rec;
}

// -------------------------------------------------------------------------- reduce
// Mean of the R ray values of each cell (Eq. 8) and its standard error; total steps.  The
// slots of a group of cells are loaded coalesced into LDS (padded against bank conflicts).
// FP64 sums: four lanes per cell, lane u summing the slots r = u mod 4 in order, the four
// partial sums combined as (s0 + s1) + (s2 + s3) (a fixed order: reproducible); compensated and
// plain FP32 sums: one lane per cell in slot order.
constexpr int kRedVals = 4096;
constexpr int kRedThreads = 256;                     // threads per workgroup of k_reduce
constexpr int kRedPer = kRedVals / kRedThreads;      // values each thread loads per group
__device__ __forceinline__ int red_pad(int q) { return q + (q >> 5); }

template <class Real>
__global__ void __launch_bounds__(kRedThreads) k_reduce(const void *__restrict__ Yv, const uint32_t *__restrict__ st,
                                                uint64_t nc, int R, int accum, double *__restrict__ divq,
                                                double *__restrict__ se, unsigned long long *part)
{
    __shared__ Real ys[kRedVals + kRedVals / 32];
    __shared__ uint32_t ss[kRedVals + kRedVals / 32];
    const int cpg = kRedVals / R;                 // cells per group
    unsigned long long steps = 0, capped = 0;
    for (uint64_t base = (uint64_t)blockIdx.x * cpg; base < nc; base += (uint64_t)gridDim.x * cpg) {
        const int ncell = (int)min((uint64_t)cpg, nc - base);
        const int nval = ncell * R;
        // all of the thread's loads are issued before the first LDS store (kRedPer in flight)
        if constexpr (sizeof(Real) == 4) {
            const uint2 *yb = reinterpret_cast<const uint2 *>(Yv) + base * R;
            uint2 v[kRedPer];
#pragma unroll
            for (int m = 0; m < kRedPer; ++m) {
                const int q = (int)threadIdx.x + m * kRedThreads;
                if (q < nval) v[m] = yb[q];
            }
#pragma unroll
            for (int m = 0; m < kRedPer; ++m) {
                const int q = (int)threadIdx.x + m * kRedThreads;
                if (q < nval) {
                    ys[red_pad(q)] = __uint_as_float(v[m].x);
                    ss[red_pad(q)] = v[m].y;
                }
            }
        } else {
            const double *yb = reinterpret_cast<const double *>(Yv) + base * R;
            const uint32_t *sb = st + base * R;
            double v[kRedPer];
            uint32_t w[kRedPer];
#pragma unroll
            for (int m = 0; m < kRedPer; ++m) {
                const int q = (int)threadIdx.x + m * kRedThreads;
                if (q < nval) {
                    v[m] = yb[q];
                    w[m] = sb[q];
                }
            }
#pragma unroll
            for (int m = 0; m < kRedPer; ++m) {
                const int q = (int)threadIdx.x + m * kRedThreads;
                if (q < nval) {
                    ys[red_pad(q)] = v[m];
                    ss[red_pad(q)] = w[m];
                }
            }
        }
        __syncthreads();
        if (accum == RMC_ACC_F64) {
            const int u = (int)(threadIdx.x & 3);
            // every lane of a group of four runs the same number of passes (the shuffles below)
            for (int cq0 = 0; cq0 < ncell; cq0 += (int)(blockDim.x >> 2)) {
                const int cq = cq0 + (int)(threadIdx.x >> 2);
                const bool live = cq < ncell;
                const int o = cq * R;
                double sum = 0.0;
                if (live)
                    for (int r = u; r < R; r += 4) sum += (double)ys[red_pad(o + r)];
                sum += __shfl_xor(sum, 1);
                sum += __shfl_xor(sum, 2);
                const double mean = sum / R;
                double sq = 0.0;
                if (live)
                    for (int r = u; r < R; r += 4) {
                        const double dv = (double)ys[red_pad(o + r)] - mean;
                        sq += dv * dv;
                        const uint32_t w = ss[red_pad(o + r)];
                        steps += w & 0x0FFFFFFFu;
                        capped += (w >> 28) == (uint32_t)kEndCap ? 1ull : 0ull;
                    }
                sq += __shfl_xor(sq, 1);
                sq += __shfl_xor(sq, 2);
                if (live && u == 0) {
                    divq[base + cq] = mean;
                    if (se) se[base + cq] = R > 1 ? sqrt(sq / (R - 1) / R) : 0.0;
                }
            }
        } else
        for (int cq = threadIdx.x; cq < ncell; cq += blockDim.x) {
            const int o = cq * R;
            double mean;
            if (accum == RMC_ACC_COMP_F32) {
                float sum = 0.0f, comp = 0.0f;   // Neumaier's compensated summation
                for (int r = 0; r < R; ++r) {
                    const float v = (float)ys[red_pad(o + r)];
                    const float t = sum + v;
                    if (fabsf(sum) >= fabsf(v)) comp += (sum - t) + v;
                    else comp += (v - t) + sum;
                    sum = t;
                }
                mean = (double)(sum + comp) / R;
            } else {
                float sum = 0.0f;
                for (int r = 0; r < R; ++r) sum += (float)ys[red_pad(o + r)];
                mean = (double)sum / R;
            }
            double sq = 0.0;
            for (int r = 0; r < R; ++r) {
                const double dv = (double)ys[red_pad(o + r)] - mean;
                sq += dv * dv;
                const uint32_t w = ss[red_pad(o + r)];
                steps += w & 0x0FFFFFFFu;
                capped += (w >> 28) == (uint32_t)kEndCap ? 1ull : 0ull;
            }
            divq[base + cq] = mean;
            if (se) se[base + cq] = R > 1 ? sqrt(sq / (R - 1) / R) : 0.0;
        }
        __syncthreads();
    }
    // the workgroup's step and capped-ray counts, summed later in block order (one counter
    // updated by every wavefront would serialise them)
    for (int off = 32; off > 0; off >>= 1) {
        steps += __shfl_xor(steps, off);
        capped += __shfl_xor(capped, off);
    }
    __shared__ unsigned long long wsum[2][4];
    if ((threadIdx.x & 63) == 0) {
        wsum[0][threadIdx.x >> 6] = steps;
        wsum[1][threadIdx.x >> 6] = capped;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += wsum[0][w]; b += wsum[1][w]; }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// sums of the reduction's per-workgroup counts into the compute's counters (one workgroup)
__global__ void __launch_bounds__(256) k_reduce_counts(const unsigned long long *__restrict__ part, int nblk,
                                                       unsigned long long *counters)
{
    __shared__ unsigned long long sa[256], sb[256];
    unsigned long long a = 0, b = 0;
    for (int q = threadIdx.x; q < nblk; q += blockDim.x) { a += part[2 * q]; b += part[2 * q + 1]; }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { sa[threadIdx.x] += sa[threadIdx.x + w]; sb[threadIdx.x] += sb[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counters[0] += sa[0];
        counters[1] += sb[0];
        counters[2] += sa[0];
    }
}

}  // namespace

// ============================================================================ host side
namespace {

thread_local std::string g_err;

// Address of `scratch` on each device (each GPU holds its own copy of the array), taken once
// per device by rmc_create with that device current; the error of a failed lookup is kept
// and reported by the allocation-free compute.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

rmc_status fail(rmc_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            (void)hipGetLastError();                                                            \
            return fail(e_ == hipErrorOutOfMemory ? RMC_OUT_OF_MEMORY : RMC_DEVICE_ERROR,       \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                         \
        }                                                                                       \
    } while (0)

struct DBuf;

// Bump allocation from the device's static scratch array during an allocation-free compute
// (rmc_compute_divergence_noalloc): while an arena is active on the calling thread, every
// buffer the compute sizes is carved from the array instead of allocated, and the buffer's
// own allocation and size are put back when the arena is closed.
struct Arena {
    static constexpr int kMaxBufs = 96;
    unsigned char *base = nullptr;
    size_t cap = 0, used = 0;
    int nsaved = 0;
    struct Saved {
        DBuf *b;
        void *p;
        size_t bytes;
    } saved[kMaxBufs];
    rmc_status carve(DBuf &b, size_t want);
    void restore();
};
thread_local Arena *t_arena = nullptr;

struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    rmc_status ensure(size_t want)
    {
        if (t_arena) return t_arena->carve(*this, want);
        if (want <= bytes && p) return RMC_OK;
        if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
        if (want == 0) want = 16;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return fail(RMC_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed: %s", want, hipGetErrorString(e));
        }
        bytes = want;
        return RMC_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }   // with the owning context's device current (rmc_destroy)
};

rmc_status Arena::carve(DBuf &b, size_t want)
{
    int q = 0;
    while (q < nsaved && saved[q].b != &b) ++q;
    if (q == nsaved) {   // first use in this call: keep the buffer's own allocation aside
        if (nsaved == kMaxBufs) return fail(RMC_UNSUPPORTED, "too many scratch buffers in one compute");
        saved[nsaved++] = Saved{&b, b.p, b.bytes};
        b.p = nullptr;
        b.bytes = 0;
    }
    if (want <= b.bytes && b.p) return RMC_OK;
    if (want == 0) want = 16;
    const size_t off = (used + 255) & ~(size_t)255;
    if (off > cap || want > cap - off)
        return fail(RMC_UNSUPPORTED, "the allocation-free compute needs more than its %zu MiB of scratch "
                                     "(ncells * R too large)", cap >> 20);
    b.p = base + off;
    b.bytes = want;
    used = off + want;
    return RMC_OK;
}

void Arena::restore()
{
    for (int q = nsaved - 1; q >= 0; --q) {
        saved[q].b->p = saved[q].p;
        saved[q].b->bytes = saved[q].bytes;
    }
    nsaved = 0;
}

// Pinned host memory (hipHostMalloc): readbacks of the ingest kernels and the per-compute
// descriptor uploads, so that those copies are plain DMA transfers.
struct PinBuf {
    void *p = nullptr;
    size_t bytes = 0;
    rmc_status ensure(size_t want)
    {
        if (want <= bytes && p) return RMC_OK;
        if (p) { (void)hipHostFree(p); p = nullptr; bytes = 0; }
        hipError_t e = hipHostMalloc(&p, want < 256 ? 256 : want, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return fail(RMC_OUT_OF_MEMORY, "hipHostMalloc of %zu bytes failed: %s", want, hipGetErrorString(e));
        }
        bytes = want < 256 ? 256 : want;
        return RMC_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
    PinBuf() = default;
    PinBuf(const PinBuf &) = delete;
    PinBuf &operator=(const PinBuf &) = delete;
    ~PinBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

struct rmc_ctx {
    int device = 0;
    // grid
    bool have_grid = false;
    int nx = 0, ny = 0, nz = 0;
    std::vector<double> xf, yf, zf;
    // walls: y always; x and z in a closed box
    bool have_walls = false;
    double Tw[2] = {0, 0}, epsw[2] = {1, 1};
    bool closed = false;
    double Tbox[4] = {0, 0, 0, 0}, epsbox[4] = {1, 1, 1, 1};   // x0, x1, z0, z1
    // tables
    bool have_kdist = false;
    int nb = 0, ng = 0, ns = 0, nT = 0;
    double T0 = 0, dT = 1;
    DBuf k64, k32, Ib, dnu, wg;   // k32: the same k values in FP32 (exact), read by the march
    std::vector<double> k64_host;   // for the march order heuristic (kappa at T_max per (n, g))
    // fields
    bool have_T = false, have_X = false;
    DBuf T, X, stage, stage2;
    double Tmax_cells = 0;
    double xhat[8] = {0};
    int graphs = 0;         // live graphs capturing this context
    // options
    rmc_options opt{};
    // per-cell pdf mode
    bool have_q = false;
    DBuf q, cpdf, ccdf_b, ccdf_g, ccdf_o;
    // learned allocation: network, features, per-ray draws, training state and scratch
    bool have_alloc = false;
    int adam_t = 0;
    DBuf prm, musd, nu_c, gxs, kp, feat, fmask, bng, lfaces, dstrat, dprob, adam1, adam2, lpp;
    DBuf tr_feat, tr_mask, tr_act, tr_del, tr_dz, tr_Lc, tr_scal, tr_err, tr_part, tr_grad, tr_loss;
    // pdf and fields of the last compute
    DBuf pdf_scratch, p, cdf_b, cdf_g, W, Iw, status;
    DBuf rec;               // cell records of the march (table coordinate, mole fractions), bricked
    int rec_rw_log2 = 0;    // 16-byte words per record, log2
    DBuf mgT, mgX, mgrec;   // multigrid: coarse-level fields and records
    // slots
    DBuf Y, st;
    DBuf rbkt;              // bucket of each ray (counting pass -> scatter pass)
    double *wall_dev = nullptr;   // wall flux tally of the compute in progress (rmc_compute_wall_flux)
    DBuf wallbuf;           // its device buffer for host outputs
    PinBuf hread, hup;      // pinned readback of the ingest kernels; pinned descriptor uploads
    hipEvent_t up_evt = nullptr;   // the last descriptor upload from hup (hup is reused after it)
    bool up_pending = false;
    int slots_R = 0, slots_real = 0;
    // shared pipeline workspace (used when this context leads a batch)
    DBuf hist, bucket_total, rstart, run_len, region_len, rtile0, nchunks, chunk_bucket, items, faces, snaps, tile_info, counters, red_part,
        outbuf, tune_out;
    DBuf trace_rec, trace_cells, border, kmin, cont, cont_count, probe;
    std::vector<float> h_kmin;         // per (n, g) pair: kappa lower bound, then reference kappa
    double Tmin_cells = 0;
    double xmin[8] = {0};
    // host staging of the per-compute descriptors (kept alive until the next compute)
    std::vector<double> h_faces;
    std::vector<unsigned char> h_snaps;
    std::vector<TileInfo> h_tiles;
    std::vector<uint32_t> h_rtile0;
    std::vector<uint32_t> h_order;
    DBuf small;             // ingest results
    DBuf scal;              // [0]: max cell temperature, [1..8]: largest mole fraction per species
    uint64_t config_version = 0;   // bumped by every set_* that changes sizes or kernel arguments
    uint64_t input_version = 0;    // bumped by every set_* that changes the learned allocation's inputs
    // learned allocation cache (alloc_cache): per cell and pair the softmax's pair sums, per cell
    // the normaliser's inverse and the reference of the exponentials; valid for input_version
    DBuf acache, acinv, acmax;
    uint64_t acache_version = ~0ull;
    size_t lds_max = 64 * 1024;     // LDS a workgroup may use on the device
    // timing: a ring of event sets, one per compute in flight; counters[0..1] are the last
    // compute's steps / capped rays, counters[2] the steps accumulated since the last reset
    struct EvSet {
        hipEvent_t e[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        bool pending = false;
        int64_t rays = 0;
    };
    std::vector<EvSet> ring;
    size_t ring_head = 0;
    int last_set = -1;
    bool have_counters = false;
    float last_ms[5] = {0, 0, 0, 0, 0};     // prep, alloc, lane march, long-ray march, reduce
    int64_t last_rays = 0;
    int64_t n_computes = 0, sum_rays = 0;
    double sum_ms[5] = {0, 0, 0, 0, 0};
};

namespace {

uint64_t ncells_of(const rmc_ctx *c) { return (uint64_t)c->nx * c->ny * c->nz; }

// LDS left to the march kernels' face tables and table slots on the context's device.
size_t march_lds_budget(const rmc_ctx *c) { return c->lds_max - kMarchStaticLds; }
uint64_t ncpad_of(const rmc_ctx *c)
{
    return (uint64_t)round_up(c->nx, 4) * round_up(c->ny, 4) * round_up(c->nz, 4);
}

// Default allocation tile: about 1024 tiles over the pass, whole bricks, 256 to 8192 cells.
int auto_tile_cells(uint64_t total_ncpad)
{
    return (int)std::min<uint64_t>(8192, std::max<uint64_t>(256, (total_ncpad / 1024 + 63) / 64 * 64));
}

// Regions of the march order: the tiles of a snapshot grouped by the brick row (bi, bj) of
// their first brick into blocks of gx x gy rows (all of z, which a row spans) holding about
// region_cells cells, compact in x and y; region_cells < 0: the snapshot is one region.  By
// default (0) regions of kDefaultRegionCells cells, for snapshots of at least twice that (a
// smaller record field stays in L2 anyway, and splitting its buckets only shortens the runs).
constexpr int kDefaultRegionCells = 262144;

void tile_regions(uint64_t ncpad, int nby, int nbz, int ntiles, int tile_cells, int region_cells,
                  std::vector<uint32_t> &region)
{
    region.assign(ntiles, 0u);
    if (region_cells < 0 || (region_cells == 0 && ncpad < 2ull * kDefaultRegionCells)) return;
    const uint64_t rows = std::max<uint64_t>(1, (uint64_t)(region_cells > 0 ? region_cells : kDefaultRegionCells) /
                                                    (64ull * nbz));
    const int gy = std::max(1, std::min((int)std::lround(std::sqrt((double)rows)), nby));
    const int gx = (int)std::max<uint64_t>(1, rows / gy);
    const int ry = (nby + gy - 1) / gy;
    for (int t = 0; t < ntiles; ++t) {
        const uint64_t row = (uint64_t)t * (tile_cells / 64) / nbz;   // brick row of the tile's first brick
        const int bj = (int)(row % nby), bi = (int)(row / nby);
        region[t] = (uint32_t)((bi / gx) * ry + bj / gy);
    }
}

// Temperature and emissivity of wall w (x0, x1, y0, y1, z0, z1); in a periodic box the x and z
// entries repeat the y0 wall (never hit, but kept inside the table range).
double wall_T(const rmc_ctx *c, int w)
{
    if (w == 2 || w == 3) return c->Tw[w - 2];
    if (!c->closed) return c->Tw[0];
    return c->Tbox[w < 2 ? w : w - 2];
}

double walls_Tmax(const rmc_ctx *c)
{
    double m = 0.0;
    for (int w = 0; w < 6; ++w) m = std::max(m, wall_T(c, w));
    return m;
}

double wall_eps(const rmc_ctx *c, int w)
{
    if (w == 2 || w == 3) return c->epsw[w - 2];
    if (!c->closed) return 1.0;
    return c->epsbox[w < 2 ? w : w - 2];
}

rmc_status check_ctx(const rmc_ctx *c)
{
    if (!c) return fail(RMC_INVALID_ARG, "null context");
    return RMC_OK;
}

rmc_status check_options(const rmc_options *o)
{
    if (o->rays_per_cell < 1 || o->rays_per_cell > 255)
        return fail(RMC_INVALID_ARG, "rays_per_cell must be in [1, 255] (got %d)", o->rays_per_cell);
    if (o->snapshot >= (1u << 27)) return fail(RMC_INVALID_ARG, "snapshot must be < 2^27");
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(RMC_INVALID_ARG, "tol must be finite and >= 0");
    if (o->max_steps < 1 || o->max_steps >= (1 << 28))
        return fail(RMC_INVALID_ARG, "max_steps must be in [1, 2^28)");
    if (o->march != RMC_F32 && o->march != RMC_F64) return fail(RMC_INVALID_ARG, "march must be RMC_F32 or RMC_F64");
    if (o->accum != RMC_ACC_F64 && o->accum != RMC_ACC_COMP_F32 && o->accum != RMC_ACC_F32)
        return fail(RMC_INVALID_ARG, "bad accum");
    if (o->sampling != RMC_SAMPLING_PLAIN && o->sampling != RMC_SAMPLING_PDF && o->sampling != RMC_SAMPLING_LEARNED)
        return fail(RMC_INVALID_ARG, "bad sampling");
    if (o->sampling != RMC_SAMPLING_PLAIN && !(o->mix_eps >= 0.0 && o->mix_eps <= 1.0))
        return fail(RMC_INVALID_ARG, "mix_eps must be in [0, 1]");
    if (o->block_threads != 0 && o->block_threads != 256)
        return fail(RMC_UNSUPPORTED, "block_threads: only 0 (default) and 256 are built");
    if (o->long_ray_steps < 0) return fail(RMC_INVALID_ARG, "long_ray_steps must be >= 0");
    if (o->xcd_span != 0 && (o->xcd_span < 4 || o->xcd_span > (1 << 20) || (o->xcd_span & (o->xcd_span - 1))))
        return fail(RMC_INVALID_ARG, "xcd_span must be 0 or a power of two in [4, 2^20]");
    if (o->length_sort != 0 && o->length_sort != 1) return fail(RMC_INVALID_ARG, "length_sort must be 0 or 1");
    if (o->bucket_order != 0 && o->bucket_order != 1) return fail(RMC_INVALID_ARG, "bucket_order must be 0 or 1");
    if (o->mg_levels < -1 || o->mg_levels > kMaxLev)
        return fail(RMC_INVALID_ARG, "mg_levels must be -1 (all the grid allows), 0, 1 or up to %d", kMaxLev);
    if (o->mg_steps < 0 || o->mg_steps > (1 << 24)) return fail(RMC_INVALID_ARG, "mg_steps must be in [0, 2^24]");
    if (o->alloc_tile != 0 && (o->alloc_tile < 256 || o->alloc_tile > 65536 || o->alloc_tile % 64))
        return fail(RMC_INVALID_ARG, "alloc_tile must be 0 or a multiple of 64 in [256, 65536]");
    if (o->long_ray_form < 0 || o->long_ray_form > 2) return fail(RMC_INVALID_ARG, "long_ray_form must be 0, 1 or 2");
    if (o->alloc_cache != 0 && o->alloc_cache != 1) return fail(RMC_INVALID_ARG, "alloc_cache must be 0 or 1");
    if (o->region_cells < -1 || (o->region_cells > 0 && o->region_cells < 64))
        return fail(RMC_INVALID_ARG, "region_cells must be -1, 0 or at least 64");
    return RMC_OK;
}

rmc_status check_ready(const rmc_ctx *c)
{
    if (!c->have_grid) return fail(RMC_BAD_STATE, "rmc_set_grid missing");
    if (!c->have_walls) return fail(RMC_BAD_STATE, "rmc_set_walls missing");
    if (!c->have_kdist) return fail(RMC_BAD_STATE, "rmc_set_kdist missing");
    if (!c->have_T) return fail(RMC_BAD_STATE, "rmc_set_temperature missing");
    if (!c->have_X) return fail(RMC_BAD_STATE, "rmc_set_species missing");
    if (c->opt.sampling == RMC_SAMPLING_PDF && !c->have_q) return fail(RMC_BAD_STATE, "rmc_set_cell_pdf missing");
    if (c->opt.sampling == RMC_SAMPLING_LEARNED && !c->have_alloc)
        return fail(RMC_BAD_STATE, "rmc_set_allocator missing");
    for (int w = 0; w < 6; ++w) {
        const double u = (wall_T(c, w) - c->T0) / c->dT;
        if (!(u >= 0.0 && u <= (double)(c->nT - 1)))
            return fail(RMC_OUT_OF_RANGE, "wall temperature %g outside the table range", wall_T(c, w));
    }
    if (c->closed && c->opt.sampling == RMC_SAMPLING_LEARNED)
        return fail(RMC_UNSUPPORTED, "the learned allocation's features assume periodic x and z (no closed box)");
    if ((uint64_t)ncells_of(c) * c->opt.rays_per_cell >= (1ull << 32))
        return fail(RMC_UNSUPPORTED, "ncells * R must stay below 2^32");
    return RMC_OK;
}

// Grid levels an nx x ny x nz grid allows: halve every axis while each is even and its half
// at least 3 (the paper's coarsening ratio 2 down to 3^3 meshes).
int level_count(int nx, int ny, int nz)
{
    int L = 1;
    while (L < kMaxLev && nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx / 2 >= 3 && ny / 2 >= 3 && nz / 2 >= 3) {
        nx /= 2; ny /= 2; nz /= 2;
        ++L;
    }
    return L;
}

uint64_t ncpad_level(const rmc_ctx *c, int L)
{
    return (uint64_t)round_up(c->nx >> L, 4) * round_up(c->ny >> L, 4) * round_up(c->nz >> L, 4);
}

// Face tables of every grid level of a snapshot (level L: every 2^L-th face), appended to
// `faces` unless the same tables are already there (snapshots of one grid share them);
// records their offsets in D.  `blocks` lists the (start, length) of the tables appended so far.
void append_faces(const rmc_ctx *c, SnapDesc &D, std::vector<double> &faces,
                  std::vector<std::pair<int, int>> &blocks)
{
    const int start = (int)faces.size();
    int lev[kMaxLev];
    for (int L = 0; L < D.nlev; ++L) {
        lev[L] = (int)faces.size() - start;
        for (int q = 0; q <= (c->nx >> L); ++q) faces.push_back(c->xf[(size_t)q << L]);
        for (int q = 0; q <= (c->ny >> L); ++q) faces.push_back(c->yf[(size_t)q << L]);
        for (int q = 0; q <= (c->nz >> L); ++q) faces.push_back(c->zf[(size_t)q << L]);
    }
    const int len = (int)faces.size() - start;
    int at = start;
    for (const auto &b : blocks)   // same levels of the same grid: the same table layout
        if (b.second == len && memcmp(faces.data() + b.first, faces.data() + start, sizeof(double) * len) == 0) {
            at = b.first;
            faces.resize(start);
            break;
        }
    if (at == start) blocks.emplace_back(start, len);
    D.face_off = at;
    for (int L = 0; L < D.nlev; ++L) D.lev_face[L] = at + lev[L];
}

// width of a uniformly spaced axis (faces equal to f0 + q h within 1e-12 of the length), else 0
double uniform_width(const std::vector<double> &f)
{
    const int n = (int)f.size() - 1;
    const double L = f[n] - f[0], h = L / n;
    for (int q = 0; q <= n; ++q)
        if (std::fabs(f[q] - (f[0] + q * h)) > 1e-12 * L) return 0.0;
    return h;
}

// Bucket order of the march: (band, g) pairs by increasing kappa at T_max (longest rays
// first, so the longest-running wavefronts start early), octants consecutive.
void march_order(const rmc_ctx *c, std::vector<uint32_t> &order)
{
    const int nb = c->nb, ng = c->ng;
    const double Tmax = std::max(c->Tmax_cells, walls_Tmax(c));
    const double u = (Tmax - c->T0) / c->dT;
    int t = (int)std::floor(u);
    if (t > c->nT - 2) t = c->nT - 2;
    if (t < 0) t = 0;
    const double f = u - t;
    std::vector<std::pair<double, int>> key(nb * ng);
    for (int pr = 0; pr < nb * ng; ++pr) {
        double kap = 0.0;
        for (int sp = 0; sp < c->ns; ++sp) {
            const double *tab = c->k64_host.data() + ((size_t)sp * nb * ng + pr) * c->nT;
            kap += c->xhat[sp] * (tab[t] + f * (tab[t + 1] - tab[t]));
        }
        key[pr] = {kap, pr};
    }
    std::stable_sort(key.begin(), key.end(), [](const std::pair<double, int> &a, const std::pair<double, int> &b) {
        return a.first < b.first;
    });
    if (c->opt.bucket_order == 1) {
        // band-major: the g-points of a band next to each other (they share the band's
        // intensity table), bands ordered by their smallest kappa
        std::vector<int> rank(nb, nb * ng);
        for (int q = 0; q < nb * ng; ++q) rank[key[q].second / ng] = std::min(rank[key[q].second / ng], q);
        std::stable_sort(key.begin(), key.end(), [&](const std::pair<double, int> &a, const std::pair<double, int> &b) {
            return rank[a.second / ng] < rank[b.second / ng];
        });
    }
    order.resize((size_t)nb * ng * 8);
    for (int q = 0; q < nb * ng; ++q)
        for (int o = 0; o < 8; ++o) order[(size_t)q * 8 + o] = (uint32_t)(key[q].second * 8 + o);
}

// 16-byte words of a cell record (FP64 table coordinate, ns mole fractions of `xbytes`
// bytes), log2, rounded up to a power of two.
int record_words_log2(int ns, size_t xbytes)
{
    const size_t words = (8 + xbytes * (size_t)ns + 15) / 16;
    int l = 0;
    while ((1u << l) < words) ++l;
    return l;
}

// per-snapshot plan: buffers and the snapshot descriptor (no work enqueued)
// Lower bound of kappa_{n,g} over the field: smallest mole fractions times the smallest table
// value over the nodes bracketing the field's temperature range (linear interpolation never
// goes below the smaller of its two nodes).  Bounds how far a ray can march with tau > tol.
void kappa_lower_bounds(const rmc_ctx *c, std::vector<float> &out)
{
    const int nb = c->nb, ng = c->ng;
    int tlo = (int)std::floor((c->Tmin_cells - c->T0) / c->dT);
    int thi = (int)std::floor((std::max(c->Tmax_cells, c->Tmin_cells) - c->T0) / c->dT) + 1;
    tlo = std::max(0, std::min(tlo, c->nT - 1));
    thi = std::max(tlo, std::min(thi, c->nT - 1));
    out.assign((size_t)nb * ng, 0.0f);
    for (int pr = 0; pr < nb * ng; ++pr) {
        double kap = 0.0;
        for (int sp = 0; sp < c->ns; ++sp) {
            const double *tab = c->k64_host.data() + ((size_t)sp * nb * ng + pr) * c->nT;
            double m = tab[tlo];
            for (int t = tlo; t <= thi; ++t) m = std::min(m, tab[t]);
            kap += c->xmin[sp] * m;
        }
        out[pr] = (float)(kap * (1.0 - 1e-6));
    }
}

// Reference kappa per (n, g) pair for the expected-length classes: the mixture at the middle of
// the field's temperature range and of each species' mole-fraction range.
void kappa_reference(const rmc_ctx *c, std::vector<float> &out)
{
    const int nb = c->nb, ng = c->ng;
    const double Tm = 0.5 * (c->Tmin_cells + std::max(c->Tmax_cells, c->Tmin_cells));
    const double u = std::min(std::max((Tm - c->T0) / c->dT, 0.0), (double)(c->nT - 1));
    const int t = std::min((int)u, c->nT - 2);
    const double f = u - t;
    out.assign((size_t)nb * ng, 0.0f);
    for (int pr = 0; pr < nb * ng; ++pr) {
        double kap = 0.0;
        for (int sp = 0; sp < c->ns; ++sp) {
            const double *tab = c->k64_host.data() + ((size_t)sp * nb * ng + pr) * c->nT;
            kap += 0.5 * (c->xmin[sp] + c->xhat[sp]) * (tab[t] + f * (tab[t + 1] - tab[t]));
        }
        out[pr] = (float)kap;
    }
}

// ------------------------------------------------------------ learned allocation (host)
// Workgroups of the allocation kernels: single wavefronts, one cell at a time each, in turn
// over the cells (each holds the network's weights in registers once).
constexpr unsigned kNetBlocks = 4096;

// buffers of the features and of the per-ray draws; the face table for the features kernel
rmc_status plan_features(rmc_ctx *c)
{
    rmc_status st;
    const uint64_t nc = ncells_of(c);
    const size_t nf = (size_t)c->nx + c->ny + c->nz + 3;
    if ((st = c->kp.ensure(sizeof(double) * c->ns * c->nT)) || (st = c->feat.ensure(sizeof(float) * 3 * nc)) ||
        (st = c->fmask.ensure(nc)) || (st = c->lfaces.ensure(sizeof(double) * nf)))
        return st;
    std::vector<double> f;
    f.reserve(nf);
    for (double v : c->xf) f.push_back(v);
    for (double v : c->yf) f.push_back(v);
    for (double v : c->zf) f.push_back(v);
    HIPCHK(hipMemcpy(c->lfaces.p, f.data(), sizeof(double) * nf, hipMemcpyHostToDevice));
    return RMC_OK;
}

rmc_status plan_learned(rmc_ctx *c)
{
    rmc_status st;
    if ((st = plan_features(c))) return st;
    if (net_wave_lds(c->nb * c->ng, c->nb) > 64 * 1024)
        return fail(RMC_UNSUPPORTED, "nb * ng too large for the allocation kernel");
    if ((st = c->bng.ensure(sizeof(float) * c->nb * c->ng * kHid)) || (st = c->lpp.ensure(sizeof(double) * c->nb * c->ng)) ||
        (st = c->dstrat.ensure(sizeof(uint32_t) * ncells_of(c) * c->opt.rays_per_cell)))
        return st;
    if (c->opt.alloc_cache) {
        const uint64_t nc = ncells_of(c);
        const void *before = c->acache.p;
        if ((st = c->acache.ensure(sizeof(float) * nc * c->nb * c->ng)) || (st = c->acinv.ensure(sizeof(double) * nc)) ||
            (st = c->acmax.ensure(sizeof(float) * nc)))
            return st;
        if (c->acache.p != before) c->acache_version = ~0ull;   // a new buffer holds nothing yet
    }
    return RMC_OK;
}

rmc_status enqueue_features(rmc_ctx *c, hipStream_t s)
{
    const uint64_t nc = ncells_of(c);
    hipLaunchKernelGGL(k_kp_tables, dim3((c->ns * c->nT + 255) / 256), dim3(256), 0, s, c->k64.as<double>(),
                       c->Ib.as<double>(), c->dnu.as<double>(), c->wg.as<double>(), c->ns, c->nb, c->ng, c->nT, c->T0,
                       c->dT, c->kp.as<double>());
    HIPCHK(hipGetLastError());
    FeatArgs F;
    F.T = c->T.as<double>();
    F.X = c->X.as<double>();
    F.xf = c->lfaces.as<double>();
    F.yf = F.xf + c->nx + 1;
    F.zf = F.yf + c->ny + 1;
    F.kp = c->kp.as<double>();
    F.nx = c->nx; F.ny = c->ny; F.nz = c->nz; F.ns = c->ns; F.nT = c->nT;
    F.T0 = c->T0; F.dT = c->dT; F.Tw0 = c->Tw[0]; F.Tw1 = c->Tw[1];
    F.feat = c->feat.as<float>();
    F.mask = c->fmask.as<uint8_t>();
    hipLaunchKernelGGL(k_features, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, F);
    HIPCHK(hipGetLastError());
    return RMC_OK;
}

AllocNetArgs net_args(rmc_ctx *c)
{
    AllocNetArgs A{};
    A.prm = c->prm.as<float>();
    A.mu = c->musd.as<float>();
    A.sd = A.mu + 5;
    A.bng = c->bng.as<float>();
    A.feat = c->feat.as<float>();
    A.mask = c->fmask.as<uint8_t>();
    A.P = c->nb * c->ng;
    A.nb = c->nb; A.ng = c->ng; A.R = c->opt.rays_per_cell;
    A.k0 = (uint32_t)c->opt.seed; A.k1 = (uint32_t)(c->opt.seed >> 32);
    A.mix_eps = c->opt.mix_eps;
    A.snap_id = c->opt.snapshot;
    return A;
}

rmc_status enqueue_spec(rmc_ctx *c, hipStream_t s)
{
    const int n = c->nb * c->ng * kHid;
    hipLaunchKernelGGL(k_mlp_spec, dim3((n + 255) / 256), dim3(256), 0, s, c->prm.as<float>(), c->musd.as<float>(),
                       c->musd.as<float>() + 5, c->nu_c.as<double>(), c->gxs.as<double>(), c->nb, c->ng,
                       c->bng.as<float>());
    HIPCHK(hipGetLastError());
    return RMC_OK;
}

// features, spectral half of layer 1, then the fused per-cell network + draws (kernels only)
rmc_status enqueue_learned(rmc_ctx *c, hipStream_t s)
{
    rmc_status st;
    if ((st = enqueue_features(c, s)) || (st = enqueue_spec(c, s))) return st;
    const int P = c->nb * c->ng;
    hipLaunchKernelGGL(k_log_pdf, dim3((P + 255) / 256), dim3(256), 0, s, c->p.as<double>(), P, c->lpp.as<double>());
    HIPCHK(hipGetLastError());
    AllocNetArgs A = net_args(c);
    A.ncell = (int)ncells_of(c);
    A.pplain = c->p.as<double>();
    A.lpp = c->lpp.as<double>();
    A.dstrat = c->dstrat.as<uint32_t>();
    A.dprob = c->dprob.as<double>();
    const dim3 grid((unsigned)std::min<int64_t>(A.ncell, kNetBlocks)), block(64);
    const size_t lds = net_wave_lds(A.P, A.nb);
    if (!c->opt.alloc_cache) {
        hipLaunchKernelGGL(k_alloc_draw<0>, grid, block, lds, s, A);
    } else {
        A.acache = c->acache.as<float>();
        A.acinv = c->acinv.as<double>();
        A.acmax = c->acmax.as<float>();
        if (c->acache_version == c->input_version) {
            hipLaunchKernelGGL(k_alloc_draw<2>, grid, block, lds, s, A);
        } else {
            hipLaunchKernelGGL(k_alloc_draw<1>, grid, block, lds, s, A);
            c->acache_version = c->input_version;   // filled by this launch, ahead of any later one
        }
    }
    HIPCHK(hipGetLastError());
    return RMC_OK;
}

template <class Real> rmc_status plan_snapshot(rmc_ctx *c, SnapDesc &D)
{
    rmc_status st;
    const int nb = c->nb, ng = c->ng, nbucket = nb * ng * 8;
    const uint64_t nc = ncells_of(c);
    const int R = c->opt.rays_per_cell;
    if ((st = c->pdf_scratch.ensure(sizeof(double) * (nb * ng + nb))) || (st = c->p.ensure(sizeof(double) * nb * ng)) ||
        (st = c->cdf_b.ensure(sizeof(double) * nb)) || (st = c->cdf_g.ensure(sizeof(double) * nb * ng)) ||
        (st = c->W.ensure(sizeof(double) * nbucket)) || (st = c->Iw.ensure(sizeof(double) * 6 * nb)) ||
        (st = c->status.ensure(sizeof(int))) ||
        (st = c->rec.ensure(sizeof(uint4) * (ncpad_of(c) << record_words_log2(c->ns, sizeof(Real))))) ||
        (st = c->Y.ensure(sizeof(uint64_t) * nc * R)) ||
        (sizeof(Real) == 8 && (st = c->st.ensure(sizeof(uint32_t) * nc * R))))
        return st;
    D = SnapDesc{};
    D.nx = c->nx; D.ny = c->ny; D.nz = c->nz;
    D.nbx = round_up(c->nx, 4) / 4; D.nby = round_up(c->ny, 4) / 4; D.nbz = round_up(c->nz, 4) / 4;
    D.ncpad = ncpad_of(c);
    D.snap_id = c->opt.snapshot;
    D.Lx = c->xf[c->nx] - c->xf[0];
    D.Lz = c->zf[c->nz] - c->zf[0];
    D.hx = uniform_width(c->xf);
    D.hz = uniform_width(c->zf);
    D.W = c->W.as<double>(); D.Iw = c->Iw.as<double>();
    for (int w = 0; w < 6; ++w) D.epsw[w] = wall_eps(c, w);
    D.closed = c->closed ? 1 : 0;
    D.reflect = 0;
    for (int w = 0; w < 6; ++w) D.reflect |= D.epsw[w] < 1.0 ? 1 : 0;
    D.p = c->p.as<double>(); D.cdf_b = c->cdf_b.as<double>(); D.cdf_g = c->cdf_g.as<double>();
    if (c->opt.sampling == RMC_SAMPLING_PDF) {
        const uint64_t m = (uint64_t)nb * ng * 8;
        if ((st = c->cpdf.ensure(sizeof(double) * nc * m)) || (st = c->ccdf_b.ensure(sizeof(double) * nc * nb)) ||
            (st = c->ccdf_g.ensure(sizeof(double) * nc * nb * ng)) || (st = c->ccdf_o.ensure(sizeof(double) * nc * m)))
            return st;
        D.cpdf = c->cpdf.as<double>(); D.ccdf_b = c->ccdf_b.as<double>();
        D.ccdf_g = c->ccdf_g.as<double>(); D.ccdf_o = c->ccdf_o.as<double>();
    }
    if (c->opt.sampling != RMC_SAMPLING_PLAIN) {
        if ((st = c->dprob.ensure(sizeof(double) * nc * R))) return st;
        D.dprob = c->dprob.as<double>();
    }
    if (c->opt.sampling == RMC_SAMPLING_LEARNED) {
        if ((st = plan_learned(c))) return st;
        D.dstrat = c->dstrat.as<uint32_t>();
        D.rbkt = c->dstrat.as<uint32_t>();   // the drawn strata are the buckets
    } else {
        if ((st = c->rbkt.ensure(sizeof(uint32_t) * nc * R))) return st;
        D.rbkt = c->rbkt.as<uint32_t>();
    }
    D.rw_log2 = record_words_log2(c->ns, sizeof(Real));
    D.rec = c->rec.as<uint4>();
    c->rec_rw_log2 = D.rw_log2;
    D.wallq = c->wall_dev;
    // multigrid levels
    const int allowed = level_count(c->nx, c->ny, c->nz);
    D.nlev = c->opt.mg_levels < 0 ? allowed : std::max(1, c->opt.mg_levels);
    if (D.nlev > allowed)
        return fail(RMC_INVALID_ARG, "mg_levels %d exceeds the %d grid levels a %dx%dx%d grid allows", D.nlev, allowed,
                    c->nx, c->ny, c->nz);
    D.mg_steps = c->opt.mg_steps > 0 ? c->opt.mg_steps : 5;
    if (D.wallq && (D.nlev > 1 || D.reflect))
        return fail(RMC_UNSUPPORTED, "the wall flux needs black walls and the DNS grid only (no multigrid)");
    if (D.nlev > 1) {
        uint64_t off = 0, cells = 0;
        for (int L = 1; L < D.nlev; ++L) {
            D.lev_off[L] = off;
            off += ncpad_level(c, L);
            cells += (uint64_t)(c->nx >> L) * (c->ny >> L) * (c->nz >> L);
        }
        D.mg_stride = off;
        if ((st = c->mgT.ensure(sizeof(double) * cells)) || (st = c->mgX.ensure(sizeof(double) * cells * c->ns)) ||
            (st = c->mgrec.ensure(sizeof(uint4) * (off << D.rw_log2))))
            return st;
        D.mg_rec = c->mgrec.as<uint4>();
    }
    D.Y = c->Y.p;
    D.st = sizeof(Real) == 8 ? c->st.as<uint32_t>() : nullptr;
    c->slots_R = R;
    c->slots_real = (int)sizeof(Real);
    return RMC_OK;
}

// per-snapshot work: spectral pdf, per-cell pdfs, property fields (kernels only)
template <class Real>
rmc_status enqueue_snapshot(rmc_ctx *c, const SnapDesc &D, const double *dfaces, hipStream_t s)
{
    rmc_status st;
    const int nb = c->nb, ng = c->ng;
    const uint64_t nc = ncells_of(c);
    PdfArgs A;
    A.k64 = c->k64.as<double>();
    A.Ib = c->Ib.as<double>();
    A.dnu = c->dnu.as<double>();
    A.wg = c->wg.as<double>();
    A.nb = nb; A.ng = ng; A.ns = c->ns; A.nT = c->nT;
    A.T0 = c->T0; A.dT = c->dT;
    for (int w = 0; w < 6; ++w) A.Tw[w] = wall_T(c, w);
    A.scal = c->scal.as<double>();
    A.e = c->pdf_scratch.as<double>();
    A.eb = A.e + nb * ng;
    A.p = c->p.as<double>(); A.cdf_b = c->cdf_b.as<double>(); A.cdf_g = c->cdf_g.as<double>();
    A.W = c->W.as<double>(); A.Iw = c->Iw.as<double>(); A.status = c->status.as<int>();
    hipLaunchKernelGGL(k_plain_pdf, dim3(1), dim3(256), 0, s, A);
    HIPCHK(hipGetLastError());
    if (c->opt.sampling == RMC_SAMPLING_LEARNED && (st = enqueue_learned(c, s))) return st;
    if (c->opt.sampling == RMC_SAMPLING_PDF) {
        hipLaunchKernelGGL(k_cell_pdf, dim3((unsigned)((nc + 127) / 128)), dim3(128), 0, s, c->q.as<double>(),
                           c->p.as<double>(), nc, nb, ng, c->opt.mix_eps, c->cpdf.as<double>(),
                           c->ccdf_b.as<double>(), c->ccdf_g.as<double>(), c->ccdf_o.as<double>());
        HIPCHK(hipGetLastError());
    }
    const uint64_t ncpad = ncpad_of(c);
    hipLaunchKernelGGL(k_records<Real>, dim3((unsigned)((ncpad + 255) / 256)), dim3(256), 0, s, c->T.as<double>(),
                       c->X.as<double>(), c->ns, nc, c->T0, c->dT, D, c->rec.as<uint4>());
    HIPCHK(hipGetLastError());
    // multigrid: fields of each coarser level from the one below, then its records
    const double *Tin = c->T.as<double>(), *Xin = c->X.as<double>();
    uint64_t toff = 0;
    for (int L = 1; L < D.nlev; ++L) {
        const int px = c->nx >> (L - 1), py = c->ny >> (L - 1), pz = c->nz >> (L - 1);
        const uint64_t ncc = (uint64_t)(px >> 1) * (py >> 1) * (pz >> 1);
        double *Tc = c->mgT.as<double>() + toff, *Xc = c->mgX.as<double>() + toff * c->ns;
        const double *xf = dfaces + D.lev_face[L - 1];
        hipLaunchKernelGGL(k_coarsen, dim3((unsigned)((ncc + 255) / 256)), dim3(256), 0, s, Tin, Xin, c->ns, px, py,
                           pz, xf, xf + px + 1, xf + px + py + 2, Tc, Xc);
        HIPCHK(hipGetLastError());
        SnapDesc Dl = D;
        Dl.nx = px >> 1; Dl.ny = py >> 1; Dl.nz = pz >> 1;
        Dl.nbx = round_up(Dl.nx, 4) / 4; Dl.nby = round_up(Dl.ny, 4) / 4; Dl.nbz = round_up(Dl.nz, 4) / 4;
        Dl.ncpad = ncpad_level(c, L);
        hipLaunchKernelGGL(k_records<Real>, dim3((unsigned)((Dl.ncpad + 255) / 256)), dim3(256), 0, s, Tc, Xc,
                           c->ns, ncc, c->T0, c->dT, Dl, c->mgrec.as<uint4>() + (D.lev_off[L] << D.rw_log2));
        HIPCHK(hipGetLastError());
        Tin = Tc;
        Xin = Xc;
        toff += ncc;
    }
    return RMC_OK;
}

// wait for one event set and fold its phase times into the accumulated statistics
rmc_status harvest(rmc_ctx *L, rmc_ctx::EvSet &set)
{
    HIPCHK(hipEventSynchronize(set.e[5]));
    float t[5];
    for (int q = 0; q < 5; ++q) HIPCHK(hipEventElapsedTime(&t[q], set.e[q], set.e[q + 1]));
    for (int q = 0; q < 5; ++q) L->sum_ms[q] += t[q];
    ++L->n_computes;
    L->sum_rays += set.rays;
    if (&set == &L->ring[L->last_set]) {
        for (int q = 0; q < 5; ++q) L->last_ms[q] = t[q];
        L->last_rays = set.rays;
    }
    set.pending = false;
    return RMC_OK;
}

rmc_status harvest_all(rmc_ctx *L)
{
    if (L->ring.empty()) return RMC_OK;
    const size_t n = L->ring.size();
    for (size_t q = 0; q < n; ++q) {   // oldest first
        rmc_ctx::EvSet &set = L->ring[(L->ring_head + q) % n];
        if (set.pending)
            if (rmc_status st = harvest(L, set)) return st;
    }
    return RMC_OK;
}

// Everything the enqueue phase needs; built on the host by plan_pipeline.
struct Plan {
    std::vector<rmc_ctx *> ctxs;
    std::vector<SnapDesc> D;
    int nfaces = 0, ntiles = 0, tile_cells = 0;
    uint64_t total_cells = 0, max_chunks = 0;
    bool inc_xz = true, pdf_mode = false;   // pdf_mode: per-ray probabilities (modes 1 and 2)
    bool multigrid = false;                 // some snapshot marches on more than one grid
    bool periodic_xz = true;                // every snapshot periodic in x and z (no closed box)
    int smode = 0;
    uint32_t cont_cap = 0;
    // device copies of the host-built tables the kernels read: the leader's buffers, or for a
    // captured graph its own copies (later computes or traces led by the same context rewrite
    // the leader's buffers)
    double *d_faces = nullptr;
    SnapDesc *d_snaps = nullptr;
    TileInfo *d_tiles = nullptr;
    uint32_t *d_rtile0 = nullptr;
    int nregion = 0;
    uint32_t *d_border = nullptr;
    float *d_kmin = nullptr;
};

// Host part of a compute: buffers (allocated or grown), descriptors and their upload on s.
template <class Real> rmc_status plan_pipeline(rmc_ctx *const *ctxs, int nsnap, Plan &P, hipStream_t s)
{
    rmc_ctx *L = ctxs[0];   // leader: owns the shared workspace and the timers
    rmc_status st;
    const rmc_options &O = L->opt;
    const int nb = L->nb, ng = L->ng, nbucket = nb * ng * 8, R = O.rays_per_cell;
    P = Plan{};
    P.ctxs.assign(ctxs, ctxs + nsnap);
    P.smode = (int)O.sampling;
    P.pdf_mode = P.smode != RMC_SAMPLING_PLAIN;
    P.D.resize(nsnap);
    uint64_t total_ncpad = 0;
    std::vector<double> &faces = L->h_faces;
    faces.clear();
    std::vector<std::pair<int, int>> blocks;
    for (int q = 0; q < nsnap; ++q) {
        if ((st = plan_snapshot<Real>(ctxs[q], P.D[q]))) return st;
        append_faces(ctxs[q], P.D[q], faces, blocks);
        P.total_cells += ncells_of(ctxs[q]);
        total_ncpad += P.D[q].ncpad;
        P.multigrid = P.multigrid || P.D[q].nlev > 1;
    }
    P.nfaces = (int)faces.size();
    if (march_lds_bytes(P.nfaces, L->nT, L->ns) > march_lds_budget(L))
        return fail(RMC_UNSUPPORTED, "face tables of all distinct grids and four table slots (%d nodes, %d species) "
                                     "exceed %d KiB of LDS", L->nT, L->ns, (int)(march_lds_budget(L) / 1024));
    // tiles: whole bricks; about 1024 in total unless the options fix the size
    P.tile_cells = O.alloc_tile > 0 ? O.alloc_tile : auto_tile_cells(total_ncpad);
    // tiles of each snapshot numbered region by region (regions numbered over the pass)
    std::vector<TileInfo> &tiles = L->h_tiles;
    std::vector<uint32_t> &rtile0 = L->h_rtile0;
    tiles.clear();
    rtile0.clear();
    std::vector<uint32_t> reg;
    std::vector<int> perm;
    for (int q = 0; q < nsnap; ++q) {
        SnapDesc &D = P.D[q];
        D.tile_begin = P.ntiles;
        D.ntiles = (int)((D.ncpad + P.tile_cells - 1) / P.tile_cells);
        P.ntiles += D.ntiles;
        tile_regions(D.ncpad, D.nby, D.nbz, D.ntiles, P.tile_cells, O.region_cells, reg);
        perm.resize(D.ntiles);
        for (int t = 0; t < D.ntiles; ++t) perm[t] = t;
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return reg[a] < reg[b]; });
        for (int u = 0; u < D.ntiles; ++u) {
            const int t = perm[u];
            if (u == 0 || reg[t] != reg[perm[u - 1]]) rtile0.push_back((uint32_t)tiles.size());
            tiles.push_back(TileInfo{q, (uint32_t)((uint64_t)t * P.tile_cells), (uint32_t)(rtile0.size() - 1), 0u});
        }
        P.inc_xz = P.inc_xz && D.hx > 0.0 && D.hz > 0.0 && !D.closed;
        P.periodic_xz = P.periodic_xz && !D.closed;
    }
    P.nregion = (int)rtile0.size();
    rtile0.push_back((uint32_t)tiles.size());
    const uint64_t nrun = (uint64_t)P.nregion * nbucket;
    const uint64_t max_items = (P.total_cells * R + nrun * 63 + 63) / 64 * 64;
    P.max_chunks = max_items / 64;
    if (max_items >= (1ull << 32)) return fail(RMC_UNSUPPORTED, "more than 2^32 rays in one pass");
    if ((uint64_t)nbucket * P.ntiles > (1ull << 30))
        return fail(RMC_UNSUPPORTED, "per-tile bucket histograms above 2^30 counters: choose a larger alloc_tile");
    if ((st = L->hist.ensure(sizeof(uint32_t) * (uint64_t)nbucket * P.ntiles)) ||
        (st = L->bucket_total.ensure(sizeof(uint32_t) * nbucket)) ||
        (st = L->rstart.ensure(sizeof(uint32_t) * (nrun + 1))) || (st = L->run_len.ensure(sizeof(uint32_t) * nrun)) ||
        (st = L->region_len.ensure(sizeof(uint32_t) * P.nregion)) ||
        (st = L->rtile0.ensure(sizeof(uint32_t) * (P.nregion + 1))) ||
        (st = L->nchunks.ensure(sizeof(uint32_t))) ||
        (st = L->chunk_bucket.ensure(sizeof(uint32_t) * P.max_chunks)) ||
        (st = L->items.ensure(sizeof(uint2) * max_items)) || (st = L->faces.ensure(sizeof(double) * P.nfaces)) ||
        (st = L->snaps.ensure(sizeof(SnapDesc) * nsnap)) || (st = L->tile_info.ensure(sizeof(TileInfo) * P.ntiles)) ||
        (st = L->border.ensure(sizeof(uint32_t) * nbucket)) ||
        (st = L->counters.ensure(sizeof(unsigned long long) * 4)) ||
        (st = L->red_part.ensure(sizeof(unsigned long long) * 2 * 2048)) ||
        (st = L->kmin.ensure(sizeof(float) * 2 * nb * ng)) || (st = L->cont_count.ensure(sizeof(uint32_t))))
        return st;
    // continuation records of long rays: one per 32 rays of the pass, at least 2^20 (a ray that
    // finds the list full is finished by its lane in the lane kernel, while the wavefront's other
    // lanes wait: learned sampling at R = 128 on the DNS-size grid has more than 2^20 long rays);
    // 2^16 in the allocation-free compute, whose scratch is small
    const uint64_t nrays = P.total_cells * R;
    P.cont_cap = (uint32_t)std::min<uint64_t>(nrays, t_arena ? (1u << 16) : std::max<uint64_t>(1u << 20, nrays / 32));
    if ((st = L->cont.ensure(sizeof(ContRec) * P.cont_cap))) return st;
    {   // kappa lower bound over all snapshots of the batch, then the mean reference kappa
        std::vector<float> tmp, ref, acc((size_t)nb * ng, 0.0f);
        kappa_lower_bounds(ctxs[0], L->h_kmin);
        for (int q = 0; q < nsnap; ++q) {
            if (q > 0) {
                kappa_lower_bounds(ctxs[q], tmp);
                for (size_t u = 0; u < tmp.size(); ++u) L->h_kmin[u] = std::min(L->h_kmin[u], tmp[u]);
            }
            kappa_reference(ctxs[q], ref);
            for (size_t u = 0; u < ref.size(); ++u) acc[u] += ref[u] / (float)nsnap;
        }
        L->h_kmin.insert(L->h_kmin.end(), acc.begin(), acc.end());
    }
    if (t_arena) {   // scratch counters: cleared by a fill kernel at every allocation-free compute
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, L->counters.as<unsigned long long>(), 4);
        HIPCHK(hipGetLastError());
    } else if (!L->have_counters) {
        HIPCHK(hipMemsetAsync(L->counters.p, 0, sizeof(unsigned long long) * 4, s));
        L->have_counters = true;
    }
    L->h_snaps.resize(sizeof(SnapDesc) * nsnap);
    memcpy(L->h_snaps.data(), P.D.data(), sizeof(SnapDesc) * nsnap);
    march_order(L, L->h_order);
    // descriptor uploads from one pinned staging buffer (reused once the last upload is done)
    constexpr int kUp = 6;
    const size_t sz[kUp] = {sizeof(double) * P.nfaces, sizeof(SnapDesc) * nsnap, sizeof(TileInfo) * P.ntiles,
                            sizeof(uint32_t) * nbucket, sizeof(float) * 2 * nb * ng, sizeof(uint32_t) * rtile0.size()};
    const void *src[kUp] = {faces.data(), L->h_snaps.data(), tiles.data(), L->h_order.data(), L->h_kmin.data(),
                            rtile0.data()};
    P.d_faces = L->faces.as<double>();
    P.d_snaps = L->snaps.as<SnapDesc>();
    P.d_tiles = L->tile_info.as<TileInfo>();
    P.d_border = L->border.as<uint32_t>();
    P.d_kmin = L->kmin.as<float>();
    P.d_rtile0 = L->rtile0.as<uint32_t>();
    void *dst[kUp] = {P.d_faces, P.d_snaps, P.d_tiles, P.d_border, P.d_kmin, P.d_rtile0};
    size_t off[kUp], total = 0;
    for (int u = 0; u < kUp; ++u) {
        off[u] = total;
        total += (sz[u] + 255) & ~(size_t)255;
    }
    if (t_arena) {
        // allocation-free compute: copies from the host staging vectors themselves (pageable;
        // they stay unchanged until this context's next compute)
        for (int u = 0; u < kUp; ++u) HIPCHK(hipMemcpyAsync(dst[u], src[u], sz[u], hipMemcpyHostToDevice, s));
        return RMC_OK;
    }
    if (L->up_pending) {
        HIPCHK(hipEventSynchronize(L->up_evt));
        L->up_pending = false;
    }
    if ((st = L->hup.ensure(total))) return st;
    if (!L->up_evt) HIPCHK(hipEventCreateWithFlags(&L->up_evt, hipEventDisableTiming));
    unsigned char *stage = L->hup.as<unsigned char>();
    for (int u = 0; u < kUp; ++u) {
        memcpy(stage + off[u], src[u], sz[u]);
        HIPCHK(hipMemcpyAsync(dst[u], stage + off[u], sz[u], hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipEventRecord(L->up_evt, s));
    L->up_pending = true;
    return RMC_OK;
}

// Device part of a compute: kernel launches only (no allocation, host copy or memset), so
// that the sequence can be captured into a HIP graph.  divq / se are device pointers.
// With EV, phase events are recorded (eager path only).
template <class Real>
rmc_status enqueue_pipeline(const Plan &P, double *const *divq, double *const *se, hipStream_t s,
                            rmc_ctx::EvSet *EV)
{
    rmc_ctx *L = P.ctxs[0];
    rmc_status st;
    const rmc_options &O = L->opt;
    const int nsnap = (int)P.ctxs.size();
    const int nb = L->nb, ng = L->ng, nbucket = nb * ng * 8, R = O.rays_per_cell;
    if (EV) HIPCHK(hipEventRecord(EV->e[0], s));
    // 1-2. per-snapshot pdf and property fields
    for (int q = 0; q < nsnap; ++q)
        if ((st = enqueue_snapshot<Real>(P.ctxs[q], P.D[q], P.d_faces, s))) return st;
    if (EV) HIPCHK(hipEventRecord(EV->e[1], s));

    // 3. allocation: histogram per tile, scan per bucket, layout, scatter
    AllocArgs AA;
    AA.snaps = P.d_snaps;
    AA.tiles = P.d_tiles;
    AA.btotal = L->bucket_total.as<uint32_t>();
    AA.rtile0 = P.d_rtile0;
    AA.ntiles = P.ntiles;
    AA.tile_cells = P.tile_cells;
    AA.nb = nb; AA.ng = ng; AA.nbucket = nbucket; AA.R = R;
    AA.k0 = (uint32_t)O.seed; AA.k1 = (uint32_t)(O.seed >> 32);
    AA.hist = L->hist.as<uint32_t>();
    AA.rstart = L->rstart.as<uint32_t>();
    AA.items = L->items.as<uint2>();
    // 1024 threads per tile unless the bucket counters and the per-thread buckets overflow 64 KiB;
    // the tile's bricks and the plain cdfs go to LDS where they fit beside them
    constexpr size_t kLds = 64 * 1024;
    const int at = sizeof(uint32_t) * (nbucket + kAllocThreads) <= kLds ? kAllocThreads : 256;
    AA.lds_bricks = alloc_scatter_lds(true, nbucket, at, P.tile_cells) <= kLds ? 1 : 0;
    AA.lds_cdf = P.smode != 0 ? 0
                 : alloc_count_lds(2, AA.lds_bricks, nb, ng, nbucket, P.tile_cells) <= kLds ? 2
                 : alloc_count_lds(1, AA.lds_bricks, nb, ng, nbucket, P.tile_cells) <= kLds ? 1 : 0;
    const size_t lds_count = alloc_count_lds(AA.lds_cdf, AA.lds_bricks, nb, ng, nbucket, P.tile_cells);
    const size_t lds_scatter = alloc_scatter_lds(AA.lds_bricks, nbucket, at, P.tile_cells);
    if (P.smode == 2) hipLaunchKernelGGL(k_alloc_count<2>, dim3(P.ntiles), dim3(at), lds_count, s, AA);
    else if (P.smode == 1) hipLaunchKernelGGL(k_alloc_count<1>, dim3(P.ntiles), dim3(at), lds_count, s, AA);
    else hipLaunchKernelGGL(k_alloc_count<0>, dim3(P.ntiles), dim3(at), lds_count, s, AA);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_bucket_scan, dim3(nbucket), dim3(64), 0, s, L->hist.as<uint32_t>(), P.ntiles,
                       L->bucket_total.as<uint32_t>());
    HIPCHK(hipGetLastError());
    const uint64_t nrun = (uint64_t)P.nregion * nbucket;
    hipLaunchKernelGGL(k_run_len, dim3((unsigned)((nrun + 255) / 256)), dim3(256), 0, s, L->hist.as<uint32_t>(),
                       L->bucket_total.as<uint32_t>(), P.ntiles, P.d_rtile0, nbucket, nrun, L->run_len.as<uint32_t>());
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_run_region_sum, dim3(P.nregion), dim3(1024), 0, s, L->run_len.as<uint32_t>(), nbucket,
                       L->region_len.as<uint32_t>());
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_run_layout, dim3(P.nregion), dim3(1024), 0, s, L->run_len.as<uint32_t>(),
                       L->region_len.as<uint32_t>(), P.d_border, nbucket, P.nregion, L->rstart.as<uint32_t>(),
                       L->nchunks.as<uint32_t>());
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_chunk_map, dim3((unsigned)((nrun + 3) / 4)), dim3(64, 4), 0, s, L->hist.as<uint32_t>(),
                       L->bucket_total.as<uint32_t>(), P.ntiles, P.d_rtile0, L->rstart.as<uint32_t>(), nbucket, nrun,
                       L->chunk_bucket.as<uint32_t>(), L->items.as<uint2>());
    HIPCHK(hipGetLastError());
    if (P.smode == 2) hipLaunchKernelGGL(k_alloc_scatter<2>, dim3(P.ntiles), dim3(at), lds_scatter, s, AA);
    else if (P.smode == 1) hipLaunchKernelGGL(k_alloc_scatter<1>, dim3(P.ntiles), dim3(at), lds_scatter, s, AA);
    else hipLaunchKernelGGL(k_alloc_scatter<0>, dim3(P.ntiles), dim3(at), lds_scatter, s, AA);
    HIPCHK(hipGetLastError());
    if (EV) HIPCHK(hipEventRecord(EV->e[2], s));

    // 4. march: one wavefront per 64-ray chunk
    MarchArgs<Real> MA;
    MA.snaps = P.d_snaps;
    MA.faces = P.d_faces;
    MA.nfaces = P.nfaces;
    MA.items = L->items.as<uint2>();
    MA.chunk_bucket = L->chunk_bucket.as<uint32_t>();
    MA.nchunks = L->nchunks.as<uint32_t>();
    MA.dnu = L->dnu.as<double>();
    MA.wg = L->wg.as<double>();
    MA.nb = nb; MA.ng = ng; MA.R = R;
    MA.k0 = AA.k0; MA.k1 = AA.k1;
    MA.tol = (Real)O.tol;
    MA.max_steps = O.max_steps;
    // long rays are segmented only in the FP32 march over uniform periodic x and z
    const bool segment = sizeof(Real) == 4 && P.inc_xz && P.periodic_xz;
    const int lrs = O.long_ray_steps > 0 ? O.long_ray_steps : 512;
    MA.cap = segment ? std::min(lrs, O.max_steps) : O.max_steps;
    MA.kmin = P.d_kmin;
    MA.kref = P.d_kmin + (size_t)nb * ng;
    MA.cont = L->cont.as<ContRec>();
    MA.cont_count = L->cont_count.as<uint32_t>();
    MA.cont_cap = P.cont_cap;
    MA.long_steps = L->counters.as<unsigned long long>() + 3;
    MA.log_inv_tol = O.tol > 0.0 ? (float)std::log(1.0 / O.tol) : 1e30f;
    MA.long_form = O.long_ray_form;
    MA.Ib = L->Ib.as<double>();
    MA.k32 = L->k32.as<float>();
    MA.nT = L->nT;
    MA.ns = L->ns;
    MA.tab_off = (P.nfaces + 1) & ~1;
    MA.slot_dbl = table_slot_doubles(L->nT, L->ns);
    MA.span_log2 = 0;
    for (int sp = O.xcd_span > 0 ? O.xcd_span : 256; sp > 1; sp >>= 1) ++MA.span_log2;
    for (const SnapDesc &d : P.D)
        if (d.wallq) {   // wall flux tally of this compute (a fill kernel: no memset, graph-safe)
            const uint64_t nw = 2 * ((uint64_t)d.ny * d.nz + (uint64_t)d.nx * d.nz + (uint64_t)d.nx * d.ny);
            hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, d.wallq, nw);
        }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, L->cont_count.as<uint32_t>(), 1);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, L->counters.as<unsigned long long>() + 3, 1);
    HIPCHK(hipGetLastError());
    const unsigned mblocks = (unsigned)xcd_blocks(P.max_chunks, MA.span_log2);
    const size_t lds_faces = march_lds_bytes(P.nfaces, L->nT, L->ns);   // faces and four table slots
    const bool multi = nsnap > 1;
    const bool lsort = O.length_sort == 1;
#define RMC_MARCH(PDF_, INC_, MULTI_)                                                                             \
    do {                                                                                                        \
        if (lsort) hipLaunchKernelGGL((k_march_lane<Real, PDF_, INC_, MULTI_, true>), dim3(mblocks), dim3(256), \
                                      lds_faces, s, MA);                                                        \
        else hipLaunchKernelGGL((k_march_lane<Real, PDF_, INC_, MULTI_, false>), dim3(mblocks), dim3(256),      \
                                lds_faces, s, MA);                                                              \
    } while (0)
#define RMC_MARCH_MG(PDF_, INC_, MULTI_) \
    hipLaunchKernelGGL((k_march_mg<Real, PDF_, INC_, MULTI_>), dim3(mblocks), dim3(256), lds_faces, s, MA)
    if (P.multigrid) {
        if (P.pdf_mode) {
            if (P.inc_xz) { if (multi) RMC_MARCH_MG(true, true, true); else RMC_MARCH_MG(true, true, false); }
            else { if (multi) RMC_MARCH_MG(true, false, true); else RMC_MARCH_MG(true, false, false); }
        } else {
            if (P.inc_xz) { if (multi) RMC_MARCH_MG(false, true, true); else RMC_MARCH_MG(false, true, false); }
            else { if (multi) RMC_MARCH_MG(false, false, true); else RMC_MARCH_MG(false, false, false); }
        }
    } else if (P.pdf_mode) {
        if (P.inc_xz) { if (multi) RMC_MARCH(true, true, true); else RMC_MARCH(true, true, false); }
        else { if (multi) RMC_MARCH(true, false, true); else RMC_MARCH(true, false, false); }
    } else {
        if (P.inc_xz) { if (multi) RMC_MARCH(false, true, true); else RMC_MARCH(false, true, false); }
        else { if (multi) RMC_MARCH(false, false, true); else RMC_MARCH(false, false, false); }
    }
#undef RMC_MARCH
#undef RMC_MARCH_MG
    HIPCHK(hipGetLastError());
    if (EV) HIPCHK(hipEventRecord(EV->e[3], s));
    if constexpr (sizeof(Real) == 4) {
        if (segment && MA.cap < O.max_steps) {
            // a workgroup or a wavefront per long ray (chosen on the device by their count);
            // the workgroups past the work exit at once
            const dim3 lg(4096), lb(256);
            if (P.pdf_mode) {
                if (multi) hipLaunchKernelGGL((k_march_long<true, true>), lg, lb, lds_faces, s, MA);
                else hipLaunchKernelGGL((k_march_long<true, false>), lg, lb, lds_faces, s, MA);
            } else {
                if (multi) hipLaunchKernelGGL((k_march_long<false, true>), lg, lb, lds_faces, s, MA);
                else hipLaunchKernelGGL((k_march_long<false, false>), lg, lb, lds_faces, s, MA);
            }
            HIPCHK(hipGetLastError());
        }
    }
    if (EV) HIPCHK(hipEventRecord(EV->e[4], s));

    // 5. per-cell reduction into the (device) output buffers
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, L->counters.as<unsigned long long>(), 2);
    HIPCHK(hipGetLastError());
    for (int q = 0; q < nsnap; ++q) {
        rmc_ctx *c = P.ctxs[q];
        const uint64_t nc = ncells_of(c);
        const uint64_t groups = (nc + (kRedVals / R) - 1) / (kRedVals / R);
        const int nblk = (int)std::min<uint64_t>(groups, 2048);
        hipLaunchKernelGGL(k_reduce<Real>, dim3((unsigned)nblk), dim3(kRedThreads), 0, s, c->Y.p,
                           sizeof(Real) == 8 ? c->st.as<uint32_t>() : nullptr, nc, R, (int)O.accum, divq[q],
                           se ? se[q] : nullptr, L->red_part.as<unsigned long long>());
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_reduce_counts, dim3(1), dim3(256), 0, s, L->red_part.as<unsigned long long>(), nblk,
                           L->counters.as<unsigned long long>());
        HIPCHK(hipGetLastError());
    }
    if (EV) HIPCHK(hipEventRecord(EV->e[5], s));
    return RMC_OK;
}

// Eager compute: plan, enqueue with phase events, copy host outputs back.
template <class Real>
rmc_status run_pipeline(rmc_ctx *const *ctxs, int nsnap, double *const *divq, double *const *se, rmc_mem mem,
                        hipStream_t s)
{
    rmc_ctx *L = ctxs[0];
    rmc_status st;
    if (L->ring.empty()) {
        L->ring.resize(256);
        for (auto &set : L->ring)
            for (auto &e : set.e) HIPCHK(hipEventCreate(&e));
    }
    const int set_idx = (int)(L->ring_head % L->ring.size());
    rmc_ctx::EvSet &EV = L->ring[set_idx];
    if (EV.pending && (st = harvest(L, EV))) return st;
    Plan P;
    if ((st = plan_pipeline<Real>(ctxs, nsnap, P, s))) return st;
    std::vector<double *> dq(nsnap), sq(nsnap, nullptr);
    for (int q = 0; q < nsnap; ++q) {
        const uint64_t nc = ncells_of(ctxs[q]);
        dq[q] = divq[q];
        sq[q] = se ? se[q] : nullptr;
        if (mem == RMC_HOST) {
            if ((st = ctxs[q]->outbuf.ensure(sizeof(double) * 2 * nc))) return st;
            dq[q] = ctxs[q]->outbuf.as<double>();
            sq[q] = (se && se[q]) ? dq[q] + nc : nullptr;
        }
    }
    if ((st = enqueue_pipeline<Real>(P, dq.data(), sq.data(), s, &EV))) return st;
    if (mem == RMC_HOST)
        for (int q = 0; q < nsnap; ++q) {
            const uint64_t nc = ncells_of(ctxs[q]);
            HIPCHK(hipMemcpyAsync(divq[q], dq[q], sizeof(double) * nc, hipMemcpyDeviceToHost, s));
            if (sq[q]) HIPCHK(hipMemcpyAsync(se[q], sq[q], sizeof(double) * nc, hipMemcpyDeviceToHost, s));
        }
    EV.pending = true;
    EV.rays = (int64_t)P.total_cells * L->opt.rays_per_cell;
    L->last_set = set_idx;
    ++L->ring_head;
    return RMC_OK;
}

// Temperature ingest, enqueued: conversion to FP64, range check, maximum and minimum into the
// context's reduction slots and (pinned) readback; ingest_T_finish reads them after a sync.
rmc_status ingest_T_enqueue(rmc_ctx *c, const void *src, rmc_dtype dt, rmc_mem mem, hipStream_t s)
{
    ++c->input_version;   // the fields change: the learned allocation cache is stale
    const uint64_t nc = ncells_of(c);
    const size_t esz = dt == RMC_F32 ? 4 : 8;
    rmc_status st;
    if ((st = c->T.ensure(sizeof(double) * nc)) || (st = c->small.ensure(256)) ||
        (st = c->scal.ensure(sizeof(double) * 9)) || (st = c->hread.ensure(256)))
        return st;
    const void *dsrc = src;
    if (mem == RMC_HOST) {
        if ((st = c->stage.ensure(esz * nc))) return st;
        HIPCHK(hipMemcpyAsync(c->stage.p, src, esz * nc, hipMemcpyHostToDevice, s));
        dsrc = c->stage.p;
    }
    unsigned long long *mx = c->small.as<unsigned long long>() + kSmallT;
    unsigned int *flag = reinterpret_cast<unsigned int *>(mx + 1);
    hipLaunchKernelGGL(k_small_init, dim3(1), dim3(64), 0, s, c->small.as<unsigned long long>(), 0, 1);
    const unsigned blocks = (unsigned)std::min<uint64_t>(512, (nc + 255) / 256);
    if (dt == RMC_F32)
        hipLaunchKernelGGL(k_ingest_T<float>, dim3(blocks), dim3(256), 0, s, (const float *)dsrc, c->T.as<double>(),
                           nc, c->T0, c->dT, c->nT, mx, flag);
    else
        hipLaunchKernelGGL(k_ingest_T<double>, dim3(blocks), dim3(256), 0, s, (const double *)dsrc,
                           c->T.as<double>(), nc, c->T0, c->dT, c->nT, mx, flag);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->hread.as<unsigned long long>() + kSmallT, mx, 24, hipMemcpyDeviceToHost, s));
    // the maximum's bits are the double itself: copied on the device before the caller's sync
    // (a rejected field is never used, so the copy needs no check)
    HIPCHK(hipMemcpyAsync(c->scal.p, mx, sizeof(double), hipMemcpyDeviceToDevice, s));
    return RMC_OK;
}

rmc_status ingest_T_finish(rmc_ctx *c)
{
    const unsigned long long *host = c->hread.as<unsigned long long>() + kSmallT;
    if ((unsigned)host[1] & 1u) {
        c->have_T = false;
        return fail(RMC_OUT_OF_RANGE, "temperature outside the table range [%g, %g] or NaN", c->T0,
                    c->T0 + c->dT * (c->nT - 1));
    }
    memcpy(&c->Tmax_cells, &host[0], 8);
    memcpy(&c->Tmin_cells, &host[2], 8);
    c->have_T = true;
    return RMC_OK;
}

// Mole-fraction ingest, enqueued (see ingest_T_enqueue); maxima x-hat and minima per species.
rmc_status ingest_X_enqueue(rmc_ctx *c, int ns, const void *X, rmc_dtype dt, rmc_mem mem, hipStream_t s)
{
    ++c->input_version;   // the fields change: the learned allocation cache is stale
    const uint64_t nc = ncells_of(c);
    const size_t esz = dt == RMC_F32 ? 4 : 8;
    rmc_status st;
    if ((st = c->X.ensure(sizeof(double) * nc * ns)) || (st = c->small.ensure(256)) ||
        (st = c->scal.ensure(sizeof(double) * 9)) || (st = c->hread.ensure(256)))
        return st;
    const void *dsrc = X;
    if (mem == RMC_HOST) {
        if ((st = c->stage2.ensure(esz * nc * ns))) return st;
        HIPCHK(hipMemcpyAsync(c->stage2.p, X, esz * nc * ns, hipMemcpyHostToDevice, s));
        dsrc = c->stage2.p;
    }
    unsigned long long *mx = c->small.as<unsigned long long>() + kSmallX;
    unsigned int *flag = reinterpret_cast<unsigned int *>(mx + 16);
    hipLaunchKernelGGL(k_small_init, dim3(1), dim3(64), 0, s, c->small.as<unsigned long long>(), 1, 0);
    const unsigned blocks = (unsigned)std::min<uint64_t>(512, (nc + 255) / 256);
    if (dt == RMC_F32)
        hipLaunchKernelGGL(k_ingest_X<float>, dim3(blocks), dim3(256), 0, s, (const float *)dsrc, c->X.as<double>(),
                           nc, ns, mx, flag);
    else
        hipLaunchKernelGGL(k_ingest_X<double>, dim3(blocks), dim3(256), 0, s, (const double *)dsrc,
                           c->X.as<double>(), nc, ns, mx, flag);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->hread.as<unsigned long long>() + kSmallX, mx, sizeof(unsigned long long) * 17,
                          hipMemcpyDeviceToHost, s));
    // the maxima's bits are the doubles themselves: copied on the device before the caller's sync
    HIPCHK(hipMemcpyAsync(c->scal.as<double>() + 1, mx, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
    return RMC_OK;
}

rmc_status ingest_X_finish(rmc_ctx *c, int ns)
{
    const unsigned long long *host = c->hread.as<unsigned long long>() + kSmallX;
    if ((unsigned)host[16] & 1u) {
        c->have_X = false;
        return fail(RMC_OUT_OF_RANGE, "mole fractions must be finite and >= 0");
    }
    for (int q = 0; q < ns; ++q) {
        memcpy(&c->xhat[q], &host[q], 8);
        memcpy(&c->xmin[q], &host[8 + q], 8);
    }
    c->have_X = true;
    return RMC_OK;
}

}  // namespace

struct rmc_graph {
    int device = 0;
    std::vector<rmc_ctx *> ctxs;
    std::vector<uint64_t> versions;
    std::vector<std::vector<void *>> ptrs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DBuf faces, snaps, tile_info, border, kmin, rtile0;   // the graph's own copies of the planned tables
};

namespace {

// device buffers a captured compute reads or writes (a change means they were reallocated)
std::vector<void *> buffer_ptrs(const rmc_ctx *c)
{
    const DBuf *b[] = {&c->k64, &c->k32, &c->Ib, &c->dnu, &c->wg, &c->T, &c->X, &c->scal, &c->q, &c->cpdf, &c->ccdf_b,
                       &c->ccdf_g, &c->ccdf_o, &c->pdf_scratch, &c->p, &c->cdf_b, &c->cdf_g, &c->W, &c->Iw,
                       &c->status, &c->rec, &c->Y, &c->st, &c->hist, &c->bucket_total,
                       &c->rstart, &c->run_len, &c->region_len, &c->rtile0, &c->nchunks, &c->chunk_bucket, &c->items, &c->faces,
                       &c->snaps, &c->tile_info, &c->border, &c->counters, &c->red_part, &c->kmin, &c->cont, &c->cont_count,
                       &c->rbkt, &c->mgT, &c->mgX, &c->mgrec, &c->dprob, &c->dstrat, &c->lpp, &c->prm,
                       &c->musd, &c->nu_c, &c->gxs, &c->kp, &c->feat, &c->fmask, &c->bng, &c->lfaces};
    std::vector<void *> v;
    for (const DBuf *d : b) v.push_back(d->p);
    return v;
}

// shared validation of a batch (compute or capture)
rmc_status check_batch(rmc_ctx *const *ctxs, int nsnap)
{
    if (!ctxs || nsnap < 1 || nsnap > 32767) return fail(RMC_INVALID_ARG, "bad batch arguments");
    rmc_ctx *L = ctxs[0];
    if (!L) return fail(RMC_INVALID_ARG, "null context");
    for (int q = 0; q < nsnap; ++q) {
        rmc_ctx *c = ctxs[q];
        if (!c) return fail(RMC_INVALID_ARG, "null context in the batch");
        if (rmc_status st = check_ready(c)) return st;
        if (c->device != L->device) return fail(RMC_INVALID_ARG, "batch contexts must share one device");
        if (c->nb != L->nb || c->ng != L->ng || c->ns != L->ns || c->nT != L->nT || c->T0 != L->T0 ||
            c->dT != L->dT)
            return fail(RMC_INVALID_ARG, "batch contexts must share the tables");
        const rmc_options &a = c->opt, &b = L->opt;
        if (a.rays_per_cell != b.rays_per_cell || a.seed != b.seed || a.tol != b.tol || a.max_steps != b.max_steps ||
            a.march != b.march || a.accum != b.accum || a.sampling != b.sampling)
            return fail(RMC_INVALID_ARG, "batch contexts must share the options (snapshot ids may differ)");
        for (int q2 = 0; q2 < q; ++q2)
            if (ctxs[q2] == c) return fail(RMC_INVALID_ARG, "a context appears twice in the batch");
    }
    return RMC_OK;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

const char *rmc_last_error(void) { return g_err.c_str(); }

void rmc_default_options(rmc_options *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->rays_per_cell = 16;
    o->seed = 0;
    o->snapshot = 0;
    o->tol = 1e-6;
    o->max_steps = 65536;
    o->march = RMC_F32;
    o->accum = RMC_ACC_F64;
    o->sampling = RMC_SAMPLING_PLAIN;
    o->mix_eps = 0.1;
    o->block_threads = 0;
}

rmc_status rmc_create(int device, rmc_ctx **out)
{
    g_err.clear();
    if (!out) return fail(RMC_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(RMC_DEVICE_ERROR, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return fail(RMC_INVALID_ARG, "device %d out of range [0, %d)", device, ndev);
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            DeviceGuard g(device);
            void *ptr = nullptr;
            const hipError_t se = g.ok ? hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) : hipErrorInvalidDevice;
            if (se == hipSuccess && ptr) g_scratch_ptr[device] = ptr;
            else {
                (void)hipGetLastError();
                g_scratch_err[device] = se == hipSuccess ? hipErrorInvalidSymbol : se;
            }
        }
    }
    rmc_ctx *c = new (std::nothrow) rmc_ctx();
    if (!c) return fail(RMC_OUT_OF_MEMORY, "context allocation failed");
    c->device = device;
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
            lds >= 64 * 1024)
            c->lds_max = (size_t)lds;
        (void)hipGetLastError();
    }
    rmc_default_options(&c->opt);
    *out = c;
    return RMC_OK;
}

void rmc_destroy(rmc_ctx *c)
{
    if (!c) return;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        DBuf *bufs[] = {&c->k64, &c->k32, &c->Ib, &c->dnu, &c->wg, &c->T, &c->X, &c->stage, &c->stage2, &c->q, &c->cpdf, &c->ccdf_b,
                        &c->ccdf_g, &c->ccdf_o, &c->pdf_scratch, &c->p, &c->cdf_b, &c->cdf_g, &c->W, &c->Iw,
                        &c->status, &c->rec, &c->Y, &c->st, &c->hist, &c->bucket_total, &c->rstart, &c->run_len, &c->region_len, &c->rtile0,
                        &c->nchunks, &c->chunk_bucket, &c->items, &c->faces, &c->snaps, &c->tile_info,
                        &c->counters, &c->red_part, &c->outbuf, &c->tune_out, &c->trace_rec, &c->trace_cells, &c->border, &c->small, &c->scal,
                        &c->kmin, &c->cont, &c->cont_count};
        for (DBuf *b : bufs) b->release();
        for (auto &set : c->ring)
            for (auto &ev : set.e) (void)hipEventDestroy(ev);
        if (c->up_evt) (void)hipEventDestroy(c->up_evt);
        delete c;   // the remaining buffers are released with the device still current
    }
}

rmc_status rmc_set_grid(rmc_ctx *c, int nx, int ny, int nz, const double *xf, const double *yf, const double *zf)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    ++c->input_version;
    if (nx < 1 || ny < 1 || nz < 1 || nx > 1023 || ny > 1023 || nz > 1023)
        return fail(RMC_INVALID_ARG, "grid dimensions must be in [1, 1023]");
    if (!xf || !yf || !zf) return fail(RMC_INVALID_ARG, "null face array");
    auto mono = [](const double *f, int n) {
        for (int q = 0; q <= n; ++q)
            if (!std::isfinite(f[q]) || (q > 0 && !(f[q] > f[q - 1]))) return false;
        return true;
    };
    if (!mono(xf, nx) || !mono(yf, ny) || !mono(zf, nz))
        return fail(RMC_INVALID_ARG, "face coordinates must be finite and strictly increasing");
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->xf.assign(xf, xf + nx + 1);
    c->yf.assign(yf, yf + ny + 1);
    c->zf.assign(zf, zf + nz + 1);
    c->have_grid = true;
    c->have_T = c->have_X = c->have_q = false;
    ++c->config_version;
    return RMC_OK;
}

rmc_status rmc_set_walls(rmc_ctx *c, double T0, double T1, double e0, double e1)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    ++c->input_version;
    if (!std::isfinite(T0) || !std::isfinite(T1) || T0 < 0 || T1 < 0)
        return fail(RMC_INVALID_ARG, "wall temperatures must be finite and >= 0");
    if (!(e0 >= 0.0 && e0 <= 1.0) || !(e1 >= 0.0 && e1 <= 1.0))
        return fail(RMC_INVALID_ARG, "wall emissivities must lie in [0, 1]");
    c->Tw[0] = T0;
    c->Tw[1] = T1;
    c->epsw[0] = e0;
    c->epsw[1] = e1;
    c->have_walls = true;
    ++c->config_version;
    return RMC_OK;
}

rmc_status rmc_set_box_walls(rmc_ctx *c, const double *T, const double *eps)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    ++c->input_version;
    if (!T) {
        c->closed = false;
        ++c->config_version;
        return RMC_OK;
    }
    if (!eps) return fail(RMC_INVALID_ARG, "eps must be given with T");
    for (int q = 0; q < 4; ++q) {
        if (!std::isfinite(T[q]) || T[q] < 0) return fail(RMC_INVALID_ARG, "wall temperatures must be finite and >= 0");
        if (!(eps[q] >= 0.0 && eps[q] <= 1.0)) return fail(RMC_INVALID_ARG, "wall emissivities must lie in [0, 1]");
    }
    for (int q = 0; q < 4; ++q) {
        c->Tbox[q] = T[q];
        c->epsbox[q] = eps[q];
    }
    c->closed = true;
    ++c->config_version;
    return RMC_OK;
}

rmc_status rmc_set_kdist(rmc_ctx *c, int nb, int ng, int ns, int nT, double T0, double dT, const double *dnu,
                         const double *wg, const void *k, rmc_dtype kdt, const double *Ib)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    ++c->input_version;
    if (nb < 1 || nb > 4096 || ng < 1 || ng > 255 || ns < 1 || ns > 8 || nT < 2)
        return fail(RMC_INVALID_ARG, "table sizes out of range");
    if (nb * ng > 2000) return fail(RMC_UNSUPPORTED, "nb * ng must not exceed 2000");
    if (!(std::isfinite(T0) && T0 >= 0.0 && std::isfinite(dT) && dT > 0.0))
        return fail(RMC_INVALID_ARG, "T0 must be >= 0 and dT > 0");
    if (!dnu || !wg || !k || !Ib) return fail(RMC_INVALID_ARG, "null table pointer");
    if (kdt != RMC_F32 && kdt != RMC_BF16) return fail(RMC_INVALID_ARG, "k dtype must be RMC_F32 or RMC_BF16");
    const size_t nk = (size_t)ns * nb * ng * nT;
    std::vector<double> k64(nk);
    for (size_t q = 0; q < nk; ++q) {
        double v;
        if (kdt == RMC_F32) v = ((const float *)k)[q];
        else {
            uint32_t u = (uint32_t)((const uint16_t *)k)[q] << 16;
            float f;
            memcpy(&f, &u, 4);
            v = f;
        }
        if (!(v >= 0.0 && std::isfinite(v))) return fail(RMC_INVALID_ARG, "absorption coefficients must be finite and >= 0");
        k64[q] = v;
    }
    for (int q = 0; q < nb; ++q)
        if (!(dnu[q] > 0.0 && std::isfinite(dnu[q]))) return fail(RMC_INVALID_ARG, "band widths must be > 0");
    for (int q = 0; q < ng; ++q)
        if (!(wg[q] > 0.0 && std::isfinite(wg[q]))) return fail(RMC_INVALID_ARG, "quadrature weights must be > 0");
    for (size_t q = 0; q < (size_t)nb * nT; ++q)
        if (!(Ib[q] >= 0.0 && std::isfinite(Ib[q]))) return fail(RMC_INVALID_ARG, "Planck table must be finite and >= 0");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    rmc_status st;
    if ((st = c->k64.ensure(sizeof(double) * nk)) || (st = c->k32.ensure(sizeof(float) * nk)) ||
        (st = c->Ib.ensure(sizeof(double) * nb * nT)) || (st = c->dnu.ensure(sizeof(double) * nb)) ||
        (st = c->wg.ensure(sizeof(double) * ng)))
        return st;
    HIPCHK(hipMemcpy(c->k64.p, k64.data(), sizeof(double) * nk, hipMemcpyHostToDevice));
    {
        std::vector<float> k32(nk);
        for (size_t q = 0; q < nk; ++q) k32[q] = (float)k64[q];   // exact: F32 or BF16 inputs
        HIPCHK(hipMemcpy(c->k32.p, k32.data(), sizeof(float) * nk, hipMemcpyHostToDevice));
    }
    c->k64_host = k64;
    HIPCHK(hipMemcpy(c->Ib.p, Ib, sizeof(double) * nb * nT, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->dnu.p, dnu, sizeof(double) * nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->wg.p, wg, sizeof(double) * ng, hipMemcpyHostToDevice));
    const bool same_range = c->have_kdist && c->T0 == T0 && c->dT == dT && c->nT == nT;
    c->nb = nb; c->ng = ng; c->nT = nT; c->T0 = T0; c->dT = dT;
    if (c->ns != ns) c->have_X = false;
    c->ns = ns;
    c->have_kdist = true;
    if (!same_range) c->have_T = false;   // temperatures must be re-validated against the new range
    c->have_q = false;
    c->have_alloc = false;                // band centres and g abscissae belong to the tables
    ++c->config_version;
    return RMC_OK;
}

rmc_status rmc_set_temperature(rmc_ctx *c, const void *T, rmc_dtype dt, rmc_mem mem, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!c->have_grid || !c->have_kdist) return fail(RMC_BAD_STATE, "set_grid and set_kdist must come first");
    if (!T) return fail(RMC_INVALID_ARG, "null temperature pointer");
    if (dt != RMC_F32 && dt != RMC_F64) return fail(RMC_INVALID_ARG, "temperature dtype must be RMC_F32 or RMC_F64");
    if (mem != RMC_HOST && mem != RMC_DEVICE) return fail(RMC_INVALID_ARG, "bad memory kind");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    if (rmc_status st = ingest_T_enqueue(c, T, dt, mem, s)) return st;
    HIPCHK(hipStreamSynchronize(s));
    return ingest_T_finish(c);
}

rmc_status rmc_set_species(rmc_ctx *c, int ns, const void *X, rmc_dtype dt, rmc_mem mem, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!c->have_grid || !c->have_kdist) return fail(RMC_BAD_STATE, "set_grid and set_kdist must come first");
    if (ns != c->ns) return fail(RMC_INVALID_ARG, "ns = %d does not match the tables (%d)", ns, c->ns);
    if (!X) return fail(RMC_INVALID_ARG, "null species pointer");
    if (dt != RMC_F32 && dt != RMC_F64) return fail(RMC_INVALID_ARG, "species dtype must be RMC_F32 or RMC_F64");
    if (mem != RMC_HOST && mem != RMC_DEVICE) return fail(RMC_INVALID_ARG, "bad memory kind");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    if (rmc_status st = ingest_X_enqueue(c, ns, X, dt, mem, s)) return st;
    HIPCHK(hipStreamSynchronize(s));
    return ingest_X_finish(c, ns);
}

rmc_status rmc_set_fields(rmc_ctx *c, const void *T, rmc_dtype T_dtype, int ns, const void *X, rmc_dtype X_dtype,
                          rmc_mem mem, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!c->have_grid || !c->have_kdist) return fail(RMC_BAD_STATE, "set_grid and set_kdist must come first");
    if (!T) return fail(RMC_INVALID_ARG, "null temperature pointer");
    if (!X) return fail(RMC_INVALID_ARG, "null species pointer");
    if (ns != c->ns) return fail(RMC_INVALID_ARG, "ns = %d does not match the tables (%d)", ns, c->ns);
    if ((T_dtype != RMC_F32 && T_dtype != RMC_F64) || (X_dtype != RMC_F32 && X_dtype != RMC_F64))
        return fail(RMC_INVALID_ARG, "field dtypes must be RMC_F32 or RMC_F64");
    if (mem != RMC_HOST && mem != RMC_DEVICE) return fail(RMC_INVALID_ARG, "bad memory kind");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    if (rmc_status st = ingest_T_enqueue(c, T, T_dtype, mem, s)) return st;
    if (rmc_status st = ingest_X_enqueue(c, ns, X, X_dtype, mem, s)) return st;
    HIPCHK(hipStreamSynchronize(s));
    const rmc_status st_T = ingest_T_finish(c);
    const std::string err_T = g_err;
    const rmc_status st_X = ingest_X_finish(c, ns);
    if (st_T) {   // report the temperature's error first
        g_err = err_T;
        return st_T;
    }
    return st_X;
}

rmc_status rmc_set_options(rmc_ctx *c, const rmc_options *o)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!o) return fail(RMC_INVALID_ARG, "null options");
    if (rmc_status st = check_options(o)) return st;
    c->opt = *o;
    ++c->config_version;
    return RMC_OK;
}

rmc_status rmc_get_options(const rmc_ctx *c, rmc_options *o)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!o) return fail(RMC_INVALID_ARG, "null options");
    *o = c->opt;
    return RMC_OK;
}

}  // extern "C"

namespace {

// Workload signature of an autotuning cache line: the device architecture and everything that
// sets the amount and the shape of the work (every grid of a batch).
std::string tune_signature(rmc_ctx *const *ctxs, int nsnap)
{
    const rmc_ctx *c = ctxs[0];
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    char buf[256];
    snprintf(buf, sizeof buf, "rmc-tune-2 %s %d %d %d %d %d %d %d %d %d %d %d", arch.c_str(), c->nb, c->ng, c->ns,
             c->opt.rays_per_cell, (int)c->opt.march, (int)c->opt.sampling, c->opt.long_ray_steps, c->opt.max_steps,
             c->opt.mg_levels, c->opt.mg_steps, nsnap);
    std::string sig = buf;
    for (int q = 0; q < nsnap; ++q) {
        snprintf(buf, sizeof buf, " %dx%dx%d", ctxs[q]->nx, ctxs[q]->ny, ctxs[q]->nz);
        sig += buf;
    }
    return sig;
}

bool tune_cache_lookup(const char *path, const std::string &sig, int &span, int &sort, int &tile)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    std::vector<char> line(sig.size() + 256);
    bool hit = false;
    while (fgets(line.data(), (int)line.size(), f)) {
        const char *sep = strstr(line.data(), " : ");
        if (!sep || (size_t)(sep - line.data()) != sig.size() || strncmp(line.data(), sig.c_str(), sig.size()) != 0)
            continue;
        int a = 0, b = 0, t = 0;
        if (sscanf(sep + 3, "%d %d %d", &a, &b, &t) == 3) { span = a; sort = b; tile = t; hit = true; }   // last line wins
    }
    fclose(f);
    return hit;
}

}  // namespace

extern "C" {

rmc_status rmc_autotune_batch(rmc_ctx *const *ctxs, int nsnap, int reps, const char *cache_path, rmc_options *out,
                              void *stream)
{
    g_err.clear();
    if (rmc_status st = check_batch(ctxs, nsnap)) return st;
    if (reps < 1 || reps > 100) return fail(RMC_INVALID_ARG, "reps must be in [1, 100]");
    rmc_ctx *c = ctxs[0];   // the leader's options govern the schedule of a batch
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    const std::string sig = tune_signature(ctxs, nsnap);
    rmc_options best = c->opt;
    int span = 0, sort = 0, tile = 0;
    if (cache_path && tune_cache_lookup(cache_path, sig, span, sort, tile)) {
        best.xcd_span = span;
        best.length_sort = sort;
        best.alloc_tile = tile;
        if (rmc_status st = check_options(&best)) return fail(st, "bad autotuning cache entry in %s", cache_path);
    } else {
        hipStream_t s = (hipStream_t)stream;
        rmc_status st;
        std::vector<double *> dq(nsnap), se(nsnap);
        uint64_t total_ncpad = 0;
        for (int q = 0; q < nsnap; ++q) {
            const uint64_t nc = ncells_of(ctxs[q]);
            if ((st = ctxs[q]->tune_out.ensure(sizeof(double) * 2 * nc))) return st;
            dq[q] = ctxs[q]->tune_out.as<double>();
            se[q] = dq[q] + nc;
            total_ncpad += ncpad_of(ctxs[q]);
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const rmc_options base = c->opt;
        float best_ms = 0.0f;
        bool have = false;
        auto time_candidate = [&](const rmc_options &o) -> rmc_status {
            c->opt = o;
            rmc_status r = rmc_compute_batch(ctxs, nsnap, dq.data(), se.data(), RMC_DEVICE, stream);   // warm-up
            if (r) return r;
            if (hipEventRecord(e0, s) != hipSuccess) return fail(RMC_DEVICE_ERROR, "hipEventRecord failed");
            for (int q = 0; q < reps && !r; ++q) r = rmc_compute_batch(ctxs, nsnap, dq.data(), se.data(), RMC_DEVICE, stream);
            if (r) return r;
            float ms = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return fail(RMC_DEVICE_ERROR, "timing the autotuning candidates failed");
            if (!have || ms < best_ms) { best_ms = ms; best = o; have = true; }
            return RMC_OK;
        };
        // stage 1: chunk order and length sort at the automatic tile size
        const int spans[] = {16, 64, 256, 1024};
        for (int srt = 0; srt < 2 && !st; ++srt)
            for (int sp : spans) {
                rmc_options o = base;
                o.xcd_span = sp;
                o.length_sort = srt;
                o.alloc_tile = 0;
                if ((st = time_candidate(o))) break;
            }
        // stage 2: the tile size at the best schedule of stage 1
        const int t0 = auto_tile_cells(total_ncpad);
        for (int t : {t0 / 2 / 64 * 64, 2 * t0}) {
            if (st) break;
            if (t < 256 || t > 16384) continue;
            rmc_options o = best;
            o.alloc_tile = t;
            st = time_candidate(o);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c->opt = base;
        if (st) return st;
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (!f) return fail(RMC_INVALID_ARG, "cannot append to the autotuning cache %s", cache_path);
            fprintf(f, "%s : %d %d %d\n", sig.c_str(), best.xcd_span, best.length_sort, best.alloc_tile);
            fclose(f);
        }
        for (int q = 0; q < nsnap; ++q)
            if ((st = rmc_reset_stats(ctxs[q]))) return st;
    }
    for (int q = 0; q < nsnap; ++q) {   // schedule knobs only: snapshot ids stay per context
        rmc_options &o = ctxs[q]->opt;
        o.xcd_span = best.xcd_span;
        o.length_sort = best.length_sort;
        o.alloc_tile = best.alloc_tile;
        ++ctxs[q]->config_version;
    }
    if (out) *out = c->opt;
    return RMC_OK;
}

rmc_status rmc_autotune(rmc_ctx *c, int reps, const char *cache_path, rmc_options *out, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    rmc_ctx *cs[1] = {c};
    return rmc_autotune_batch(cs, 1, reps, cache_path, out, stream);
}

rmc_status rmc_set_cell_pdf(rmc_ctx *c, const double *q, rmc_mem mem, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!c->have_grid || !c->have_kdist) return fail(RMC_BAD_STATE, "set_grid and set_kdist must come first");
    if (!q) return fail(RMC_INVALID_ARG, "null pdf pointer");
    const uint64_t n = ncells_of(c) * (uint64_t)c->nb * c->ng * 8;
    if (n > (1ull << 27)) return fail(RMC_UNSUPPORTED, "per-cell pdf larger than 2^27 entries");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    rmc_status st;
    if ((st = c->q.ensure(sizeof(double) * n))) return st;
    HIPCHK(hipMemcpyAsync(c->q.p, q, sizeof(double) * n,
                          mem == RMC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, (hipStream_t)stream));
    c->have_q = true;
    return RMC_OK;
}

rmc_status rmc_compute_batch(rmc_ctx *const *ctxs, int nsnap, double *const *divq, double *const *se, rmc_mem mem,
                             void *stream)
{
    g_err.clear();
    if (!divq) return fail(RMC_INVALID_ARG, "null outputs");
    if (mem != RMC_HOST && mem != RMC_DEVICE) return fail(RMC_INVALID_ARG, "bad memory kind");
    if (rmc_status st = check_batch(ctxs, nsnap)) return st;
    for (int q = 0; q < nsnap; ++q)
        if (!divq[q]) return fail(RMC_INVALID_ARG, "null output in the batch");
    rmc_ctx *L = ctxs[0];
    DeviceGuard g(L->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", L->device);
    hipStream_t s = (hipStream_t)stream;
    if (L->opt.march == RMC_F64) return run_pipeline<double>(ctxs, nsnap, divq, se, mem, s);
    return run_pipeline<float>(ctxs, nsnap, divq, se, mem, s);
}

rmc_status rmc_compute_divergence(rmc_ctx *c, double *divq, double *se, rmc_mem mem, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!divq) return fail(RMC_INVALID_ARG, "null output");
    rmc_ctx *cs[1] = {c};
    double *d[1] = {divq};
    double *e[1] = {se};
    return rmc_compute_batch(cs, 1, d, e, mem, stream);
}

rmc_status rmc_compute_divergence_noalloc(rmc_ctx *c, double *divq, double *se, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!divq) return fail(RMC_INVALID_ARG, "null output");
    if (c->opt.sampling != RMC_SAMPLING_PLAIN)
        return fail(RMC_UNSUPPORTED, "the allocation-free compute runs the plain (T_max) sampling only");
    rmc_ctx *cs[1] = {c};
    if (rmc_status st = check_batch(cs, 1)) return st;
    if (c->device >= kMaxDevices) return fail(RMC_UNSUPPORTED, "device index above %d", kMaxDevices - 1);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[c->device];
        if (!base)
            return fail(RMC_DEVICE_ERROR, "no scratch address on device %d: %s", c->device,
                        hipGetErrorString(g_scratch_err[c->device]));
    }
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    const bool dbl = c->opt.march == RMC_F64;
    // every buffer the compute sizes is carved from the scratch; the context's own buffers and
    // the state describing them (slot layout of the last compute) are put back afterwards
    const int slots_R = c->slots_R, slots_real = c->slots_real, rw_log2 = c->rec_rw_log2;
    Arena A;
    A.base = static_cast<unsigned char *>(base);
    A.cap = kScratchBytes;
    t_arena = &A;
    Plan P;
    rmc_status st = dbl ? plan_pipeline<double>(cs, 1, P, s) : plan_pipeline<float>(cs, 1, P, s);
    if (!st) {
        double *d[1] = {divq};
        double *e[1] = {se};
        st = dbl ? enqueue_pipeline<double>(P, d, e, s, nullptr) : enqueue_pipeline<float>(P, d, e, s, nullptr);
    }
    t_arena = nullptr;
    A.restore();
    c->slots_R = slots_R;
    c->slots_real = slots_real;
    c->rec_rw_log2 = rw_log2;
    return st;
}

rmc_status rmc_compute_wall_flux(rmc_ctx *c, double *divq, double *se, double *q_wall, rmc_mem mem, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!divq || !q_wall) return fail(RMC_INVALID_ARG, "null output");
    if (mem != RMC_HOST && mem != RMC_DEVICE) return fail(RMC_INVALID_ARG, "bad memory kind");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    const size_t nw = 2 * ((size_t)c->ny * c->nz + (size_t)c->nx * c->nz + (size_t)c->nx * c->ny);
    double *dev = q_wall;
    if (mem == RMC_HOST) {
        if (rmc_status st = c->wallbuf.ensure(sizeof(double) * nw)) return st;
        dev = c->wallbuf.as<double>();
    }
    c->wall_dev = dev;
    const rmc_status st = rmc_compute_divergence(c, divq, se, mem, stream);
    c->wall_dev = nullptr;
    if (st) return st;
    if (mem == RMC_HOST)
        HIPCHK(hipMemcpyAsync(q_wall, dev, sizeof(double) * nw, hipMemcpyDeviceToHost, (hipStream_t)stream));
    return RMC_OK;
}

rmc_status rmc_graph_capture(rmc_ctx *const *ctxs, int nsnap, double *const *divq, double *const *se, void *stream,
                             rmc_graph **out)
{
    g_err.clear();
    if (!out) return fail(RMC_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (!divq) return fail(RMC_INVALID_ARG, "null outputs");
    if (!stream) return fail(RMC_INVALID_ARG, "graph capture needs a stream other than the null stream");
    if (rmc_status st = check_batch(ctxs, nsnap)) return st;
    for (int q = 0; q < nsnap; ++q)
        if (ctxs[q]->opt.sampling == RMC_SAMPLING_LEARNED && ctxs[q]->opt.alloc_cache)
            return fail(RMC_UNSUPPORTED, "alloc_cache cannot be captured (a replay cannot tell whether the field changed)");
    for (int q = 0; q < nsnap; ++q)
        if (!divq[q]) return fail(RMC_INVALID_ARG, "null output in the batch");
    rmc_ctx *L = ctxs[0];
    DeviceGuard g(L->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", L->device);
    hipStream_t s = (hipStream_t)stream;
    const bool dbl = L->opt.march == RMC_F64;
    Plan P;
    rmc_status st = dbl ? plan_pipeline<double>(ctxs, nsnap, P, s) : plan_pipeline<float>(ctxs, nsnap, P, s);
    if (st) return st;
    rmc_graph *G = new (std::nothrow) rmc_graph();
    if (!G) return fail(RMC_OUT_OF_MEMORY, "graph allocation failed");
    {   // the graph reads its own copies of the planned tables
        const size_t nb_ = (size_t)L->nb * L->ng;
        const size_t sz[6] = {sizeof(double) * P.nfaces, sizeof(SnapDesc) * nsnap, sizeof(TileInfo) * P.ntiles,
                              sizeof(uint32_t) * nb_ * 8, sizeof(float) * 2 * nb_, sizeof(uint32_t) * (P.nregion + 1)};
        DBuf *dst[6] = {&G->faces, &G->snaps, &G->tile_info, &G->border, &G->kmin, &G->rtile0};
        const void *src[6] = {P.d_faces, P.d_snaps, P.d_tiles, P.d_border, P.d_kmin, P.d_rtile0};
        for (int u = 0; u < 6; ++u) {
            if ((st = dst[u]->ensure(sz[u]))) { delete G; return st; }
            if (hipMemcpyAsync(dst[u]->p, src[u], sz[u], hipMemcpyDeviceToDevice, s) != hipSuccess) {
                delete G;
                return fail(RMC_DEVICE_ERROR, "copy of the planned tables failed");
            }
        }
        P.d_faces = G->faces.as<double>();
        P.d_snaps = G->snaps.as<SnapDesc>();
        P.d_tiles = G->tile_info.as<TileInfo>();
        P.d_border = G->border.as<uint32_t>();
        P.d_kmin = G->kmin.as<float>();
        P.d_rtile0 = G->rtile0.as<uint32_t>();
    }
    if (hipStreamSynchronize(s) != hipSuccess) { delete G; return fail(RMC_DEVICE_ERROR, "hipStreamSynchronize failed"); }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete G;
        return fail(RMC_DEVICE_ERROR, "hipStreamBeginCapture failed");
    }
    st = dbl ? enqueue_pipeline<double>(P, divq, se, s, nullptr) : enqueue_pipeline<float>(P, divq, se, s, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (st || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        delete G;
        if (st) return st;
        return fail(RMC_DEVICE_ERROR, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        delete G;
        return fail(RMC_DEVICE_ERROR, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    }
    G->device = L->device;
    G->ctxs.assign(ctxs, ctxs + nsnap);
    for (rmc_ctx *c : G->ctxs) {
        G->versions.push_back(c->config_version);
        G->ptrs.push_back(buffer_ptrs(c));
        ++c->graphs;
    }
    G->graph = graph;
    G->exec = exec;
    *out = G;
    return RMC_OK;
}

rmc_status rmc_graph_launch(rmc_graph *G, void *stream)
{
    g_err.clear();
    if (!G || !G->exec) return fail(RMC_INVALID_ARG, "null graph");
    for (size_t q = 0; q < G->ctxs.size(); ++q) {
        const rmc_ctx *c = G->ctxs[q];
        if (c->config_version != G->versions[q] || buffer_ptrs(c) != G->ptrs[q] || !c->have_T || !c->have_X)
            return fail(RMC_BAD_STATE, "a captured context changed since the capture; capture again");
    }
    DeviceGuard g(G->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", G->device);
    HIPCHK(hipGraphLaunch(G->exec, (hipStream_t)stream));
    return RMC_OK;
}

void rmc_graph_destroy(rmc_graph *G)
{
    if (!G) return;
    for (rmc_ctx *c : G->ctxs) --c->graphs;
    DeviceGuard g(G->device);
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;   // its table copies are released with the device current
}

rmc_status rmc_get_ray_values(rmc_ctx *c, const int64_t *cells, int ncell, double *Y, int32_t *steps, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!cells || ncell < 0 || !Y) return fail(RMC_INVALID_ARG, "bad arguments");
    if (!c->slots_R) return fail(RMC_BAD_STATE, "no compute has run");
    const uint64_t nc = ncells_of(c);
    for (int q = 0; q < ncell; ++q)
        if (cells[q] < 0 || (uint64_t)cells[q] >= nc) return fail(RMC_INVALID_ARG, "cell index out of range");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    const int R = c->slots_R;
    std::vector<uint64_t> tmp(R);
    std::vector<uint32_t> st(R);
    for (int q = 0; q < ncell; ++q) {
        const size_t off = (size_t)cells[q] * R;
        HIPCHK(hipMemcpy(tmp.data(), c->Y.as<uint64_t>() + off, sizeof(uint64_t) * R, hipMemcpyDeviceToHost));
        if (c->slots_real == 8)
            HIPCHK(hipMemcpy(st.data(), c->st.as<uint32_t>() + off, sizeof(uint32_t) * R, hipMemcpyDeviceToHost));
        for (int r = 0; r < R; ++r) {
            double y;
            uint32_t w;
            if (c->slots_real == 4) {   // {value bits, steps | end << 28}
                float f;
                const uint32_t lo = (uint32_t)tmp[r];
                memcpy(&f, &lo, 4);
                y = (double)f;
                w = (uint32_t)(tmp[r] >> 32);
            } else {
                memcpy(&y, &tmp[r], 8);
                w = st[r];
            }
            Y[(size_t)q * R + r] = y;
            if (steps) steps[(size_t)q * R + r] = (int32_t)(w & 0x0FFFFFFFu);
        }
    }
    return RMC_OK;
}

rmc_status rmc_trace_cells(rmc_ctx *c, const int64_t *cells, int ncell, rmc_ray_record *out, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!cells || ncell < 0 || !out) return fail(RMC_INVALID_ARG, "bad arguments");
    if (rmc_status st = check_ready(c)) return st;
    const uint64_t nc = ncells_of(c);
    for (int q = 0; q < ncell; ++q)
        if (cells[q] < 0 || (uint64_t)cells[q] >= nc) return fail(RMC_INVALID_ARG, "cell index out of range");
    if (ncell == 0) return RMC_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    const int R = c->opt.rays_per_cell;
    const bool dbl = c->opt.march == RMC_F64;
    const int smode = (int)c->opt.sampling;
    SnapDesc D;
    rmc_status st = dbl ? plan_snapshot<double>(c, D) : plan_snapshot<float>(c, D);
    if (st) return st;
    const bool inc_xz = D.hx > 0.0 && D.hz > 0.0 && !D.closed;
    std::vector<double> &fd = c->h_faces;
    fd.clear();
    std::vector<std::pair<int, int>> fblocks;
    append_faces(c, D, fd, fblocks);
    const int nfaces = (int)fd.size();
    const size_t nrec = (size_t)ncell * R;
    if ((st = c->faces.ensure(sizeof(double) * nfaces)) || (st = c->snaps.ensure(sizeof(SnapDesc))) ||
        (st = c->trace_cells.ensure(sizeof(int64_t) * ncell)) ||
        (st = c->trace_rec.ensure(sizeof(rmc_ray_record) * nrec)))
        return st;
    if ((size_t)nfaces * 8 > march_lds_budget(c))
        return fail(RMC_UNSUPPORTED, "face tables exceed %d KiB of LDS", (int)(march_lds_budget(c) / 1024));
    HIPCHK(hipMemcpyAsync(c->faces.p, fd.data(), (size_t)nfaces * 8, hipMemcpyHostToDevice, s));
    if ((st = dbl ? enqueue_snapshot<double>(c, D, c->faces.as<double>(), s)
                  : enqueue_snapshot<float>(c, D, c->faces.as<double>(), s)))
        return st;
    HIPCHK(hipMemcpyAsync(c->snaps.p, &D, sizeof(SnapDesc), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->trace_cells.p, cells, sizeof(int64_t) * ncell, hipMemcpyHostToDevice, s));
    const unsigned blocks = (unsigned)((nrec + 255) / 256);
    const uint32_t k0 = (uint32_t)c->opt.seed, k1 = (uint32_t)(c->opt.seed >> 32);
    if (dbl) {
        TraceArgs<double> A{c->snaps.as<SnapDesc>(), c->faces.as<double>(), nfaces, c->trace_cells.as<int64_t>(),
                            ncell, c->dnu.as<double>(), c->wg.as<double>(), c->nb, c->ng, R, k0, k1,
                            c->opt.tol, c->opt.max_steps, c->trace_rec.as<rmc_ray_record>(),
                            c->Ib.as<double>(), c->k32.as<float>(), c->nT, c->ns};
        if (smode == 2) hipLaunchKernelGGL((k_trace<double, 2, false>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
        else if (smode == 1) hipLaunchKernelGGL((k_trace<double, 1, false>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
        else hipLaunchKernelGGL((k_trace<double, 0, false>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
    } else {
        TraceArgs<float> A{c->snaps.as<SnapDesc>(), c->faces.as<double>(), nfaces, c->trace_cells.as<int64_t>(),
                           ncell, c->dnu.as<double>(), c->wg.as<double>(), c->nb, c->ng, R, k0, k1,
                           (float)c->opt.tol, c->opt.max_steps, c->trace_rec.as<rmc_ray_record>(),
                           c->Ib.as<double>(), c->k32.as<float>(), c->nT, c->ns};
        if (inc_xz) {
            if (smode == 2) hipLaunchKernelGGL((k_trace<float, 2, true>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
            else if (smode == 1) hipLaunchKernelGGL((k_trace<float, 1, true>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
            else hipLaunchKernelGGL((k_trace<float, 0, true>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
        } else {
            if (smode == 2) hipLaunchKernelGGL((k_trace<float, 2, false>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
            else if (smode == 1) hipLaunchKernelGGL((k_trace<float, 1, false>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
            else hipLaunchKernelGGL((k_trace<float, 0, false>), dim3(blocks), dim3(256), 8 * nfaces, s, A);
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, c->trace_rec.p, sizeof(rmc_ray_record) * nrec, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return RMC_OK;
}

rmc_status rmc_get_pdf(rmc_ctx *c, double *p, double *cdf_b, double *cdf_g, double *T_max, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!c->p.p) return fail(RMC_BAD_STATE, "no compute has run");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    int status = 0;
    HIPCHK(hipMemcpy(&status, c->status.p, sizeof(int), hipMemcpyDeviceToHost));
    if (status) return fail(RMC_INVALID_ARG, "the spectral pdf has zero total emission at T_max");
    if (p) HIPCHK(hipMemcpy(p, c->p.p, sizeof(double) * c->nb * c->ng, hipMemcpyDeviceToHost));
    if (cdf_b) HIPCHK(hipMemcpy(cdf_b, c->cdf_b.p, sizeof(double) * c->nb, hipMemcpyDeviceToHost));
    if (cdf_g) HIPCHK(hipMemcpy(cdf_g, c->cdf_g.p, sizeof(double) * c->nb * c->ng, hipMemcpyDeviceToHost));
    if (T_max) *T_max = std::max(c->Tmax_cells, walls_Tmax(c));
    return RMC_OK;
}

rmc_status rmc_get_stats(rmc_ctx *c, rmc_stats *out)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (!out) return fail(RMC_INVALID_ARG, "null output");
    if (c->last_set < 0) return fail(RMC_BAD_STATE, "no compute has run");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    if (rmc_status st = harvest_all(c)) return st;
    unsigned long long cnt[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpy(cnt, c->counters.p, sizeof cnt, hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    out->rays = c->last_rays;
    out->steps = (int64_t)cnt[0];
    out->capped_rays = (int64_t)cnt[1];
    out->ms_prep = c->last_ms[0];
    out->ms_alloc = c->last_ms[1];
    out->ms_march = c->last_ms[2] + c->last_ms[3];
    out->ms_reduce = c->last_ms[4];
    out->ms_total = c->last_ms[0] + c->last_ms[1] + c->last_ms[2] + c->last_ms[3] + c->last_ms[4];
    out->long_steps = (int64_t)cnt[3];
    out->ms_march_lane = c->last_ms[2];
    out->sum_ms_march_lane = c->sum_ms[2];
    out->computes = c->n_computes;
    out->sum_rays = c->sum_rays;
    out->sum_steps = (int64_t)cnt[2];
    out->sum_ms_prep = c->sum_ms[0];
    out->sum_ms_alloc = c->sum_ms[1];
    out->sum_ms_march = c->sum_ms[2] + c->sum_ms[3];
    out->sum_ms_reduce = c->sum_ms[4];
    return RMC_OK;
}

rmc_status rmc_gather_probe(rmc_ctx *c, int steps, double *ms, double *bytes, void *stream)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    if (steps < 1 || steps > 65536 || !ms || !bytes) return fail(RMC_INVALID_ARG, "bad arguments");
    if (!c->rec.p || c->slots_real != 4 || c->slots_R < 1)
        return fail(RMC_BAD_STATE, "the probe reads the cell records of a previous compute with the FP32 march");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    hipStream_t s = (hipStream_t)stream;
    SnapDesc D{};
    D.nx = c->nx; D.ny = c->ny; D.nz = c->nz;
    D.nbx = round_up(c->nx, 4) / 4; D.nby = round_up(c->ny, 4) / 4; D.nbz = round_up(c->nz, 4) / 4;
    D.ncpad = ncpad_of(c);
    D.rec = c->rec.as<uint4>();
    D.rw_log2 = c->rec_rw_log2;
    const uint64_t lanes = ncells_of(c) * (uint64_t)c->slots_R;
    const uint32_t nchunks = (uint32_t)((lanes + 63) / 64);
    int span_log2 = 0;
    for (int sp = c->opt.xcd_span > 0 ? c->opt.xcd_span : 256; sp > 1; sp >>= 1) ++span_log2;
    rmc_status st;
    if ((st = c->probe.ensure(sizeof(double) * nchunks))) return st;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)xcd_blocks(nchunks, span_log2)), dim3(256), 0, s, D,
                       c->nb * c->ng, steps, nchunks, span_log2, c->probe.as<double>());
    const hipError_t le = hipGetLastError();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(le);
    *ms = t;
    *bytes = (double)lanes * steps * sizeof(uint4) + (double)nchunks * sizeof(double);
    return RMC_OK;
}

rmc_status rmc_reset_stats(rmc_ctx *c)
{
    g_err.clear();
    if (rmc_status st = check_ctx(c)) return st;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(RMC_DEVICE_ERROR, "hipSetDevice(%d) failed", c->device);
    if (rmc_status st = harvest_all(c)) return st;
    c->n_computes = 0;
    c->sum_rays = 0;
    for (double &v : c->sum_ms) v = 0.0;
    if (c->have_counters) {
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemset(c->counters.as<unsigned long long>() + 2, 0, sizeof(unsigned long long)));
    }
    return RMC_OK;
}

}  // extern "C"

#include "learn_api.inc"
