// rmc_device.h -- device building blocks of the gfx950 ERMC solver: counter-based random
// numbers, ray initialisation and the face-to-face march (Algorithm 1 of Silvestri &
// Pecnik).  Included once, by rmc.hip.
//
// The whole translation unit is compiled with -ffp-contract=off: every a*b+c below rounds
// twice unless an fma is written out, which keeps the FP64 path on the operation order the
// paper's algorithm states.  The float march writes its fused multiply-adds explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmc {

constexpr uint32_t kTagAlloc = 1u;      // random stream of the (band, g, octant) draws
constexpr uint32_t kTagDir = 2u;        // random stream of the direction draws
constexpr uint32_t kInvalidItem = 0xFFFFFFFFu;
constexpr int kEndTol = 0, kEndWallLo = 1, kEndWallHi = 2, kEndCap = 3;   // y walls, step cap
// Walls, in the order their terms are taken (x, y, z; low side first): bit / index w of a
// wall mask, and the end code of a ray that a black wall w stops.
constexpr int kWallX0 = 0, kWallX1 = 1, kWallY0 = 2, kWallY1 = 3, kWallZ0 = 4, kWallZ1 = 5;
__device__ __forceinline__ int wall_end_code(int w) { return w < 2 ? 4 + w : (w < 4 ? w - 1 : w + 2); }
// ...and back: the wall (x0, x1, y0, y1, z0, z1) a ray ended on, -1 if it did not end on a wall
__device__ __forceinline__ int wall_of_end(int end)
{
    return end == 1 || end == 2 ? end + 1 : (end == 4 || end == 5 ? end - 4 : (end == 6 || end == 7 ? end - 2 : -1));
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each two 32x32->64 bit products of
// counter words with fixed multipliers, xor-mixed with the other words and the round key;
// the key is bumped by two Weyl constants after every round.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        // each product as one 32x32->64 multiply (one instruction, not a low and a high half)
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u, p1 = (uint64_t)c2 * 0xCD9E8D57u;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Load through a global-memory pointer.  Pointers read from descriptors are generic to the
// compiler; without the address space the loads become flat loads, which wait on the LDS
// counter as well and serialise the march.
template <class T> __device__ __forceinline__ T gld(const T *p)
{
    typedef const __attribute__((address_space(1))) T gT;
    return *(gT *)(p);
}

__device__ __forceinline__ uint4 gld(const uint4 *p)
{
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) v4u gv4u;
    const v4u v = *(gv4u *)(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint2 gld(const uint2 *p)
{
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) v2u gv2u;
    const v2u v = *(gv2u *)(p);
    return make_uint2(v.x, v.y);
}

__device__ __forceinline__ float4 gld(const float4 *p)
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) v4f gv4f;
    const v4f v = *(gv4f *)(p);
    return make_float4(v.x, v.y, v.z, v.w);
}

// Spectral / octant variate: all 32 bits, (w + 1/2) 2^-32, exact in double, in (0, 1).
__device__ __forceinline__ double unif_alloc(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// Direction variate: top 23 bits, ((w >> 9) + 1/2) 2^-23, exact in float and double.
template <class Real> __device__ __forceinline__ Real unif_dir(uint32_t w)
{
    return ((Real)(w >> 9) + (Real)0.5) * (Real)0x1p-23;
}

// First index i < n with u < cdf[i] (cdf non-decreasing, cdf[n-1] = 1 > u).  Inversion of
// the discrete spectral cdf (Sec. 2.1) by bisection; same answer as a linear scan.
__device__ __forceinline__ int cdf_search(const double *__restrict__ cdf, int n, double u)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Store through a global-memory pointer (a generic store also waits on the LDS counter).
template <class T> __device__ __forceinline__ void gst(T *p, T v)
{
    typedef __attribute__((address_space(1))) T gT;
    *(gT *)(p) = v;
}

// The same index as cdf_search for a cdf non-decreasing over [0, n - 2] (cumulative sums are):
// the count of cdf[0 .. n-2] at or below u.  For a table in global memory: the loads are
// independent, so their latencies overlap instead of adding up along a bisection.
__device__ __forceinline__ int cdf_rank(const double *cdf, int n, double u)
{
    int c = 0;
    for (int m0 = 0; m0 < n - 1; m0 += 16) {
        double v[16];   // sixteen loads at a time, the index clamped into the table
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = gld(cdf + min(m0 + q, n - 2));
#pragma unroll
        for (int q = 0; q < 16; ++q) c += (m0 + q < n - 1 && v[q] <= u) ? 1 : 0;
    }
    return c;
}

// Isotropic direction inside octant o (bit 0: -x, bit 1: -y, bit 2: -z): mu = cos(theta) =
// 1 - 2 R_theta about the y axis, phi = 2 pi R_phi (inversion of Eq. 9).  Double precision in
// both march precisions: it is done once per ray and fixes the path geometry.
__device__ __forceinline__ void octant_direction(uint32_t w0, uint32_t w1, int o, double &dx, double &dy,
                                                 double &dz)
{
    const double mu = 1.0 - 2.0 * unif_dir<double>(w0);
    const double phi = 2.0 * M_PI * unif_dir<double>(w1);
    const double s = sqrt((1.0 - mu) * (1.0 + mu));
    double sn, cs;
    sincos(phi, &sn, &cs);
    dx = fabs(s * cs);
    dy = fabs(mu);
    dz = fabs(s * sn);
    if (o & 1) dx = -dx;
    if (o & 2) dy = -dy;
    if (o & 4) dz = -dz;
}

// Bricked layout of the property fields: 4x4x4 bricks in raster order (bk fastest), Morton
// order inside a brick (bits i1 j1 k1 i0 j0 k0).  The offset is a sum of per-axis terms.
__device__ __forceinline__ int brick_x(int i, int sx_) { return __mul24(i >> 2, sx_) + ((i & 1) << 2) + ((i & 2) << 4); }
__device__ __forceinline__ int brick_y(int j, int sy_) { return __mul24(j >> 2, sy_) + ((j & 1) << 1) + ((j & 2) << 3); }
__device__ __forceinline__ int brick_z(int k) { return ((k >> 2) << 6) + (k & 1) + ((k & 2) << 2); }

// Properties of the cells a ray crosses (Sec. 2.2: linear interpolation of the tables in T,
// mixture kappa = sum_s x_s k^s).  The march reads one record per cell: the table coordinate
// u = (T - T0) / dT of the cell's temperature (FP64) and its mole fractions (march precision),
// in 16-byte words, 2^rw_log2 words per cell, bricked layout.  The record does not depend on
// the band or g-point, so every (band, g) pair reads the same field; kappa_{n,g} and I_n are
// interpolated from the ray's tables (I_n FP64, k^s FP32-exact values) with the FP64
// operations of the reference and rounded to march precision for kappa.
template <class Real> struct Props {
    const uint4 *rec;           // records of the grid level
    const double *ib;           // I_n at the table nodes [nT]
    const float *k;             // k^s_{n,g} at the table nodes: species s at k + s * kstride
    int kstride;
    int ns;
    int tmax;                   // nT - 2: the last interval of the table
    int rw_log2;                // record words per cell, log2
};

template <class Real> __device__ __forceinline__ uint4 prop_fetch(const Props<Real> &P, int cell)
{
    return gld(P.rec + ((size_t)(uint32_t)cell << P.rw_log2));
}

__device__ __forceinline__ double lerp_node(const float *tab, int t, double f)
{
    const double a = (double)tab[t], b = (double)tab[t + 1];
    return a + f * (b - a);
}

// kappa_{n,g} and I_n of a cell from its record v (first word; further words read here).  I_n
// is interpolated in FP64 in both precisions (the ray sums differences of intensities of
// near-isothermal cells).  The FP64 march interpolates kappa with the reference's FP64
// operations; the FP32 march interpolates the FP32-exact table values in FP32 (a few ulp of
// kappa, far below its parity bar) at a third of the instructions.
template <class Real>
__device__ __forceinline__ void prop_eval(const Props<Real> &P, uint4 v, int cell, Real &kap, double &I)
{
    const double u = __hiloint2double((int)v.y, (int)v.x);
    int t = (int)u;             // u >= 0: temperatures are checked against the table range
    t = t > P.tmax ? P.tmax : t;
    const double f = u - (double)t;
    const double i0 = P.ib[t], i1 = P.ib[t + 1];
    if constexpr (sizeof(Real) == 4) {
        I = fma(f, i1 - i0, i0);
        const float ff = (float)f;
        const float *k0 = P.k + t;
        float kp = __uint_as_float(v.z) * fmaf(ff, k0[1] - k0[0], k0[0]);
        if (P.ns > 1) {
            const float *k1 = k0 + P.kstride;
            kp = fmaf(__uint_as_float(v.w), fmaf(ff, k1[1] - k1[0], k1[0]), kp);
        }
#pragma unroll 1
        for (int s = 2; s < P.ns; ++s) {   // words 1.. hold four fractions each
            const float *xw = reinterpret_cast<const float *>(P.rec + ((size_t)(uint32_t)cell << P.rw_log2) + 1);
            const float *ks = k0 + s * P.kstride;
            kp = fmaf(gld(xw + (s - 2)), fmaf(ff, ks[1] - ks[0], ks[0]), kp);
        }
        kap = kp;
    } else {
        I = i0 + f * (i1 - i0);
        double kp = __hiloint2double((int)v.w, (int)v.z) * lerp_node(P.k, t, f);
#pragma unroll 1
        for (int s = 1; s < P.ns; ++s) {   // words 1.. hold two fractions each
            const double *xw = reinterpret_cast<const double *>(P.rec + ((size_t)(uint32_t)cell << P.rw_log2) + 1);
            kp += gld(xw + (s - 1)) * lerp_node(P.k + s * P.kstride, t, f);
        }
        kap = kp;
    }
}

template <class Real> __device__ __forceinline__ void prop_load(const Props<Real> &P, int cell, Real &kap, double &I)
{
    prop_eval(P, prop_fetch(P, cell), cell, kap, I);
}

// Geometry of one snapshot as seen by a ray.
struct RayGeo {
    const double *xf, *yf, *zf; // face coordinates (LDS), nx+1, ny+1, nz+1
    int nx, ny, nz;
    int bsx, bsy;               // brick strides of the x and y brick index (in cells)
    double Lx, Lz;              // periodic lengths
    bool closed;                // walls on x and z too (else x and z are periodic)
    bool reflect;               // some wall has emissivity below one: rays reflect
};

// Walls seen by the rays of one band: wall w has the band's intensity I[w * stride] and the
// emissivity eps[w].
struct Walls {
    const double *I;
    int stride;
    const double *eps;
};

// FP32 cell absorption: alpha = 1 - exp(-x) and the transmission factor exp(-x) of a
// segment with optical thickness x = kappa ds (Eqs. 2-3).  The transmission is the
// exponential itself (relative accuracy at any x, so tau stays accurate behind optically
// thick cells); alpha is 1 - exp(-x) for x >= 1/4 and the Taylor series of 1 - exp(-x)
// through x^7 below (truncation < 2e-9 relative), which avoids the cancellation.
__device__ __forceinline__ void absorb_f32(float x, float &a, float &e)
{
    e = __expf(-x);
    float p = fmaf(x, -1.0f / 5040.0f, 1.0f / 720.0f);
    p = fmaf(x, -p, 1.0f / 120.0f);
    p = fmaf(x, -p, 1.0f / 24.0f);
    p = fmaf(x, -p, 1.0f / 6.0f);
    p = fmaf(x, -p, 0.5f);
    p = fmaf(x, -p, 1.0f);
    a = x < 0.25f ? x * p : 1.0f - e;
}

// One ray of the march (Algorithm 1, March).
//
// Per step: ds = distance to the nearest face, alpha = 1 - exp(-kappa ds) (Eq. 2),
// acc += tau alpha (I_src - I_cell), tau *= 1 - alpha (Eq. 3); every axis whose face is
// reached steps; x and z wrap, leaving y hits a black wall (alpha = 1, I = I_b(T_wall)).
// The ray stops at tau <= tol or after max_steps and adds the residual tau (I_src - I_last).
//
// The path geometry (face parameters t, segment lengths) and intensity differences are
// double in both precisions, and so are tau and the accumulated sum (MI355X runs FP64
// add/mul/fma at the rate of unpacked FP32; rays of thousands of steps would otherwise lose
// 1e-5 to rounding).  Real sets the arithmetic of kappa and alpha: FP64 follows the reference
// operation by operation (divisions, expm1, tau *= 1 - alpha); FP32 evaluates alpha and the
// transmission in float (absorb_f32), uses one reciprocal per axis, and with INC_XZ advances
// the uniform periodic axes by a constant parameter increment instead of re-reading face
// coordinates.
//
// A step is split into its geometry (which cell comes next) and its absorption (physics of
// the current cell), so that the next cell's record is requested before the current cell's
// physics runs; the march loop is unrolled twice with two register sets, so a load is always
// in flight while the other set is consumed.
template <class Real, bool INC_XZ> struct Ray {
    double tx, ty, tz, t;       // next-face parameters per axis, current parameter
    double ox, oy, oz;          // origin (cell centre)
    double rx, ry, rz;          // 1 / direction (FP32 path) or the direction (FP64 path)
    double dtx, dtz;            // INC_XZ: parameter increment per x / z cell
    double Isrc;                // source intensity
    double tau, acc;
    int i, j, k, wi, wk;        // current cell (x, z local index and wrap count)
    int px, py, pz;             // brick offsets of the current cell
    int sgn;                    // bit 0/1/2: x/y/z direction negative
    int stx, stz, wx, wz;       // INC_XZ: x / z step (+-1) and the index a step past the edge wraps to
    int steps, end;
};

struct XzUniform {
    double hx, hz;              // uniform cell widths along x and z (INC_XZ)
};

// Starts the ray at the centre of cell (ci, cj, ck); returns the source cell's kappa and I.
template <class Real, bool INC_XZ>
__device__ __forceinline__ void ray_init(Ray<Real, INC_XZ> &R, const RayGeo &G, const XzUniform &U,
                                         const Props<Real> &P, int ci, int cj, int ck, double dx, double dy,
                                         double dz, Real &kc, double &Ic)
{
    R.ox = 0.5 * (G.xf[ci] + G.xf[ci + 1]);
    R.oy = 0.5 * (G.yf[cj] + G.yf[cj + 1]);
    R.oz = 0.5 * (G.zf[ck] + G.zf[ck + 1]);
    R.sgn = (dx > 0.0 ? 0 : 1) | (dy > 0.0 ? 0 : 2) | (dz > 0.0 ? 0 : 4);
    if constexpr (sizeof(Real) == 4 && INC_XZ) {
        R.stx = dx > 0.0 ? 1 : -1;
        R.stz = dz > 0.0 ? 1 : -1;
        R.wx = R.stx > 0 ? 0 : G.nx - 1;
        R.wz = R.stz > 0 ? 0 : G.nz - 1;
    }
    if constexpr (sizeof(Real) == 8) {
        R.rx = dx; R.ry = dy; R.rz = dz;
        R.tx = (G.xf[ci + (dx > 0.0)] - R.ox) / dx;
        R.ty = (G.yf[cj + (dy > 0.0)] - R.oy) / dy;
        R.tz = (G.zf[ck + (dz > 0.0)] - R.oz) / dz;
    } else {
        R.rx = 1.0 / dx; R.ry = 1.0 / dy; R.rz = 1.0 / dz;
        R.tx = (G.xf[ci + (dx > 0.0)] - R.ox) * R.rx;
        R.ty = (G.yf[cj + (dy > 0.0)] - R.oy) * R.ry;
        R.tz = (G.zf[ck + (dz > 0.0)] - R.oz) * R.rz;
        if constexpr (INC_XZ) {
            R.dtx = U.hx * fabs(R.rx);
            R.dtz = U.hz * fabs(R.rz);
        }
    }
    R.i = ci; R.j = cj; R.k = ck; R.wi = 0; R.wk = 0;
    R.px = brick_x(ci, G.bsx); R.py = brick_y(cj, G.bsy); R.pz = brick_z(ck);
    prop_load(P, R.px + R.py + R.pz, kc, R.Isrc);
    Ic = R.Isrc;
    R.t = 0.0;
    R.tau = 1.0;
    R.acc = 0.0;
    R.steps = 0;
    R.end = kEndTol;
}

// Whether the march loop runs at all (tau = 1 must exceed tol, max_steps >= 1).
template <class Real> __device__ __forceinline__ bool march_starts(Real tol, int max_steps)
{
    return (Real)1 > tol && max_steps > 0;
}

// Specular reflection on wall `side` (0 low, 1 high) of the y axis: the ray goes on from the
// point it hit, in the wall cell, with origin and direction mirrored on the wall plane (its
// parameter t continues).  Same for x and z (closed box; there the wrap count is zero).
template <class Real, bool INC_XZ>
__device__ __forceinline__ void reflect_y(Ray<Real, INC_XZ> &R, const RayGeo &G, int side)
{
    R.j = side ? G.ny - 1 : 0;
    R.oy = 2.0 * G.yf[side ? G.ny : 0] - R.oy;
    R.ry = -R.ry;
    R.sgn ^= 2;
    const double f = G.yf[R.j + 1 - ((R.sgn >> 1) & 1)] - R.oy;
    if constexpr (sizeof(Real) == 4) R.ty = f * R.ry;
    else R.ty = f / R.ry;
}

template <class Real, bool INC_XZ>
__device__ __forceinline__ void reflect_x(Ray<Real, INC_XZ> &R, const RayGeo &G, int side)
{
    R.i = side ? G.nx - 1 : 0;
    R.ox = 2.0 * G.xf[side ? G.nx : 0] - R.ox;
    R.rx = -R.rx;
    R.sgn ^= 1;
    const double f = G.xf[R.i + 1 - (R.sgn & 1)] + (double)R.wi * G.Lx - R.ox;
    if constexpr (sizeof(Real) == 4) R.tx = f * R.rx;
    else R.tx = f / R.rx;
}

template <class Real, bool INC_XZ>
__device__ __forceinline__ void reflect_z(Ray<Real, INC_XZ> &R, const RayGeo &G, int side)
{
    R.k = side ? G.nz - 1 : 0;
    R.oz = 2.0 * G.zf[side ? G.nz : 0] - R.oz;
    R.rz = -R.rz;
    R.sgn ^= 4;
    const double f = G.zf[R.k + 1 - ((R.sgn >> 2) & 1)] + (double)R.wk * G.Lz - R.oz;
    if constexpr (sizeof(Real) == 4) R.tz = f * R.rz;
    else R.tz = f / R.rz;
}

// Geometry of a step: the segment length ds in the current cell, the axis steps, the walls
// the step ends on (mask of wall bits); returns the brick offset of the next cell.  With
// reflecting walls the ray is mirrored here and goes on in the wall cell.  A step onto a
// wall never updates that axis' brick offset, so the returned offset is always a cell of the
// grid (at a black wall the caller's load stays in bounds and its value is not used).
template <class Real, bool INC_XZ>
__device__ __forceinline__ int ray_advance(Ray<Real, INC_XZ> &R, const RayGeo &G, double &ds, int &wall)
{
    const double te = R.tx < R.ty ? (R.tz < R.tx ? R.tz : R.tx) : (R.tz < R.ty ? R.tz : R.ty);
    ds = te - R.t;
    R.t = te;
    wall = 0;
    if constexpr (sizeof(Real) == 4 && INC_XZ) {
        // uniform periodic x and z: branch-free updates
        const bool mx = R.tx == te, mz = R.tz == te;
        int i = R.i + (mx ? R.stx : 0);
        i = (unsigned)i >= (unsigned)G.nx ? R.wx : i;   // a step past either edge wraps
        R.i = i;
        R.px = brick_x(i, G.bsx);
        R.tx += mx ? R.dtx : 0.0;
        int k = R.k + (mz ? R.stz : 0);
        k = (unsigned)k >= (unsigned)G.nz ? R.wz : k;
        R.k = k;
        R.pz = brick_z(k);
        R.tz += mz ? R.dtz : 0.0;
    } else {
        if (R.tx == te) {
            R.i += (R.sgn & 1) ? -1 : 1;
            if (G.closed && (R.i < 0 || R.i >= G.nx)) {
                const int side = R.i < 0 ? 0 : 1;
                wall |= 1 << (kWallX0 + side);
                if (G.reflect) reflect_x(R, G, side);
            } else {
                if (R.i == G.nx) { R.i = 0; ++R.wi; }
                if (R.i < 0) { R.i = G.nx - 1; --R.wi; }
                R.px = brick_x(R.i, G.bsx);
                const double f = G.xf[R.i + 1 - (R.sgn & 1)] + (double)R.wi * G.Lx - R.ox;
                if constexpr (sizeof(Real) == 4) R.tx = f * R.rx;
                else R.tx = f / R.rx;
            }
        }
        if (R.tz == te) {
            R.k += (R.sgn & 4) ? -1 : 1;
            if (G.closed && (R.k < 0 || R.k >= G.nz)) {
                const int side = R.k < 0 ? 0 : 1;
                wall |= 1 << (kWallZ0 + side);
                if (G.reflect) reflect_z(R, G, side);
            } else {
                if (R.k == G.nz) { R.k = 0; ++R.wk; }
                if (R.k < 0) { R.k = G.nz - 1; --R.wk; }
                R.pz = brick_z(R.k);
                const double f = G.zf[R.k + 1 - ((R.sgn >> 2) & 1)] + (double)R.wk * G.Lz - R.oz;
                if constexpr (sizeof(Real) == 4) R.tz = f * R.rz;
                else R.tz = f / R.rz;
            }
        }
    }
    if (R.ty == te) {
        R.j += (R.sgn & 2) ? -1 : 1;
        if (R.j < 0 || R.j >= G.ny) {
            const int side = R.j < 0 ? 0 : 1;
            wall |= 1 << (kWallY0 + side);
            if (G.reflect) reflect_y(R, G, side);
        } else {
            R.py = brick_y(R.j, G.bsy);
            const double f = G.yf[R.j + 1 - ((R.sgn >> 1) & 1)] - R.oy;
            if constexpr (sizeof(Real) == 4) R.ty = f * R.ry;
            else R.ty = f / R.ry;
        }
    }
    return R.px + R.py + R.pz;
}

// Absorption of a step in the current cell (kappa kc, intensity Ic, length ds); adds the
// terms of the walls the step ended on (mask `wall`, in the order x, y, z: tau eps (I_src -
// I_w), then tau *= 1 - eps, Eq. 3) and the residual when the ray stops.  Returns true when
// the ray is finished (a black wall ends it).
template <class Real, bool INC_XZ>
__device__ __forceinline__ bool ray_absorb(Ray<Real, INC_XZ> &R, Real kc, double Ic, double ds, int wall,
                                           const Walls &W, Real tol, int max_steps)
{
    if constexpr (sizeof(Real) == 8) {
        const double dI = R.Isrc - Ic;
        const double a = -expm1(-kc * ds);
        R.acc += R.tau * a * dI;
        R.tau *= 1.0 - a;
    } else {
        const float x = kc * (float)ds;
        float a, e;
        absorb_f32(x, a, e);
        R.acc += (double)((float)R.tau * a * (float)(R.Isrc - Ic));
        R.tau *= x < 0.25f ? 1.0 - (double)a : (double)e;
    }
    ++R.steps;
    if (wall) {
        for (int w = 0; w < 6; ++w) {
            if (!((wall >> w) & 1)) continue;
            const double e = gld(W.eps + w);
            const double dw = R.Isrc - gld(W.I + w * W.stride);
            const double tw = R.tau;
            R.acc += R.tau * e * dw;
            R.tau *= 1.0 - e;
            if (e == 1.0) {
                R.end = wall_end_code(w);
                R.acc += R.tau * (R.Isrc - Ic);   // residual of a finished ray: zero
                R.tau = tw;                        // kept: the transmissivity the black wall received
                return true;
            }
        }
    }
    if (!(R.tau > (double)tol && R.steps < max_steps)) {
        if (R.steps >= max_steps && R.tau > (double)tol) R.end = kEndCap;
        R.acc += R.tau * (R.Isrc - Ic);   // residual dump into the last cell marched
        return true;
    }
    return false;
}

// The march of one ray, started by ray_init with (k0, I0) of the source cell, until it
// finishes or has taken `cap` steps.  Returns true when finished; when capped, R holds the
// state at the start of the next step (its cell, parameter and next-face parameters).  The
// next cell's record is in flight while the current cell's absorption runs.
template <class Real, bool INC_XZ>
__device__ __forceinline__ bool ray_march(Ray<Real, INC_XZ> &R, const RayGeo &G, const Props<Real> &P,
                                          const Walls &W, Real tol, int max_steps, Real k0, double I0, int cap)
{
    if (!march_starts(tol, max_steps)) return true;
    Real k1;
    double I1, ds;
    int wall;
    while (true) {
        int cell = ray_advance(R, G, ds, wall);
        const uint4 v1 = prop_fetch(P, cell);
        if (ray_absorb(R, k0, I0, ds, wall, W, tol, max_steps)) return true;
        if (R.steps >= cap) return false;
        prop_eval(P, v1, cell, k1, I1);
        cell = ray_advance(R, G, ds, wall);
        const uint4 v0 = prop_fetch(P, cell);
        if (ray_absorb(R, k1, I1, ds, wall, W, tol, max_steps)) return true;
        if (R.steps >= cap) return false;
        prop_eval(P, v0, cell, k0, I0);
    }
}

// Move a ray that stopped after its steps on one grid onto the next coarser grid G1 (every
// other face of the current one; multigrid march of Sec. 4.3).  The ray stays at its point
// on the face it last crossed; its cell becomes the coarse cell holding the current one.  A
// next face of odd index is not a face of G1: the next G1 face along that axis lies one
// current cell further.  With INC_XZ the x / z parameters advance by the current cell
// increment and the increments double; otherwise all three are recomputed from G1's faces.
template <class Real, bool INC_XZ>
__device__ __forceinline__ void ray_descend(Ray<Real, INC_XZ> &R, const RayGeo &G1)
{
    if constexpr (sizeof(Real) == 4 && INC_XZ) {
        if ((R.i + ((R.sgn & 1) ? 0 : 1)) & 1) R.tx += R.dtx;
        if ((R.k + ((R.sgn & 4) ? 0 : 1)) & 1) R.tz += R.dtz;
        R.dtx *= 2.0;
        R.dtz *= 2.0;
        R.i >>= 1;
        R.k >>= 1;
        R.wx = R.stx > 0 ? 0 : G1.nx - 1;
        R.wz = R.stz > 0 ? 0 : G1.nz - 1;
    } else {
        R.i >>= 1;
        R.k >>= 1;
        const double fx = G1.xf[R.i + 1 - (R.sgn & 1)] + (double)R.wi * G1.Lx - R.ox;
        const double fz = G1.zf[R.k + 1 - ((R.sgn >> 2) & 1)] + (double)R.wk * G1.Lz - R.oz;
        if constexpr (sizeof(Real) == 4) {
            R.tx = fx * R.rx;
            R.tz = fz * R.rz;
        } else {
            R.tx = fx / R.rx;
            R.tz = fz / R.rz;
        }
    }
    R.j >>= 1;
    const double fy = G1.yf[R.j + 1 - ((R.sgn >> 1) & 1)] - R.oy;
    if constexpr (sizeof(Real) == 4) R.ty = fy * R.ry;
    else R.ty = fy / R.ry;
    R.px = brick_x(R.i, G1.bsx);
    R.py = brick_y(R.j, G1.bsy);
    R.pz = brick_z(R.k);
}

}  // namespace rmc
