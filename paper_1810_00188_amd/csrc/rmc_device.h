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
constexpr int kEndTol = 0, kEndWallLo = 1, kEndWallHi = 2, kEndCap = 3;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each two 32x32->64 bit products of
// counter words with fixed multipliers, xor-mixed with the other words and the round key;
// the key is bumped by two Weyl constants after every round.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint32_t lo0 = c0 * 0xD2511F53u, hi0 = __umulhi(c0, 0xD2511F53u);
        const uint32_t lo1 = c2 * 0xCD9E8D57u, hi1 = __umulhi(c2, 0xCD9E8D57u);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
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
__device__ __forceinline__ int brick_x(int i, int sx_) { return (i >> 2) * sx_ + ((i & 1) << 2) + ((i & 2) << 4); }
__device__ __forceinline__ int brick_y(int j, int sy_) { return (j >> 2) * sy_ + ((j & 1) << 1) + ((j & 2) << 3); }
__device__ __forceinline__ int brick_z(int k) { return ((k >> 2) << 6) + (k & 1) + ((k & 2) << 2); }

// Geometry of one snapshot as seen by a ray.
struct RayGeo {
    const double *xf, *yf, *zf; // face coordinates (LDS), nx+1, ny+1, nz+1
    int nx, ny, nz;
    int bsx, bsy;               // brick strides of the x and y brick index (in cells)
    double Lx, Lz;              // periodic lengths
};

template <class Real> struct MarchOut {
    Real acc;                   // sum tau alpha (I_src - I_j) + wall + residual terms
    Real absacc;                // same with |I_src - I_j| (only when asked for)
    int steps;
    int end;
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

// March one ray from the centre of cell (ci, cj, ck) along (dx, dy, dz) (Algorithm 1, March):
// ds = distance to the nearest face, alpha = 1 - exp(-kappa ds) (Eq. 2), acc += tau alpha
// (I_src - I_cell), tau *= 1 - alpha (Eq. 3); every axis whose face is reached steps; x and z
// wrap, leaving y hits a black wall (alpha = 1, I = I_b(T_wall)).  Stops at tau <= tol or after
// max_steps and adds the residual tau (I_src - I_last).
//
// K is the kappa_{n,g} plane of the ray's (band, g-point), Ipl the I_n plane of its band, both
// in the bricked layout.  The path geometry (face parameters t, segment lengths) and the
// intensity differences are double in both precisions; Real sets the arithmetic of kappa,
// alpha, tau and the accumulated sum: FP64 follows the reference operation by operation, FP32
// takes the transmission as exp(-x) itself (absorb_f32).
template <class Real, bool ABS>
__device__ __forceinline__ MarchOut<Real>
march_ray(const RayGeo &G, const Real *__restrict__ K, const double *__restrict__ Ipl, int ci, int cj, int ck,
          double dx, double dy, double dz, double Isrc, double Iw0, double Iw1, Real tol, int max_steps)
{
    const double ox = 0.5 * (G.xf[ci] + G.xf[ci + 1]);
    const double oy = 0.5 * (G.yf[cj] + G.yf[cj + 1]);
    const double oz = 0.5 * (G.zf[ck] + G.zf[ck + 1]);
    const int sx = dx > 0.0 ? 1 : -1, sy = dy > 0.0 ? 1 : -1, sz = dz > 0.0 ? 1 : -1;
    const int ux = sx > 0, uy = sy > 0, uz = sz > 0;
    // FP64 march: the reference's divisions; FP32 march: one reciprocal per axis and ray
    const double rx = 1.0 / dx, ry = 1.0 / dy, rz = 1.0 / dz;
    auto face_t = [&](double num, double d, double r) -> double {
        if constexpr (sizeof(Real) == 8) return num / d;
        else return num * r;
    };
    int i = ci, j = cj, k = ck, wi = 0, wk = 0;
    double tx = face_t(G.xf[i + ux] - ox, dx, rx);
    double ty = face_t(G.yf[j + uy] - oy, dy, ry);
    double tz = face_t(G.zf[k + uz] - oz, dz, rz);
    int px = brick_x(i, G.bsx), py = brick_y(j, G.bsy), pz = brick_z(k);
    double t = 0.0, Ilast = Isrc;
    Real tau = 1, acc = 0, absacc = 0;
    int steps = 0, end = kEndTol;
    while (tau > tol && steps < max_steps) {
        const double te = fmin(tx, fmin(ty, tz));
        const int cell = px + py + pz;
        const Real kap = K[cell];
        const double Ij = Ipl[cell];
        if constexpr (sizeof(Real) == 8) {
            const double ds = te - t;
            const double dI = Isrc - Ij;
            const double a = -expm1(-kap * ds);
            acc += tau * a * dI;
            if (ABS) absacc += tau * a * fabs(dI);
            tau *= 1.0 - a;
        } else {
            const float ds = (float)(te - t);
            const float dI = (float)(Isrc - Ij);
            float a, e;
            absorb_f32(kap * ds, a, e);
            const float ta = tau * a;
            acc = fmaf(ta, dI, acc);
            if (ABS) absacc = fmaf(ta, fabsf(dI), absacc);
            tau *= e;
        }
        ++steps;
        t = te;
        Ilast = Ij;
        bool wall = false;
        if (tx == te) {
            i += sx;
            if (i == G.nx) { i = 0; ++wi; }
            if (i < 0) { i = G.nx - 1; --wi; }
            px = brick_x(i, G.bsx);
            tx = face_t(G.xf[i + ux] + (double)wi * G.Lx - ox, dx, rx);
        }
        if (ty == te) {
            j += sy;
            if (j < 0) { wall = true; end = kEndWallLo; }
            else if (j >= G.ny) { wall = true; end = kEndWallHi; }
            else {
                py = brick_y(j, G.bsy);
                ty = face_t(G.yf[j + uy] - oy, dy, ry);
            }
        }
        if (tz == te) {
            k += sz;
            if (k == G.nz) { k = 0; ++wk; }
            if (k < 0) { k = G.nz - 1; --wk; }
            pz = brick_z(k);
            tz = face_t(G.zf[k + uz] + (double)wk * G.Lz - oz, dz, rz);
        }
        if (wall) {
            const Real dw = (Real)(Isrc - (end == kEndWallLo ? Iw0 : Iw1));
            acc += tau * dw;
            if (ABS) absacc += tau * fabs(dw);
            tau = (Real)0;
            break;
        }
    }
    if (end == kEndTol && steps >= max_steps && tau > tol) end = kEndCap;
    const Real dl = (Real)(Isrc - Ilast);
    acc += tau * dl;
    if (ABS) absacc += tau * fabs(dl);
    MarchOut<Real> m;
    m.acc = acc;
    m.absacc = absacc;
    m.steps = steps;
    m.end = end;
    return m;
}

}  // namespace rmc
