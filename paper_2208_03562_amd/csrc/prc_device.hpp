// Device building blocks of the PRC-LBM sweep for gfx950.
//
// Populations are held as deviations d_a = f_a - rho0 w_a from the rest state
// (w_a: rest weights of variance c_s^2 along x and c_s^2/r^2 along y).  The
// per-node collision below is the algorithm of Appendix A of arXiv 2208.03562
// rewritten, term by term, for deviations: every moment is split into its
// rest-state part (rho0 times (1,0,0,c2,c2,0,0,0,c2^2), identical for raw and
// central moments at u = 0) and a small remainder, and only the remainders
// are carried.  The rest-state parts cancel exactly in every relaxation
// (k - k_eq), so the result is the paper's update with all large constants
// removed before rounding -- which is what keeps FP32 (and 16-bit storage)
// accurate at low Mach number.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "prc_coef.hpp"

namespace prc {

// Velocity set of Sec. 2 (e_y in units of r) and its opposite directions.
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// Lid term of an incoming population bounced at the top wall, in units of
// Coef::lid: f_7 = f~_5 - lid, f_8 = f~_6 + lid, f_4 = f~_2.
constexpr int LIDC[9] = {0, 0, 0, 0, 0, 0, 0, -1, 1};

// ---- storage element <-> arithmetic type --------------------------------
template <typename ST, typename CT> struct Conv;
template <> struct Conv<double, double> {
    static __device__ __forceinline__ double ld(double v) { return v; }
    static __device__ __forceinline__ double st(double v) { return v; }
};
template <> struct Conv<float, float> {
    static __device__ __forceinline__ float ld(float v) { return v; }
    static __device__ __forceinline__ float st(float v) { return v; }
};
template <> struct Conv<__half, float> {
    static __device__ __forceinline__ float ld(__half v) { return __half2float(v); }
    static __device__ __forceinline__ __half st(float v) { return __float2half_rn(v); }
};
template <> struct Conv<__hip_bfloat16, float> {
    static __device__ __forceinline__ float ld(__hip_bfloat16 v) { return __bfloat162float(v); }
    static __device__ __forceinline__ __hip_bfloat16 st(float v) { return __float2bfloat16(v); }
};

// ---- boundary traits -----------------------------------------------------
template <int BC> struct Bc {
    static constexpr bool wrap_x = BC != PRC_BC_CAVITY;
    static constexpr bool wrap_y = BC == PRC_BC_PERIODIC;
    static constexpr bool lid = BC != PRC_BC_PERIODIC;
};

// one period of wrap-around: v in [-n, 2n)
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// any v
__device__ __forceinline__ int wrap_any(int v, int n) { const int m = v % n; return m < 0 ? m + n : m; }
__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Coordinates of the node whose density stands in for (x, y) in the density
// gradient stencil: periodic directions wrap, walls clamp to the nearest node
// inside the domain.  Also maps tile slots beyond the grid (ragged edges, and
// grids narrower than a tile) onto real nodes.
template <int BC>
__device__ __forceinline__ void fix_coord(int &x, int &y, int nx, int ny)
{
    x = Bc<BC>::wrap_x ? wrap_any(x, nx) : clampi(x, nx);
    y = Bc<BC>::wrap_y ? wrap_any(y, ny) : clampi(y, ny);
}

// Streaming with boundaries (Appendix A, "stream"): d_a(x) = d~_a(x - e_a).
// A source outside a wall means half-way bounce-back: the population that
// left this node along opp(a) returns along a; a source above the top row
// crosses the lid and picks up the wall momentum term (corners included).
// CHECK = false is the fast path for nodes whose nine sources are all inside.
template <typename ST, typename CT, int BC, bool CHECK>
__device__ __forceinline__ void pull(const Coef<CT> &c, const ST *__restrict__ src, int x,
                                     int y, CT d[9])
{
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int sx = x - EX[a], sy = y - EY[a];
        if (!CHECK) {
            d[a] = Conv<ST, CT>::ld(src[a * c.plane + (int64_t)sy * c.pitch + sx]);
            continue;
        }
        bool out = false;
        if (Bc<BC>::wrap_x) sx = wrap(sx, c.nx);
        else out |= (sx < 0) | (sx >= c.nx);
        if (Bc<BC>::wrap_y) sy = wrap(sy, c.ny);
        else out |= (sy < 0) | (sy >= c.ny);
        if (!out) {
            d[a] = Conv<ST, CT>::ld(src[a * c.plane + (int64_t)sy * c.pitch + sx]);
        } else {
            CT v = Conv<ST, CT>::ld(src[OPP[a] * c.plane + (int64_t)y * c.pitch + x]);
            if (Bc<BC>::lid && LIDC[a] != 0 && sy >= c.ny) v += CT(LIDC[a]) * c.lid;
            d[a] = v;
        }
    }
}

template <typename CT>
__device__ __forceinline__ CT sum9(const CT d[9])
{
    return ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
}

// Hydrodynamic fields of streamed deviations (eq. hydrodynamicfields):
// rho = rho0 + sum d, rho u = sum d e + F / (2 gamma) (the rest state carries
// no momentum).
template <typename CT>
__device__ __forceinline__ void fields(const Coef<CT> &c, const CT d[9], CT &drho, CT &ux,
                                       CT &uy)
{
    drho = sum9(d);
    const CT jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    const CT jy = ((d[2] - d[4]) + (d[5] - d[8]) + (d[6] - d[7])) * c.r;
    const CT irho = CT(1) / (c.rho0 + drho);
    ux = (jx + c.fxh) * irho;
    uy = (jy + c.fyh) * irho;
}

// One node's collision, Appendix A sub-steps 1-7, on deviations.
// In: d = streamed deviations, (gx, gy) = density gradient at the node.
// Out: d = post-collision deviations.
template <typename CT>
__device__ __forceinline__ void collide(const Coef<CT> &c, CT d[9], CT gx, CT gy)
{
    // 1. raw moments on the square lattice (eq. 62), deviation parts
    const CT s13 = d[1] + d[3], s24 = d[2] + d[4];
    const CT s5678 = (d[5] + d[6]) + (d[7] + d[8]);
    const CT m00 = d[0] + s13 + s24 + s5678;
    const CT m10 = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    CT m01 = (d[2] - d[4]) + (d[5] - d[8]) + (d[6] - d[7]);
    const CT m20 = s13 + s5678;
    CT m02 = s24 + s5678;
    CT m11 = (d[5] - d[6]) + (d[7] - d[8]);
    CT m21 = (d[5] + d[6]) - (d[7] + d[8]);
    CT m12 = (d[5] - d[6]) - (d[7] - d[8]);
    CT m22 = s5678;
    // 2. scaling S: k'_mn picks up r^n
    m01 *= c.r;
    m02 *= c.r2;
    m11 *= c.r;
    m21 *= c.r;
    m12 *= c.r2;
    m22 *= c.r2;

    // fields (eq. hydrodynamicfields)
    const CT drho = m00;
    const CT rho = c.rho0 + drho;
    const CT irho = CT(1) / rho;
    const CT ux = (m10 + c.fxh) * irho;
    const CT uy = (m01 + c.fyh) * irho;
    const CT ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;

    // 3. central moments, F(u), minus the rest-state parts.  (The first-order
    // ones, k10 and k01, are exactly -F/(2 gamma) by the definition of u.)
    const CT k20 = m20 - CT(2) * ux * m10 + ux2 * rho;
    const CT k02 = m02 - CT(2) * uy * m01 + uy2 * rho;
    const CT k11 = m11 - uy * m10 - ux * m01 + uxy * rho;
    const CT M20 = c.c2rho0 + m20, M02 = c.c2rho0 + m02;  // full second raw moments
    const CT k21 = m21 - CT(2) * ux * m11 + ux2 * m01 - uy * M20 + CT(2) * uxy * m10
                 - ux2 * uy * rho;
    const CT k12 = m12 - CT(2) * uy * m11 + uy2 * m10 - ux * M02 + CT(2) * uxy * m01
                 - ux * uy2 * rho;
    const CT k22 = m22 - CT(2) * ux * m12 + ux2 * M02 - CT(2) * uy * m21
                 + CT(4) * uxy * m11 - CT(2) * ux2 * uy * m01 + uy2 * M20
                 - CT(2) * ux * uy2 * m10 + ux2 * uy2 * rho;

    // 4. collision.  Combine (operator B).
    const CT k2s = k20 + k02;  // minus 2 c2 rho0
    const CT k2d = k20 - k02;

    // base preconditioned equilibria (eq. 14), minus rest-state parts
    const CT e2s = CT(2) * c.c2 * drho + c.ig1 * rho * (ux2 + uy2);
    const CT e2d = c.ig1 * rho * (ux2 - uy2);
    const CT e11 = c.ig1 * rho * uxy;

    CT cor2s = CT(0), cor2d = CT(0), cor11 = CT(0);
    if (c.corr) {
        CT dxux = CT(0), dyuy = CT(0);
        const CT pux = c.Pg * ux2, puy = c.Pg * uy2, qux = c.Qg * ux2, quy = c.Qg * uy2;
        if (c.corr & (PRC_CORR_THETA | PRC_CORR_K11)) {
            // local strain rates from non-equilibrium moments: eq. 43, 45,
            // 46 and the solution eq. 48
            const CT A = c.Ab * ux, B = c.Bb * uy;
            const CT eb = -A * gx - B * gy;
            const CT es = -A * gx + B * gy;
            const CT R2s = k2s - e2s + eb;
            const CT R2d = k2d - e2d + es;
            const CT Cbx = (c.cb0 + CT(0.5) * (pux + quy) + CT(0.5) * c.a1) * rho;
            const CT Cby = (c.cb0 + CT(0.5) * (puy + qux) + CT(0.5) * c.a2) * rho;
            const CT Csx = (-c.cs0 + CT(0.5) * (pux - quy) + CT(0.5) * c.a1) * rho;
            const CT Csy = (c.cs0 + CT(0.5) * (qux - puy) - CT(0.5) * c.a2) * rho;
            dxux = (Csy * R2s - Cby * R2d) / (Cbx * Csy - Csx * Cby);
            dyuy = (R2s - Cbx * dxux) / Cby;
        }
        // corrections, eq. 38 (k2s), 39 (k2d), 40 (k11)
        if (c.corr & PRC_CORR_THETA) {
            const CT tbx = -(pux + quy + c.a1) * rho * c.hxi;
            const CT tby = -(puy + qux + c.a2) * rho * c.hxi;
            const CT tsx = -(pux - quy + c.a1) * rho * c.hnu;
            const CT tsy = (qux - puy - c.a2) * rho * c.hnu;
            cor2s += tbx * dxux + tby * dyuy;
            cor2d += tsx * dxux - tsy * dyuy;
        }
        if (c.corr & PRC_CORR_LAMBDA) {
            // lambda_bx = -2 Ab hxi ux, lambda_by = -2 Bb hxi uy,
            // lambda_sx = -2 Ab hnu ux, lambda_sy = +2 Bb hnu uy
            const CT ax = CT(2) * c.Ab * ux * gx, by = CT(2) * c.Bb * uy * gy;
            cor2s -= c.hxi * (ax + by);
            cor2d -= c.hnu * (ax - by);
        }
        if (c.corr & PRC_CORR_K11) {
            cor11 = -c.Qg * c.hnu * rho * uxy * (dxux + dyuy)
                  - c.ig1 * c.hnu * c.c2 * (uy * gx + ux * gy);
        }
    }

    // sources (eq. 13-central); the first-order ones are folded into k~10,
    // k~01 below
    const CT s2s = CT(2) * (c.qfx * ux + c.qfy * uy);
    const CT s2d = CT(2) * (c.qfx * ux - c.qfy * uy);
    const CT s11 = c.qfx * uy + c.qfy * ux;

    // relax (Appendix A relaxation sub-step), then segregate (B^-1).
    // k~10 = k10 + omega_1 (0 - k10) + (1 - omega_1/2) F_x / gamma = F_x/(2 gamma)
    // for every omega_1, since k10 = -F_x/(2 gamma).
    const CT t10 = c.fxh, t01 = c.fyh;
    const CT t2s = k2s + c.om_xi * (e2s + cor2s - k2s) + c.sxi * s2s;
    const CT t2d = k2d + c.om_nu * (e2d + cor2d - k2d) + c.snu * s2d;
    const CT t11 = k11 + c.om_nu * (e11 + cor11 - k11) + c.snu * s11;
    const CT t21 = k21 + c.om_3 * (c.g3 * rho * ux2 * uy - k21);
    const CT t12 = k12 + c.om_3 * (c.g3 * rho * ux * uy2 - k12);
    const CT t22 = k22 + c.om_4 * (c.c2 * c.c2 * drho - k22);
    const CT t20 = CT(0.5) * (t2s + t2d);
    const CT t02 = CT(0.5) * (t2s - t2d);

    // 5. raw moments F(-u), minus rest-state parts
    const CT T20 = c.c2rho0 + t20, T02 = c.c2rho0 + t02;
    const CT n10 = t10 + ux * rho;
    CT n01 = t01 + uy * rho;
    const CT n20 = t20 + CT(2) * ux * t10 + ux2 * rho;
    CT n02 = t02 + CT(2) * uy * t01 + uy2 * rho;
    CT n11 = t11 + uy * t10 + ux * t01 + uxy * rho;
    CT n21 = t21 + CT(2) * ux * t11 + ux2 * t01 + uy * T20 + CT(2) * uxy * t10
           + ux2 * uy * rho;
    CT n12 = t12 + CT(2) * uy * t11 + uy2 * t10 + ux * T02 + CT(2) * uxy * t01
           + ux * uy2 * rho;
    CT n22 = t22 + CT(2) * ux * t12 + ux2 * T02 + CT(2) * uy * t21 + CT(4) * uxy * t11
           + CT(2) * ux2 * uy * t01 + uy2 * T20 + CT(2) * ux * uy2 * t10
           + ux2 * uy2 * rho;
    // 6. inverse scaling S^-1
    n01 *= c.inv_r;
    n02 *= c.inv_r2;
    n11 *= c.inv_r;
    n21 *= c.inv_r;
    n12 *= c.inv_r2;
    n22 *= c.inv_r2;
    // 7. populations, P^-1 (eq. 72)
    d[0] = drho - n20 - n02 + n22;
    d[1] = CT(0.5) * (n10 + n20 - n12 - n22);
    d[2] = CT(0.5) * (n01 + n02 - n21 - n22);
    d[3] = CT(0.5) * (-n10 + n20 + n12 - n22);
    d[4] = CT(0.5) * (-n01 + n02 + n21 - n22);
    d[5] = CT(0.25) * (n11 + n21 + n12 + n22);
    d[6] = CT(0.25) * (-n11 + n21 - n12 + n22);
    d[7] = CT(0.25) * (n11 - n21 - n12 + n22);
    d[8] = CT(0.25) * (-n11 - n21 + n12 + n22);
}

}  // namespace prc
