// Host-side derivation of the per-launch constants of the PRC-LBM kernels.
//
// Every constant is computed once in double precision from prc_params and
// handed to the kernels by value in the arithmetic type of the storage
// (double for PRC_F64, float otherwise).  Products of constants are formed
// here, not per node (gfx950 has no scalar floating-point unit, so a product
// of two kernel arguments would cost a vector instruction in every thread).
// Names follow the appendix of arXiv 2208.03562: P_gamma, Q_gamma, U_gamma,
// the strain-solve coefficients of eq. 46, the correction coefficients of
// eq. 38-40 and the transport relation nu = gamma c_s^2 (1/omega_nu - 1/2).
#pragma once

#include <cmath>
#include <atomic>
#include <cstdint>

#include "prc.h"

namespace prc {

// Number of XCDs the hardware distributes workgroups over round-robin.
constexpr int kXcds = 8;
// Two state buffers larger than this do not stay in the 256 MB last-level
// cache from one sweep to the next: their stores are non-temporal.
constexpr int64_t kNtPairBytes = (int64_t)160 << 20;
// Process-wide override of that choice (prc_set_streamed): -1 by size, 0
// never, 1 always.  It changes cache policies and the load order of the
// 1024-thread two-step tiles, never a result.
inline std::atomic<int> g_streamed_mode{-1};

template <typename CT>
struct Coef {
    int32_t nx, ny;
    int32_t pitch;          // elements from one row to the next (same plane)
    uint32_t row_bytes;     // pitch * element size
    uint32_t plane_bytes;   // bytes from one population plane to the next
    uint32_t state_bytes;   // bytes of the whole state
    int32_t corr;           // correction bitmask (generic kernels only)
    int32_t frame;          // prc_frame (generic kernels only)
    int32_t nt;             // store the new state non-temporally
    int32_t tiles_x, tiles_y, tiles_per_xcd;  // sweep tile grid (set per launch)
    CT r, r2;               // y lattice speed and its square (scaling S)
    CT hinv_r, hinv_r2;     // 1/(2r), 1/(2r^2) (S^-1 with the halves of P^-1)
    CT qinv_r, qinv_r2;     // 1/(4r), 1/(4r^2) (with the halves of both axes)
    CT rho0, c2, c2x2, c2sq, c2rho0;  // c2 = c_s^2; 2 c2; c2^2; c2 rho0
    CT ig1;                 // 1/gamma - 1
    CT Pg, Qg;              // 4/gamma^2 - 1/gamma, 1/gamma^2 - 1/gamma
    CT g3;                  // 1/gamma^2 - 3/gamma + 2 (third-order equilibria, eq. 14)
    CT g3p1, g34p1;         // g3 + 1, 4 g3 + 1 (raw moments after the collision)
    CT Ab, Bb;              // (U_gamma c2 - 1)/2, (U_gamma c2 - r^2)/2 (eq. 43)
    CT a1, a2;              // 3 c2 - 1, 3 c2 - r^2 (anisotropy factors)
    CT cb0, cs0;            // -2 c2 / omega_xi, 2 c2 / omega_nu (eq. 46)
    CT mhxi, mhnu;          // -(1/omega_xi - 1/2), -(1/omega_nu - 1/2)
    CT mhxi2, mhnu2;        // twice those (density-gradient terms)
    CT kq11, kl11;          // k11 corrections: -Q_gamma h_nu, -(1/gamma - 1) h_nu c2
    CT sPQ, dPQ;            // (P_gamma + Q_gamma)/4, (P_gamma - Q_gamma)/4
    CT sa0, sb0, sc0, se0;  // constant parts of the strain system for Dx +- Dy
    CT c4hnu;               // 4 c2 h_nu
    CT c2hnu2;              // 2 c2 h_nu (half of c4hnu)
    CT okq11, okl11;        // omega_nu kq11, omega_nu kl11
    CT om_nu, om_xi, om_3, om_4;
    CT fxh, fyh;            // F / (2 gamma) (eq. hydrodynamicfields)
    CT fxg, fyg;            // F / gamma: change of the first-order central moments
    CT qfx, qfy;            // Q_gamma F (central source moments, eq. 13-central)
    CT sxi2, snu2, snu;     // 2 (1 - omega_xi/2), 2 (1 - omega_nu/2), 1 - omega_nu/2
    CT lid;                 // rho0 U c2 / (2 r^2): wall momentum term of a diagonal link
    CT ig, igg;             // 1/gamma, 1/gamma^2 (raw-moment equilibria, eq. 12)
    CT rqfx, rqfy;          // F / gamma^2 (raw source moments, eq. 13)
    CT gxa, gxb, gya, gyb;  // density-gradient stencil weights
};

inline double lattice_c2(double r)
{
    const double q = r < 1.0 ? r : 1.0;  // eq. 2
    return q * q / 3.0;
}

template <typename CT>
inline Coef<CT> make_coef(const prc_params &p, int64_t row_stride, int64_t plane_stride,
                          int64_t total, int64_t elem)
{
    const double r = p.r, g = p.gamma, c2 = lattice_c2(r);
    const double Ug = 2.0 / g + 1.0;
    const double Qg = 1.0 / (g * g) - 1.0 / g;
    const double hnu = 1.0 / p.omega_nu - 0.5, hxi = 1.0 / p.omega_xi - 0.5;
    Coef<CT> c{};
    c.nx = p.nx;
    c.ny = p.ny;
    c.pitch = (int32_t)row_stride;
    c.row_bytes = (uint32_t)(row_stride * elem);
    c.plane_bytes = (uint32_t)(plane_stride * elem);
    c.state_bytes = (uint32_t)(total * elem);
    c.corr = p.corrections;
    c.frame = p.frame;
    const int mode = g_streamed_mode.load(std::memory_order_relaxed);
    c.nt = mode >= 0 ? mode : 2 * total * elem > kNtPairBytes;
    c.r = CT(r);
    c.r2 = CT(r * r);
    c.hinv_r = CT(0.5 / r);
    c.hinv_r2 = CT(0.5 / (r * r));
    c.qinv_r = CT(0.25 / r);
    c.qinv_r2 = CT(0.25 / (r * r));
    c.rho0 = CT(p.rho0);
    c.c2 = CT(c2);
    c.c2x2 = CT(2.0 * c2);
    c.c2sq = CT(c2 * c2);
    c.c2rho0 = CT(c2 * p.rho0);
    c.ig1 = CT(1.0 / g - 1.0);
    c.Pg = CT(4.0 / (g * g) - 1.0 / g);
    c.Qg = CT(Qg);
    c.g3 = CT(1.0 / (g * g) - 3.0 / g + 2.0);
    c.g3p1 = CT(1.0 / (g * g) - 3.0 / g + 3.0);
    c.g34p1 = CT(4.0 / (g * g) - 12.0 / g + 9.0);
    c.Ab = CT(0.5 * (Ug * c2 - 1.0));
    c.Bb = CT(0.5 * (Ug * c2 - r * r));
    c.a1 = CT(3.0 * c2 - 1.0);
    c.a2 = CT(3.0 * c2 - r * r);
    c.cb0 = CT(-2.0 * c2 / p.omega_xi);
    c.cs0 = CT(2.0 * c2 / p.omega_nu);
    c.mhxi = CT(-hxi);
    c.mhnu = CT(-hnu);
    c.mhxi2 = CT(-2.0 * hxi);
    c.mhnu2 = CT(-2.0 * hnu);
    c.kq11 = CT(-Qg * hnu);
    c.kl11 = CT(-(1.0 / g - 1.0) * hnu * c2);
    {
        // coefficients of eq. 46 over rho: cbx = (P ux^2 + Q uy^2 + a1)/2 + cb0,
        // cby = (P uy^2 + Q ux^2 + a2)/2 + cb0, csx = (P ux^2 - Q uy^2 + a1)/2 - cs0,
        // csy = cs0 - (P uy^2 - Q ux^2 + a2)/2; their half sums and differences
        // are linear in ux^2 + uy^2 and ux^2 - uy^2
        const double Pg = 4.0 / (g * g) - 1.0 / g, cb0 = -2.0 * c2 / p.omega_xi;
        const double cs0 = 2.0 * c2 / p.omega_nu;
        const double bx0 = 0.5 * (3.0 * c2 - 1.0) + cb0, by0 = 0.5 * (3.0 * c2 - r * r) + cb0;
        const double sx0 = 0.5 * (3.0 * c2 - 1.0) - cs0, sy0 = cs0 - 0.5 * (3.0 * c2 - r * r);
        c.sPQ = CT(0.25 * (Pg + Qg));
        c.dPQ = CT(0.25 * (Pg - Qg));
        c.sa0 = CT(0.5 * (bx0 + by0));
        c.sb0 = CT(0.5 * (bx0 - by0));
        c.sc0 = CT(0.5 * (sx0 + sy0));
        c.se0 = CT(0.5 * (sx0 - sy0));
    }
    c.c4hnu = CT(4.0 * c2 * hnu);
    c.c2hnu2 = CT(2.0 * c2 * hnu);
    c.okq11 = CT(p.omega_nu * -Qg * hnu);
    c.okl11 = CT(p.omega_nu * -(1.0 / g - 1.0) * hnu * c2);
    c.om_nu = CT(p.omega_nu);
    c.om_xi = CT(p.omega_xi);
    c.om_3 = CT(p.omega_3);
    c.om_4 = CT(p.omega_4);
    c.fxh = CT(p.fx / (2.0 * g));
    c.fyh = CT(p.fy / (2.0 * g));
    c.fxg = CT(p.fx / g);
    c.fyg = CT(p.fy / g);
    c.qfx = CT(Qg * p.fx);
    c.qfy = CT(Qg * p.fy);
    c.sxi2 = CT(2.0 - p.omega_xi);
    c.snu2 = CT(2.0 - p.omega_nu);
    c.snu = CT(1.0 - 0.5 * p.omega_nu);
    c.lid = CT(p.rho0 * p.u_lid * c2 / (2.0 * r * r));
    c.ig = CT(1.0 / g);
    c.igg = CT(1.0 / (g * g));
    c.rqfx = CT(p.fx / (g * g));
    c.rqfy = CT(p.fy / (g * g));
    c.gxa = CT(0.5 * (1.0 - c2 / (r * r)));
    c.gxb = CT(0.25 * c2 / (r * r));
    c.gya = CT((1.0 - c2) / (2.0 * r));
    c.gyb = CT(c2 / (4.0 * r));
    return c;
}

}  // namespace prc
