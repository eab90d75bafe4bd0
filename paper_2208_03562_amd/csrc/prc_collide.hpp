// Per-node collision of the PRC-LBM (arXiv 2208.03562, Appendix A) on gfx950.
//
// The update is the appendix's f~ = P^-1 S^-1 F(-u) [m^c + B^-1 {Lambda (B
// m^{c,eq} - B m^c) + (I - Lambda/2) B Phi^c}], m^c = F(u) S P f, evaluated in
// an equivalent order chosen for few operations and small rounding errors:
//
//  * D2Q9 is the tensor product of two three-velocity lattices, and so are the
//    maps of the appendix: P and S are products of one-dimensional maps and
//    F(u) is the product of the binomial shifts along x and y.  The nine
//    central moments are formed by a three-point transform along x for each
//    row of the velocity set, then along y for each x-moment.
//  * Since the whole map is linear in the moments, f~ = f + T^-1(dk), where
//    T = F(u) S P and dk is the change of the central moments in the
//    collision (zero for k00, F/gamma for k10 and k01).  Only the increments
//    are transformed back, so the post-collision populations are the stored
//    ones plus a small correction.
//  * Populations are deviations from the rest state rho0 w.  The central
//    moments of the deviations, plus the closed-form central moments of
//    rho0 w about u minus rho0 (1,0,c2)x(1,0,c2), are the central moments of
//    f minus that constant tensor; every equilibrium below is written minus
//    the same constant, which cancels in each difference k_eq - k.
//  * The correction terms of eq. 38-40 need rho times the strain rates of
//    eq. 48; the coefficients of eq. 46 all carry a factor rho, so the solve
//    is done for rho dxux, rho dyuy directly and rho never appears.
//
// collide_plain is the method exactly as the paper runs it (every correction,
// unit rates for the non-hydrodynamic moments, no body force) with fewer
// operations: only the second central moments are formed, the correction
// terms are summed in closed form through the strain-rate equations, and the
// change of the raw moments is added to the stored deviations.
//
// collide_raw is the same update with the moments relaxed in the rest frame
// (raw moments, the PRNR-LBM of Sec. 4.1 used for comparison in Sec. 6): raw
// equilibria of eq. 12, raw sources of eq. 13, the same corrections.
#pragma once

#include "prc_device.hpp"

namespace prc {

// Correction terms of the second-order equilibria (eq. 38-40) with the local
// strain rates of eq. 43-48, from the second-order non-equilibrium parts
// n2s = k2s - k2s_eq and n2d = k2d - k2d_eq (the same in the central and the
// raw frame).  The solve is done for rho dxux, rho dyuy: the coefficients of
// eq. 46 all carry a factor rho, so rho never appears.
template <typename CT>
__device__ __forceinline__ void corrections(const Coef<CT> &c, CT ux, CT uy, CT ux2, CT uy2, CT uxy,
                                            CT n2s, CT n2d, CT gx, CT gy, CT &cor2s, CT &cor2d,
                                            CT &cor11)
{
    cor2s = CT(0);
    cor2d = CT(0);
    cor11 = CT(0);
    const int corr = c.corr;
    if (!corr) return;
    // bx = P ux^2 + Q uy^2 + a1, sx = P ux^2 - Q uy^2 + a1 (likewise by, sy)
    const CT tx = c.Pg * ux2 + c.a1, ty = c.Pg * uy2 + c.a2;
    const CT bx = tx + c.Qg * uy2, sx = tx - c.Qg * uy2;
    const CT by = ty + c.Qg * ux2, sy = ty - c.Qg * ux2;
    const CT Agx = c.Ab * ux * gx, Bgy = c.Bb * uy * gy;  // -e_b = Agx + Bgy
    CT Dx = CT(0), Dy = CT(0);                            // rho dxux, rho dyuy
    if (corr & (PRC_CORR_THETA | PRC_CORR_K11)) {
        const CT R2s = n2s - (Agx + Bgy);
        const CT R2d = n2d + (Bgy - Agx);
        const CT cbx = c.cb0 + CT(0.5) * bx, cby = c.cb0 + CT(0.5) * by;
        const CT csx = CT(0.5) * sx - c.cs0, csy = c.cs0 - CT(0.5) * sy;
        const CT det = cbx * csy - csx * cby;
        // one reciprocal serves both divisions of eq. 48
        const CT ip = recip(det * cby);
        Dx = (csy * R2s - cby * R2d) * (cby * ip);
        Dy = (R2s - cbx * Dx) * (det * ip);
    }
    if (corr & PRC_CORR_THETA) {
        // theta_bx = -bx rho h_xi, theta_by = -by rho h_xi, theta_sx =
        // -sx rho h_nu, theta_sy = -sy rho h_nu; k2d takes theta_sx dxux
        // - theta_sy dyuy
        cor2s = c.mhxi * (bx * Dx + by * Dy);
        cor2d = c.mhnu * (sx * Dx - sy * Dy);
    }
    if (corr & PRC_CORR_LAMBDA) {
        cor2s += c.mhxi2 * (Agx + Bgy);
        cor2d += c.mhnu2 * (Agx - Bgy);
    }
    if (corr & PRC_CORR_K11)
        cor11 = c.kq11 * uxy * (Dx + Dy) + c.kl11 * (uy * gx + ux * gy);
}

// The general central-moment collision: the correction bitmask and all rates
// are read at run time.  FORCE: the body force may be nonzero.
template <typename CT, bool FORCE>
__device__ __forceinline__ void collide(const Coef<CT> &c, CT d[9], CT gx, CT gy)
{
    CT q[3][3];  // [e_y + 1][e_x + 1]
#pragma unroll
    for (int a = 0; a < 9; ++a) q[QJ[a]][QI[a]] = d[a];

    // raw x-moments of each row of the velocity set (eq. 62 along x)
    CT X0[3], X1[3], X2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        X1[j] = q[j][2] - q[j][0];
        X2[j] = q[j][2] + q[j][0];
        X0[j] = X2[j] + q[j][1];
    }
    // fields (eq. hydrodynamicfields); the y lattice speed is r (scaling S)
    const CT drho = (X0[0] + X0[1]) + X0[2];
    const CT rho = c.rho0 + drho;
    const CT irho = recip(rho);
    CT jx = (X1[0] + X1[1]) + X1[2], jy = c.r * (X0[2] - X0[0]);
    if (FORCE) {
        jx += c.fxh;
        jy += c.fyh;
    }
    const CT ux = jx * irho, uy = jy * irho;
    const CT ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;

    // central x-moments of each row: binomial shift by u_x
    CT C1[3], C2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        C1[j] = X1[j] - ux * X0[j];
        C2[j] = X2[j] - ux * (X1[j] + C1[j]);
    }
    // central y-moments (lattice speed r) of each central x-moment
    auto ytrans = [&](CT A, CT B, CT Cc, CT &K0, CT &K1, CT &K2) {
        const CT Y1 = c.r * (Cc - A);
        K0 = (A + B) + Cc;
        K1 = Y1 - uy * K0;
        K2 = c.r2 * (Cc + A) - uy * (Y1 + K1);
    };
    CT K00, K01, K02, K10, K11, K12, K20, K21, K22;
    ytrans(X0[0], X0[1], X0[2], K00, K01, K02);
    ytrans(C1[0], C1[1], C1[2], K10, K11, K12);
    ytrans(C2[0], C2[1], C2[2], K20, K21, K22);
    (void)K00;
    (void)K01;
    (void)K10;
    // plus the central moments of rho0 w about u, minus rho0 (1,0,c2)x(1,0,c2)
    const CT u2s = ux2 + uy2;
    const CT k20 = K20 + c.rho0 * ux2;
    const CT k02 = K02 + c.rho0 * uy2;
    const CT k11 = K11 + c.rho0 * uxy;
    const CT k21 = K21 - uy * (c.c2rho0 + c.rho0 * ux2);
    const CT k12 = K12 - ux * (c.c2rho0 + c.rho0 * uy2);
    const CT k22 = K22 + c.rho0 * (c.c2 * u2s + ux2 * uy2);

    // combine (operator B)
    const CT k2s = k20 + k02;  // minus 2 c2 rho0
    const CT k2d = k20 - k02;

    // preconditioned equilibria (eq. 14), minus the same constants
    const CT irh = c.ig1 * rho;
    const CT e2s = c.c2x2 * drho + irh * u2s;
    const CT e2d = irh * (ux2 - uy2);
    const CT e11 = irh * uxy;

    // corrections (eq. 38-40) with the local strain rates (eq. 43-48)
    CT cor2s, cor2d, cor11;
    corrections<CT>(c, ux, uy, ux2, uy2, uxy, k2s - e2s, k2d - e2d, gx, gy, cor2s, cor2d, cor11);

    // moment increments of the relaxation (Appendix A), B^-1 folded in
    CT d2s = c.om_xi * ((e2s + cor2s) - k2s);
    CT d2d = c.om_nu * ((e2d + cor2d) - k2d);
    CT d11 = c.om_nu * ((e11 + cor11) - k11);
    if (FORCE) {
        // central source moments (eq. 13-central) with weights 1 - omega/2
        d2s += c.sxi2 * (c.qfx * ux + c.qfy * uy);
        d2d += c.snu2 * (c.qfx * ux - c.qfy * uy);
        d11 += c.snu * (c.qfx * uy + c.qfy * ux);
    }
    const CT g3r = c.g3 * rho;
    const CT d21 = c.om_3 * (g3r * ux2 * uy - k21);
    const CT d12 = c.om_3 * (g3r * ux * uy2 - k12);
    const CT d22 = c.om_4 * (c.c2sq * drho - k22);
    const CT d2sum = d2s + d2d;
    const CT d20 = CT(0.5) * d2sum, d20h = CT(0.25) * d2sum;
    const CT d02 = CT(0.5) * (d2s - d2d);

    // f~ = f + P^-1 S^-1 F(-u) dk: y-transform back for each x-moment, giving
    // half the result (the halves of the x-transform folded in; K0h = K0 / 2)
    // ...
    // (x * 0 and x + 0 are not folded away in IEEE arithmetic, so the moments
    // known to be zero get their own forms)
    CT G[3][3];  // [x-moment][e_y + 1], halved
    auto yinv = [&](CT K0, CT K0h, CT K1, CT K2, CT *g) {
        const CT R1 = K1 + uy * K0;
        const CT R2 = K2 + uy * (K1 + R1);
        const CT a = c.qinv_r * R1, b = c.qinv_r2 * R2;  // 1/(4r), 1/(4r^2)
        g[0] = b - a;
        g[1] = K0h - CT(2) * b;
        g[2] = b + a;
    };
    auto yinv_no0 = [&](CT K1, CT K2, CT *g) {  // K0 = 0
        const CT R2 = K2 + uy * (K1 + K1);
        const CT a = c.qinv_r * K1, b = c.qinv_r2 * R2;
        g[0] = b - a;
        g[1] = CT(-2) * b;
        g[2] = b + a;
    };
    if (FORCE) {
        // the first-order central moments change by F/gamma (k~10 = F/(2 gamma)
        // for any omega_1, since k10 = -F/(2 gamma) by the definition of u)
        yinv_no0(c.fyg, d02, G[0]);
        yinv(c.fxg, c.fxh, d11, d12, G[1]);  // fxh = fxg / 2
    } else {
        const CT b = c.qinv_r2 * d02;  // K0 = K1 = 0
        G[0][0] = b;
        G[0][1] = CT(-2) * b;
        G[0][2] = b;
        yinv_no0(d11, d12, G[1]);
    }
    yinv(d20, d20h, d21, d22, G[2]);
    // ... then the x-transform back for each row, added to the populations
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const CT K0 = G[0][j], K1 = G[1][j], K2 = G[2][j];
        const CT R1 = K1 + ux * K0;
        const CT R2 = K2 + ux * (K1 + R1);
        q[j][0] += R2 - R1;
        q[j][1] += CT(2) * (K0 - R2);
        q[j][2] += R2 + R1;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = q[QJ[a]][QI[a]];
}

// Changes of k2s, k2d and k11 in the collision of the method as the paper
// runs it (omega_xi = 1), from the non-equilibrium parts n2s, n2d, n11.  The
// strain rates solve the two equations of eq. 46, cbx Dx + cby Dy = R2s and
// csx Dx + csy Dy = R2d (D = rho times the strain rate); with them the
// theta and lambda terms of eq. 38-39 sum to
//   k2s: -(n2s + 2 c2 (Dx + Dy))          (omega_xi = 1)
//   k2d: -2 h_nu (n2d + (2 c2 / omega_nu) (Dx - Dy)),
// so that relaxing with omega_xi = 1 and omega_nu gives the changes
//   d2s = -2 n2s - 2 c2 (Dx + Dy),  d2d = -2 n2d - 4 c2 h_nu (Dx - Dy)
// (the same terms as in corrections(), summed in closed form), returned here
// as their halves h2s = d2s / 2, h2d = d2d / 2 (the changes of k20 and k02
// are their sum and difference).  Only Ds = Dx + Dy and Dm = Dx - Dy are
// needed, so the system is solved for them: its coefficients are linear in
// ux^2 + uy^2 and ux^2 - uy^2.  Products are grouped so that each multiply
// fuses with an add (fewer instructions; the rounding differs from the
// term-by-term sum, within FP32 rounding).
template <typename CT>
__device__ __forceinline__ void increments_plain(const Coef<CT> &c, CT ux, CT uy, CT u2s, CT u2d,
                                                 CT uxy, CT n2s, CT n2d, CT n11, CT gx, CT gy,
                                                 CT &h2s, CT &h2d, CT &d11)
{
    // a Ds + b Dm = R2s, cc Ds + e Dm = R2d with a = (cbx + cby)/2,
    // b = (cbx - cby)/2, cc = (csx + csy)/2, e = (csx - csy)/2, where
    // cbx = (P ux^2 + Q uy^2 + a1)/2 - 2 c2, csx = (P ux^2 - Q uy^2 + a1)/2
    // - 2 c2/omega_nu, likewise along y
    const CT a = c.sPQ * u2s + c.sa0;
    const CT b = c.dPQ * u2d + c.sb0;
    const CT cc = c.sPQ * u2d + c.sc0;
    const CT e = c.dPQ * u2s + c.se0;
    // -e_b = Ab ux gx + Bb uy gy, -e_s = Ab ux gx - Bb uy gy
    const CT tA = c.Ab * ux, tB = c.Bb * uy;
    const CT R2s = n2s - tA * gx - tB * gy;
    const CT R2d = n2d - tA * gx + tB * gy;
    const CT idet = recip(a * e - b * cc);
    const CT Ds = (R2s * e - b * R2d) * idet;
    const CT Dm = (a * R2d - cc * R2s) * idet;
    h2s = -c.c2 * Ds - n2s;
    h2d = -c.c2hnu2 * Dm - n2d;
    // omega_nu (cor11 - n11), cor11 = kq11 uxy Ds + kl11 (uy gx + ux gy)
    d11 = c.okq11 * uxy * Ds + c.okl11 * (uy * gx + ux * gy) - c.om_nu * n11;
}

// The method as the paper runs it (every correction, unit rates for the
// non-hydrodynamic moments, no body force), written for few operations.
// With omega_xi = omega_3 = omega_4 = 1 the post-collision k2s, k21, k12 and
// k22 are their (corrected) equilibria, so no third- or fourth-order central
// moment of f is needed: rho, j and the raw second moments give the second
// central moments (k20 = m20 - rho ux^2, k02 = m02 - rho uy^2,
// k11 = m11 - rho ux uy).  After the collision the first central moments are
// zero and j is unchanged, so the binomial shift back to raw moments has
// closed forms; the change of the raw moments goes back through P^-1 S^-1 and
// is added to the stored deviations (incremental, as in collide()).
template <typename CT>
__device__ __forceinline__ void collide_plain(const Coef<CT> &c, CT d[9], CT gx, CT gy)
{
    CT q[3][3];  // [e_y + 1][e_x + 1]
#pragma unroll
    for (int a = 0; a < 9; ++a) q[QJ[a]][QI[a]] = d[a];
    CT X0[3], X1[3], X2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        X1[j] = q[j][2] - q[j][0];
        X2[j] = q[j][2] + q[j][0];
        X0[j] = X2[j] + q[j][1];
    }
    const CT drho = (X0[0] + X0[1]) + X0[2];
    const CT rho = c.rho0 + drho;
    const CT irho = recip(rho);
    const CT jx = (X1[0] + X1[1]) + X1[2], jy = c.r * (X0[2] - X0[0]);
    const CT ux = jx * irho, uy = jy * irho;
    const CT ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const CT u2s = ux2 + uy2;

    // raw second moments of the deviations (those of rho0 w are rho0 c2,
    // rho0 c2, 0), then the central ones of f minus rho0 c2 (k20, k02), k11
    const CT m20 = (X2[0] + X2[1]) + X2[2];
    const CT m02 = c.r2 * (X0[2] + X0[0]);
    const CT m11 = c.r * (X1[2] - X1[0]);
    const CT k20 = m20 - ux * jx;
    const CT k02 = m02 - uy * jy;
    const CT k11 = m11 - uy * jx;
    const CT k2s = k20 + k02;  // minus 2 c2 rho0
    const CT k2d = k20 - k02;

    // non-equilibrium parts: minus the preconditioned equilibria (eq. 14),
    // e2s = 2 c2 drho + (1/gamma - 1) rho (ux^2 + uy^2) (minus the same
    // constants), e2d = (1/gamma - 1) rho (ux^2 - uy^2), e11 likewise
    const CT u2d = ux2 - uy2;
    const CT irh = c.ig1 * rho;
    const CT n2s = k2s - c.c2x2 * drho - irh * u2s;
    const CT n2d = k2d - irh * u2d;
    const CT n11 = k11 - irh * uxy;

    // changes of the second central moments in the collision, the same as
    // those of the raw second moments
    CT h2s, h2d, d11;
    increments_plain(c, ux, uy, u2s, u2d, uxy, n2s, n2d, n11, gx, gy, h2s, h2d, d11);
    const CT d20 = h2s + h2d, d02 = h2s - h2d;

    // raw third and fourth moments after the collision from the central ones
    // (k21 = g3 rho ux^2 uy, k12 = g3 rho ux uy^2, k22 = c2^2 rho), minus the
    // raw moments before it (those of rho0 w: 0, 0, rho0 c2^2)
    const CT A = (k20 + d20) + c.c2rho0, B = (k02 + d02) + c.c2rho0;  // k20, k02 of f
    const CT K11 = k11 + d11, K2 = K11 + K11;
    const CT rg = c.g3p1 * rho;  // (g3 + 1) rho
    const CT d21 = (uy * (rg * ux2 + A) + ux * K2) - c.r * (X2[2] - X2[0]);
    const CT d12 = (ux * (rg * uy2 + B) + uy * K2) - c.r2 * (X1[2] + X1[0]);
    const CT d22 = (((c.c2sq * drho + (c.g34p1 * rho) * (ux2 * uy2)) + (ux2 * B + uy2 * A)) +
                    CT(4) * uxy * K11) -
                   c.r2 * (X2[2] + X2[0]);

    // f~ = f + P^-1 S^-1 dm (dm00 = dm10 = dm01 = 0): y-transform back for
    // each x-moment, halved (the halves of the x-transform folded in) ...
    // G[m][e_y + 1] for x-moments m: (b0, -2 b0, b0), (b1 - a1, -2 b1, b1 + a1),
    // (b2 - a2, d20 / 2 - 2 b2, b2 + a2)
    const CT b0 = c.qinv_r2 * d02;
    const CT a1 = c.qinv_r * d11, b1 = c.qinv_r2 * d12;
    const CT a2 = c.qinv_r * d21, b2 = c.qinv_r2 * d22;
    // ... then the x-transform back for each row (K0, K1, K2 = G[0..2][row]:
    // changes K2 - K1, 2 (K0 - K2), K2 + K1), added to the populations; the
    // middle row written out so that its factors of 2 fuse
#pragma unroll
    for (int j = 0; j < 3; j += 2) {
        const CT K1 = j == 0 ? b1 - a1 : b1 + a1, K2 = j == 0 ? b2 - a2 : b2 + a2;
        q[j][0] += K2 - K1;
        q[j][1] += CT(2) * (b0 - K2);
        q[j][2] += K2 + K1;
    }
    {
        const CT H = CT(0.5) * d20 - CT(2) * b2;  // K2 of the middle row; K0 = -2 b0, K1 = -2 b1
        q[1][0] += CT(2) * b1 + H;
        q[1][1] += CT(-2) * (CT(2) * b0 + H);
        q[1][2] += CT(-2) * b1 + H;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = q[QJ[a]][QI[a]];
}

// Raw-moment (rest-frame) collision, PRNR-LBM.  Deviations and incremental
// form as in collide(); the raw moments of rho0 w are exactly the constant
// tensor rho0 (1,0,c2)x(1,0,c2), so the raw moments of the deviations are
// those of f minus that tensor, and so are the equilibria written below.
template <typename CT, bool FORCE>
__device__ __forceinline__ void collide_raw(const Coef<CT> &c, CT d[9], CT gx, CT gy)
{
    CT q[3][3];  // [e_y + 1][e_x + 1]
#pragma unroll
    for (int a = 0; a < 9; ++a) q[QJ[a]][QI[a]] = d[a];
    CT X0[3], X1[3], X2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        X1[j] = q[j][2] - q[j][0];
        X2[j] = q[j][2] + q[j][0];
        X0[j] = X2[j] + q[j][1];
    }
    const CT drho = (X0[0] + X0[1]) + X0[2];
    const CT rho = c.rho0 + drho;
    const CT irho = recip(rho);
    CT jx = (X1[0] + X1[1]) + X1[2], jy = c.r * (X0[2] - X0[0]);
    if (FORCE) {
        jx += c.fxh;
        jy += c.fyh;
    }
    const CT ux = jx * irho, uy = jy * irho;
    const CT ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const CT u2s = ux2 + uy2;

    // raw y-moments (lattice speed r) of each raw x-moment
    auto yraw = [&](CT A, CT B, CT Cc, CT &M1, CT &M2) {
        M1 = c.r * (Cc - A);
        M2 = c.r2 * (Cc + A);
        (void)B;
    };
    CT M01, M02, M11, M12, M21, M22;
    yraw(X0[0], X0[1], X0[2], M01, M02);
    yraw(X1[0], X1[1], X1[2], M11, M12);
    yraw(X2[0], X2[1], X2[2], M21, M22);
    (void)M01;
    const CT M20 = (X2[0] + X2[1]) + X2[2];
    const CT m2s = M20 + M02, m2d = M20 - M02;

    // raw equilibria (eq. 12) minus rho0 (1,0,c2)x(1,0,c2)
    const CT igr = c.ig * rho;
    const CT e2s = c.c2x2 * drho + igr * u2s;
    const CT e2d = igr * (ux2 - uy2);
    const CT e11 = igr * uxy;

    CT cor2s, cor2d, cor11;
    corrections<CT>(c, ux, uy, ux2, uy2, uxy, m2s - e2s, m2d - e2d, gx, gy, cor2s, cor2d, cor11);

    CT d2s = c.om_xi * ((e2s + cor2s) - m2s);
    CT d2d = c.om_nu * ((e2d + cor2d) - m2d);
    CT d11 = c.om_nu * ((e11 + cor11) - M11);
    if (FORCE) {
        // raw source moments (eq. 13) with weights 1 - omega/2
        d2s += c.sxi2 * (c.rqfx * ux + c.rqfy * uy);
        d2d += c.snu2 * (c.rqfx * ux - c.rqfy * uy);
        d11 += c.snu * (c.rqfx * uy + c.rqfy * ux);
    }
    const CT d21 = c.om_3 * (rho * (c.c2 * uy + c.igg * ux2 * uy) - M21);
    const CT d12 = c.om_3 * (rho * (c.c2 * ux + c.igg * uy2 * ux) - M12);
    const CT d22 = c.om_4 * ((c.c2sq * drho + rho * (c.c2 * u2s + ux2 * uy2)) - M22);
    const CT d20 = CT(0.5) * (d2s + d2d);
    const CT d02 = CT(0.5) * (d2s - d2d);

    // f~ = f + P^-1 S^-1 dm: y-transform back for each x-moment (the first
    // raw moments change by F/gamma, k00 not at all) ...
    CT G[3][3];  // [x-moment][e_y + 1]
    auto yinv = [&](CT K0, CT K1, CT K2, CT *g) {
        const CT a = c.hinv_r * K1, b = c.hinv_r2 * K2;  // halves
        g[0] = b - a;
        g[1] = K0 - CT(2) * b;
        g[2] = b + a;
    };
    auto yinv_no0 = [&](CT K1, CT K2, CT *g) {  // K0 = 0 (not folded in IEEE)
        const CT a = c.hinv_r * K1, b = c.hinv_r2 * K2;
        g[0] = b - a;
        g[1] = CT(-2) * b;
        g[2] = b + a;
    };
    if (FORCE) {
        yinv_no0(c.fyg, d02, G[0]);
        yinv(c.fxg, d11, d12, G[1]);
    } else {
        const CT b = c.hinv_r2 * d02;  // K0 = K1 = 0
        G[0][0] = b;
        G[0][1] = CT(-2) * b;
        G[0][2] = b;
        yinv_no0(d11, d12, G[1]);
    }
    yinv(d20, d21, d22, G[2]);
    // ... then the x-transform back for each row, added to the populations
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const CT K0 = G[0][j], K1 = G[1][j], K2 = G[2][j];
        const CT h1 = CT(0.5) * K1, h2 = CT(0.5) * K2;
        q[j][0] += h2 - h1;
        q[j][1] += K0 - K2;
        q[j][2] += h2 + h1;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = q[QJ[a]][QI[a]];
}

}  // namespace prc
