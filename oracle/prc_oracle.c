/*
 * FP64 reference ("oracle") for the PRC-LBM of arXiv 2208.03562.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the GPU library, never by it.
 * Shares no code with the HIP library.  See prc_oracle.h for the layout.
 *
 * The per-node collision follows the sub-steps of Appendix A in the paper's
 * order and notation (raw moments eq. 62, scaling S, central moments F(u),
 * relaxation with combine/segregate B, F(-u), S^-1, eq. 72), in full
 * populations and double precision.  Where the paper is silent or
 * self-contradictory the readings used are stated at the point of use:
 *   - eq. 45 (not the appendix's shortened form) for R2s and R2d;
 *   - eq. 38-40 for the correction coefficients (the appendix restatement
 *     carries index slips);
 *   - post-collision segregation k20 = (k2s + k2d)/2, k02 = (k2s - k2d)/2;
 *   - F(-u) maps central to raw moments (the appendix prints the binomial
 *     relations with the two sides swapped);
 *   - moving-wall half-way bounce-back with the wall momentum term taken as
 *     the part of the rest-frame equilibrium that is odd in the velocity,
 *     wall density rho0, the lid correction applied to every link whose
 *     source lies above the lid (top corners included);
 *   - density gradient: the rest-weight-weighted central difference over the
 *     eight neighbours, neighbour index clamped into the domain at walls;
 *   - initial state rho0 times the rest weights, lid moving from step 0.
 */
#include "prc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sec. 2 eq. 3a/3b (e_y in units of r) */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* moment order inside 9-vectors (eq. baremoments-m) */
enum { K00 = 0, K10, K01, K20, K02, K11, K21, K12, K22 };

#define IDX(p, a, i, j) ((size_t)(a) * (size_t)(p)->nx * (size_t)(p)->ny + \
                         (size_t)(j) * (size_t)(p)->nx + (size_t)(i))

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_lattice(double r, double *q, double *c2)
{
    /* eq. 2: c_s = q c_*, q = min(1, r); c_*^2 = 1/3 (eq. 1) */
    double qq = r < 1.0 ? r : 1.0;
    *q = qq;
    *c2 = qq * qq / 3.0;
}

double orc_omega_nu_from_re(const orc_params *p, double re)
{
    /* Re = U H / nu (Sec. 5.1), H = cavity height = ny * dy = ny * r in units
     * of dx; nu = gamma c_s^2 (1/omega_nu - 1/2) (eq. transport-coefficients) */
    double q, c2;
    orc_lattice(p->r, &q, &c2);
    double H = (double)p->ny * p->r;
    double nu = p->u_lid * H / re;
    return 1.0 / (nu / (p->gamma * c2) + 0.5);
}

/* one-dimensional rest weights: variance c2 along x, c2 / r^2 in units of r
 * along y, so that the product has central moments (1,0,0,c2,c2,0,0,0,c2^2) */
static double wx(int e, double c2) { return e == 0 ? 1.0 - c2 : 0.5 * c2; }
static double wy(int e, double c2, double r)
{
    double v = c2 / (r * r);
    return e == 0 ? 1.0 - v : 0.5 * v;
}

void orc_rest_populations(const orc_params *p, double w[9])
{
    double q, c2;
    orc_lattice(p->r, &q, &c2);
    for (int a = 0; a < 9; ++a)
        w[a] = p->rho0 * wx(EX[a], c2) * wy(EY[a], c2, p->r);
}

/* Appendix A, first sub-step (eq. 62): raw moments on the square lattice */
void orc_raw_moments_square(const double f[9], double m[9])
{
    m[K00] = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    m[K10] = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    m[K01] = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    m[K20] = f[1] + f[3] + f[5] + f[6] + f[7] + f[8];
    m[K02] = f[2] + f[4] + f[5] + f[6] + f[7] + f[8];
    m[K11] = f[5] - f[6] + f[7] - f[8];
    m[K21] = f[5] + f[6] - f[7] - f[8];
    m[K12] = f[5] - f[6] - f[7] + f[8];
    m[K22] = f[5] + f[6] + f[7] + f[8];
}

/* Appendix A, second sub-step: m <- S m, S = diag(1,1,r,1,r^2,r,r,r^2,r^2)
 * (eq. S-matrix): k'_mn picks up r^n */
void orc_scale_rect(double r, double m[9])
{
    m[K01] *= r;
    m[K02] *= r * r;
    m[K11] *= r;
    m[K21] *= r;
    m[K12] *= r * r;
    m[K22] *= r * r;
}

/* Appendix A, third sub-step: central moments by the binomial shift F(u)
 * (the explicit bare forms, equal to the definition eq. 9B) */
void orc_central_from_raw(const double m[9], double ux, double uy, double k[9])
{
    k[K00] = m[K00];
    k[K10] = m[K10] - ux * m[K00];
    k[K01] = m[K01] - uy * m[K00];
    k[K20] = m[K20] - 2.0 * ux * m[K10] + ux * ux * m[K00];
    k[K02] = m[K02] - 2.0 * uy * m[K01] + uy * uy * m[K00];
    k[K11] = m[K11] - uy * m[K10] - ux * m[K01] + ux * uy * m[K00];
    k[K21] = m[K21] - 2.0 * ux * m[K11] + ux * ux * m[K01] - uy * m[K20]
           + 2.0 * ux * uy * m[K10] - ux * ux * uy * m[K00];
    k[K12] = m[K12] - 2.0 * uy * m[K11] + uy * uy * m[K10] - ux * m[K02]
           + 2.0 * ux * uy * m[K01] - ux * uy * uy * m[K00];
    k[K22] = m[K22] - 2.0 * ux * m[K12] + ux * ux * m[K02] - 2.0 * uy * m[K21]
           + 4.0 * ux * uy * m[K11] - 2.0 * ux * ux * uy * m[K01]
           + uy * uy * m[K20] - 2.0 * ux * uy * uy * m[K10]
           + ux * ux * uy * uy * m[K00];
}

/* Appendix A, fifth sub-step: raw moments from central ones, F(-u) = F^-1
 * (the appendix prints these relations with left and right sides swapped;
 * here the raw moment is the unknown) */
void orc_raw_from_central(const double k[9], double ux, double uy, double m[9])
{
    m[K00] = k[K00];
    m[K10] = k[K10] + ux * k[K00];
    m[K01] = k[K01] + uy * k[K00];
    m[K20] = k[K20] + 2.0 * ux * k[K10] + ux * ux * k[K00];
    m[K02] = k[K02] + 2.0 * uy * k[K01] + uy * uy * k[K00];
    m[K11] = k[K11] + uy * k[K10] + ux * k[K01] + ux * uy * k[K00];
    m[K21] = k[K21] + 2.0 * ux * k[K11] + ux * ux * k[K01] + uy * k[K20]
           + 2.0 * ux * uy * k[K10] + ux * ux * uy * k[K00];
    m[K12] = k[K12] + 2.0 * uy * k[K11] + uy * uy * k[K10] + ux * k[K02]
           + 2.0 * ux * uy * k[K01] + ux * uy * uy * k[K00];
    m[K22] = k[K22] + 2.0 * ux * k[K12] + ux * ux * k[K02] + 2.0 * uy * k[K21]
           + 4.0 * ux * uy * k[K11] + 2.0 * ux * ux * uy * k[K01]
           + uy * uy * k[K20] + 2.0 * ux * uy * uy * k[K10]
           + ux * ux * uy * uy * k[K00];
}

/* Appendix A, sixth sub-step: m <- S^-1 m (eq. S-matrix-inverse) */
void orc_unscale_rect(double r, double m[9])
{
    m[K01] /= r;
    m[K02] /= r * r;
    m[K11] /= r;
    m[K21] /= r;
    m[K12] /= r * r;
    m[K22] /= r * r;
}

/* Appendix A, seventh sub-step (eq. 72): populations from square-lattice
 * raw moments, f = P^-1 m */
void orc_populations_from_square_raw(const double m[9], double f[9])
{
    f[0] = m[K00] - m[K20] - m[K02] + m[K22];
    f[1] = 0.5 * (m[K10] + m[K20] - m[K12] - m[K22]);
    f[2] = 0.5 * (m[K01] + m[K02] - m[K21] - m[K22]);
    f[3] = 0.5 * (-m[K10] + m[K20] + m[K12] - m[K22]);
    f[4] = 0.5 * (-m[K01] + m[K02] + m[K21] - m[K22]);
    f[5] = 0.25 * (m[K11] + m[K21] + m[K12] + m[K22]);
    f[6] = 0.25 * (-m[K11] + m[K21] - m[K12] + m[K22]);
    f[7] = 0.25 * (m[K11] - m[K21] - m[K12] + m[K22]);
    f[8] = 0.25 * (-m[K11] - m[K21] + m[K12] + m[K22]);
}

void orc_collide_node(const orc_params *p, const double f[9], double drx,
                      double dry, double ft[9], double *diag)
{
    const double r = p->r, g = p->gamma;
    double q, c2;
    orc_lattice(r, &q, &c2);
    const double r2 = r * r;

    /* A.1 and A.2: rectangular raw moments m = S P f */
    double m[9];
    orc_raw_moments_square(f, m);
    orc_scale_rect(r, m);

    /* hydrodynamic fields (eq. hydrodynamicfields), dt = 1 */
    const double rho = m[K00];
    const double ux = (m[K10] + p->fx / (2.0 * g)) / rho;
    const double uy = (m[K01] + p->fy / (2.0 * g)) / rho;
    const double ux2 = ux * ux, uy2 = uy * uy;

    /* A.3: central moments (or, for the raw-moment variant, the raw moments
     * themselves: the collision then happens in the rest frame) */
    const int raw = p->frame == ORC_FRAME_RAW;
    double k[9];
    if (raw)
        memcpy(k, m, sizeof k);
    else
        orc_central_from_raw(m, ux, uy, k);

    /* A.4: collision. Shorthands of the appendix: P_gamma, Q_gamma, U_gamma */
    const double Pg = 4.0 / (g * g) - 1.0 / g;
    const double Qg = 1.0 / (g * g) - 1.0 / g;
    const double Ug = 2.0 / g + 1.0;
    const double ig1 = 1.0 / g - 1.0;
    const double hnu = 1.0 / p->omega_nu - 0.5;
    const double hxi = 1.0 / p->omega_xi - 0.5;

    /* combine the diagonal second-order moments (operator B) */
    const double k2s = k[K20] + k[K02];
    const double k2d = k[K20] - k[K02];

    /* second-order non-equilibrium parts are the same in both frames
     * (Sec. 3.6); eq. 45 with eq. 43 */
    double dxux = 0.0, dyuy = 0.0, R2s = 0.0, R2d = 0.0, det = 0.0;
    if (p->corrections & (ORC_CORR_THETA | ORC_CORR_K11)) {
        const double A = 0.5 * (Ug * c2 - 1.0) * ux;
        const double B = 0.5 * (Ug * c2 - r2) * uy;
        const double eb = -A * drx - B * dry;
        const double es = -A * drx + B * dry;
        /* non-equilibrium parts: subtract the base equilibria of the frame */
        double n2s, n2d;
        if (raw) {
            n2s = k2s - (2.0 * c2 * rho + rho * (ux2 + uy2) / g);
            n2d = k2d - rho * (ux2 - uy2) / g;
        } else {
            n2s = k2s - 2.0 * c2 * rho - ig1 * (ux2 + uy2) * rho;
            n2d = k2d - ig1 * (ux2 - uy2) * rho;
        }
        R2s = n2s + eb;
        R2d = n2d + es;
        /* eq. 46 with omega_3 = omega_xi, omega_4 = omega_nu */
        const double Cbx = (-2.0 * c2 / p->omega_xi + 0.5 * (Pg * ux2 + Qg * uy2)
                            + 0.5 * (3.0 * c2 - 1.0)) * rho;
        const double Cby = (-2.0 * c2 / p->omega_xi + 0.5 * (Pg * uy2 + Qg * ux2)
                            + 0.5 * (3.0 * c2 - r2)) * rho;
        const double Csx = (-2.0 * c2 / p->omega_nu + 0.5 * (Pg * ux2 - Qg * uy2)
                            + 0.5 * (3.0 * c2 - 1.0)) * rho;
        const double Csy = (2.0 * c2 / p->omega_nu + 0.5 * (-Pg * uy2 + Qg * ux2)
                            - 0.5 * (3.0 * c2 - r2)) * rho;
        /* eq. 47 solved as in eq. 48 (no guard: the paper states none) */
        det = Cbx * Csy - Csx * Cby;
        dxux = (Csy * R2s - Cby * R2d) / det;
        dyuy = (R2s - Cbx * dxux) / Cby;
    }

    /* correction coefficients, eq. 38 (bulk), 39 (shear, diagonal),
     * 40 (shear, off-diagonal) */
    const double tbx = -(Pg * ux2 + Qg * uy2 + (3.0 * c2 - 1.0)) * rho * hxi;
    const double tby = -(Pg * uy2 + Qg * ux2 + (3.0 * c2 - r2)) * rho * hxi;
    const double lbx = -(Ug * c2 - 1.0) * hxi * ux;
    const double lby = -(Ug * c2 - r2) * hxi * uy;
    const double tsx = -(Pg * ux2 - Qg * uy2 + (3.0 * c2 - 1.0)) * rho * hnu;
    const double tsy = (-Pg * uy2 + Qg * ux2 - (3.0 * c2 - r2)) * rho * hnu;
    const double lsx = -(Ug * c2 - 1.0) * hnu * ux;
    const double lsy = (Ug * c2 - r2) * hnu * uy;
    const double t11x = -Qg * hnu * rho * ux * uy;
    const double t11y = -Qg * hnu * rho * ux * uy;
    const double l11x = -ig1 * hnu * c2 * uy;
    const double l11y = -ig1 * hnu * c2 * ux;

    double c2s = 0.0, c2d = 0.0, c11 = 0.0;
    if (p->corrections & ORC_CORR_THETA) {
        c2s += tbx * dxux + tby * dyuy;
        c2d += tsx * dxux - tsy * dyuy;
    }
    if (p->corrections & ORC_CORR_LAMBDA) {
        c2s += lbx * drx + lby * dry;
        c2d += lsx * drx + lsy * dry;
    }
    if (p->corrections & ORC_CORR_K11)
        c11 = t11x * dxux + t11y * dyuy + l11x * drx + l11y * dry;

    /* equilibria and sources of the frame, extended by the corrections */
    double eq[9], s[9];
    if (raw) {
        /* eq. 12 and eq. 13 */
        eq[K00] = rho;
        eq[K10] = rho * ux;
        eq[K01] = rho * uy;
        eq[K20] = c2 * rho + rho * ux2 / g;
        eq[K02] = c2 * rho + rho * uy2 / g;
        eq[K11] = rho * ux * uy / g;
        eq[K21] = rho * (c2 + ux2 / (g * g)) * uy;
        eq[K12] = rho * (c2 + uy2 / (g * g)) * ux;
        eq[K22] = rho * c2 * c2 + rho * c2 * (ux2 + uy2) + rho * ux2 * uy2;
        s[K00] = 0.0;
        s[K10] = p->fx / g;
        s[K01] = p->fy / g;
        s[K20] = 2.0 * p->fx * ux / (g * g);
        s[K02] = 2.0 * p->fy * uy / (g * g);
        s[K11] = (p->fx * uy + p->fy * ux) / (g * g);
    } else {
        /* eq. 14 (central equilibria, k22 as chosen below eq. 14) and
         * eq. 13-central */
        eq[K00] = rho;
        eq[K10] = 0.0;
        eq[K01] = 0.0;
        eq[K20] = c2 * rho + ig1 * rho * ux2;
        eq[K02] = c2 * rho + ig1 * rho * uy2;
        eq[K11] = ig1 * rho * ux * uy;
        eq[K21] = (1.0 / (g * g) - 3.0 / g + 2.0) * rho * ux2 * uy;
        eq[K12] = (1.0 / (g * g) - 3.0 / g + 2.0) * rho * ux * uy2;
        eq[K22] = c2 * c2 * rho;
        s[K00] = 0.0;
        s[K10] = p->fx / g;
        s[K01] = p->fy / g;
        s[K20] = Qg * 2.0 * p->fx * ux;
        s[K02] = Qg * 2.0 * p->fy * uy;
        s[K11] = Qg * (p->fx * uy + p->fy * ux);
    }
    s[K21] = s[K12] = s[K22] = 0.0;

    const double eq2s = eq[K20] + eq[K02] + c2s;
    const double eq2d = eq[K20] - eq[K02] + c2d;
    const double eq11 = eq[K11] + c11;
    const double s2s = s[K20] + s[K02];
    const double s2d = s[K20] - s[K02];

    /* relaxation with the rates of Lambda and the source terms (Appendix A,
     * collision sub-step) */
    const double w1 = p->omega_1, wxi = p->omega_xi, wnu = p->omega_nu;
    double kt[9];
    kt[K00] = k[K00];
    kt[K10] = k[K10] + w1 * (eq[K10] - k[K10]) + (1.0 - 0.5 * w1) * s[K10];
    kt[K01] = k[K01] + w1 * (eq[K01] - k[K01]) + (1.0 - 0.5 * w1) * s[K01];
    const double kt2s = k2s + wxi * (eq2s - k2s) + (1.0 - 0.5 * wxi) * s2s;
    const double kt2d = k2d + wnu * (eq2d - k2d) + (1.0 - 0.5 * wnu) * s2d;
    kt[K11] = k[K11] + wnu * (eq11 - k[K11]) + (1.0 - 0.5 * wnu) * s[K11];
    kt[K21] = k[K21] + p->omega_3 * (eq[K21] - k[K21]);
    kt[K12] = k[K12] + p->omega_3 * (eq[K12] - k[K12]);
    kt[K22] = k[K22] + p->omega_4 * (eq[K22] - k[K22]);
    /* segregate (operator B^-1) */
    kt[K20] = 0.5 * (kt2s + kt2d);
    kt[K02] = 0.5 * (kt2s - kt2d);

    /* A.5-A.7: f~ = P^-1 S^-1 F(-u) m~c */
    double mt[9];
    if (raw)
        memcpy(mt, kt, sizeof mt);
    else
        orc_raw_from_central(kt, ux, uy, mt);
    orc_unscale_rect(r, mt);
    orc_populations_from_square_raw(mt, ft);

    if (diag) {
        diag[0] = rho;
        diag[1] = ux;
        diag[2] = uy;
        diag[3] = dxux;
        diag[4] = dyuy;
        diag[5] = R2s;
        diag[6] = R2d;
        diag[7] = det;
    }
}

void orc_equilibrium_node(const orc_params *p, double rho, double ux, double uy,
                          double feq[9])
{
    /* central equilibria of eq. 14 mapped back with F(-u), S^-1, P^-1 */
    const double g = p->gamma;
    double q, c2;
    orc_lattice(p->r, &q, &c2);
    const double ig1 = 1.0 / g - 1.0;
    double k[9];
    k[K00] = rho;
    k[K10] = 0.0;
    k[K01] = 0.0;
    k[K20] = c2 * rho + ig1 * rho * ux * ux;
    k[K02] = c2 * rho + ig1 * rho * uy * uy;
    k[K11] = ig1 * rho * ux * uy;
    k[K21] = (1.0 / (g * g) - 3.0 / g + 2.0) * rho * ux * ux * uy;
    k[K12] = (1.0 / (g * g) - 3.0 / g + 2.0) * rho * ux * uy * uy;
    k[K22] = c2 * c2 * rho;
    double m[9];
    orc_raw_from_central(k, ux, uy, m);
    orc_unscale_rect(p->r, m);
    orc_populations_from_square_raw(m, feq);
}

/* wall momentum term for a population leaving along beta through a wall
 * moving with (uw, 0): rho_w times the part of the equilibrium that is odd
 * in the wall velocity, f^eq_beta - f^eq_opp(beta) at u = (uw, 0) */
static double wall_delta(const orc_params *p, int beta, double uw)
{
    double q, c2;
    orc_lattice(p->r, &q, &c2);
    /* one-dimensional equilibrium factor along x at velocity uw:
     * mean uw, second moment c2 + uw^2 */
    double phx[3];
    phx[0] = 0.5 * (c2 + uw * uw - uw); /* e_x = -1 */
    phx[1] = 1.0 - c2 - uw * uw;        /* e_x =  0 */
    phx[2] = 0.5 * (c2 + uw * uw + uw); /* e_x = +1 */
    int b = beta, o = OPP[beta];
    double fb = phx[EX[b] + 1] * wy(EY[b], c2, p->r);
    double fo = phx[EX[o] + 1] * wy(EY[o], c2, p->r);
    return p->rho0 * (fb - fo);
}

void orc_stream(const orc_params *p, const double *ft, double *f)
{
    const int nx = p->nx, ny = p->ny;
    const int px = p->bc == ORC_BC_PERIODIC || p->bc == ORC_BC_CHANNEL;
    const int py = p->bc == ORC_BC_PERIODIC;
#pragma omp parallel for schedule(static) if ((long)nx * ny > 4096)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int a = 0; a < 9; ++a) {
                /* Appendix A streaming: f_a(x) = f~_a(x - e_a) */
                int si = i - EX[a], sj = j - EY[a];
                if (px) si = (si + nx) % nx;
                if (py) sj = (sj + ny) % ny;
                double v;
                if (si >= 0 && si < nx && sj >= 0 && sj < ny) {
                    v = ft[IDX(p, a, si, sj)];
                } else {
                    /* half-way bounce-back: the population that left this node
                     * along opp(a) comes back along a; a link through the lid
                     * (source above the top row) carries the lid term */
                    int o = OPP[a];
                    v = ft[IDX(p, o, i, j)];
                    if (sj >= ny) v -= wall_delta(p, o, p->u_lid);
                }
                f[IDX(p, a, i, j)] = v;
            }
}

void orc_macros(const orc_params *p, const double *f, double *rho, double *ux,
                double *uy)
{
    /* eq. hydrodynamicfields: rho = sum f, rho u = sum f e + F dt / (2 gamma) */
    const int nx = p->nx, ny = p->ny;
    const double g = p->gamma;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double s = 0.0, jx = 0.0, jy = 0.0;
            for (int a = 0; a < 9; ++a) {
                double v = f[IDX(p, a, i, j)];
                s += v;
                jx += v * EX[a];
                jy += v * EY[a] * p->r;
            }
            size_t n = (size_t)j * nx + i;
            rho[n] = s;
            ux[n] = (jx + p->fx / (2.0 * g)) / s;
            uy[n] = (jy + p->fy / (2.0 * g)) / s;
        }
}

void orc_grad_rho(const orc_params *p, const double *rho, double *gx, double *gy)
{
    /* isotropic second-order central difference (Sec. 3.6, Appendix A):
     * d_x rho = (1/c2) sum_a w_a e_ax rho(x + e_a), likewise along y with
     * e_ay = r * EY; w_a are the rest weights.  Neighbours outside a wall are
     * replaced by the nearest node inside; periodic directions wrap. */
    const int nx = p->nx, ny = p->ny;
    const int px = p->bc == ORC_BC_PERIODIC || p->bc == ORC_BC_CHANNEL;
    const int py = p->bc == ORC_BC_PERIODIC;
    double q, c2;
    orc_lattice(p->r, &q, &c2);
    double w[9];
    for (int a = 0; a < 9; ++a) w[a] = wx(EX[a], c2) * wy(EY[a], c2, p->r);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double sx = 0.0, sy = 0.0;
            for (int a = 1; a < 9; ++a) {
                int ni = i + EX[a], nj = j + EY[a];
                if (px) ni = (ni + nx) % nx;
                else ni = ni < 0 ? 0 : (ni >= nx ? nx - 1 : ni);
                if (py) nj = (nj + ny) % ny;
                else nj = nj < 0 ? 0 : (nj >= ny ? ny - 1 : nj);
                double v = rho[(size_t)nj * nx + ni];
                sx += w[a] * EX[a] * v;
                sy += w[a] * EY[a] * p->r * v;
            }
            gx[(size_t)j * nx + i] = sx / c2;
            gy[(size_t)j * nx + i] = sy / c2;
        }
}

int orc_step(const orc_params *p, double *ft, int64_t nsteps)
{
    const size_t N = (size_t)p->nx * p->ny;
    double *f = malloc(9 * N * sizeof(double));
    double *rho = malloc(N * sizeof(double));
    double *ux = malloc(N * sizeof(double));
    double *uy = malloc(N * sizeof(double));
    double *gx = malloc(N * sizeof(double));
    double *gy = malloc(N * sizeof(double));
    if (!f || !rho || !ux || !uy || !gx || !gy) {
        free(f); free(rho); free(ux); free(uy); free(gx); free(gy);
        return -4;
    }
    const int nx = p->nx, ny = p->ny;
    for (int64_t t = 0; t < nsteps; ++t) {
        /* streaming, then the hydrodynamic fields of the streamed state
         * (Appendix A, last two sub-steps), which the next collision uses */
        orc_stream(p, ft, f);
        orc_macros(p, f, rho, ux, uy);
        orc_grad_rho(p, rho, gx, gy);
#pragma omp parallel for schedule(static) if ((long)nx * ny > 4096)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double fn[9], fo[9];
                for (int a = 0; a < 9; ++a) fn[a] = f[IDX(p, a, i, j)];
                size_t n = (size_t)j * nx + i;
                orc_collide_node(p, fn, gx[n], gy[n], fo, NULL);
                for (int a = 0; a < 9; ++a) ft[IDX(p, a, i, j)] = fo[a];
            }
    }
    free(f); free(rho); free(ux); free(uy); free(gx); free(gy);
    return 0;
}

int orc_velocity(const orc_params *p, const double *ft, double *rho, double *ux,
                 double *uy)
{
    const size_t N = (size_t)p->nx * p->ny;
    double *f = malloc(9 * N * sizeof(double));
    if (!f) return -4;
    orc_stream(p, ft, f);
    orc_macros(p, f, rho, ux, uy);
    free(f);
    return 0;
}

int orc_residual(const orc_params *p, const double *ft, double *ux_prev,
                 double *uy_prev, double out[4])
{
    /* velocity residual between checks (Sec. 5.2 uses the L2 norm of the
     * change of u over a fixed number of steps); here both components,
     * normalised by the L2 norm of u, plus the total mass */
    const size_t N = (size_t)p->nx * p->ny;
    double *rho = malloc(N * sizeof(double));
    double *ux = malloc(N * sizeof(double));
    double *uy = malloc(N * sizeof(double));
    if (!rho || !ux || !uy) {
        free(rho); free(ux); free(uy);
        return -4;
    }
    orc_velocity(p, ft, rho, ux, uy);
    double sn = 0.0, sd = 0.0, sm = 0.0, mx = 0.0;
    for (size_t n = 0; n < N; ++n) {
        double dx = ux[n] - ux_prev[n], dy = uy[n] - uy_prev[n];
        double u2 = ux[n] * ux[n] + uy[n] * uy[n];
        sn += dx * dx + dy * dy;
        sd += u2;
        sm += rho[n];
        if (!(u2 <= mx)) mx = u2; /* propagates NaN */
        ux_prev[n] = ux[n];
        uy_prev[n] = uy[n];
    }
    out[0] = sn;
    out[1] = sd;
    out[2] = sm;
    out[3] = mx;
    free(rho); free(ux); free(uy);
    return 0;
}

int orc_solve(const orc_params *p, double *ft, double tol, int64_t check_every,
              int64_t max_steps, int64_t *steps_out, double *hist,
              int64_t hist_cap, int64_t *hist_len)
{
    if (check_every <= 0 || max_steps < 0) return -1;
    const size_t N = (size_t)p->nx * p->ny;
    double *rho = malloc(N * sizeof(double));
    double *uxp = malloc(N * sizeof(double));
    double *uyp = malloc(N * sizeof(double));
    if (!rho || !uxp || !uyp) {
        free(rho); free(uxp); free(uyp);
        return -4;
    }
    orc_velocity(p, ft, rho, uxp, uyp);
    int64_t n = 0, nh = 0;
    int status = 1;
    while (n + check_every <= max_steps) {
        orc_step(p, ft, check_every);
        n += check_every;
        double out[4];
        orc_residual(p, ft, uxp, uyp, out);
        /* a NaN in either sum makes R non-finite (diverged), never 0 */
        double R = out[1] > 0.0 ? sqrt(out[0] / out[1])
                                : (out[1] == 0.0 && out[0] == 0.0 ? 0.0 : INFINITY);
        if (hist && nh < hist_cap) hist[nh] = R;
        ++nh;
        if (!isfinite(R) || !isfinite(out[2]) || !(out[3] < 1.0)) {
            status = -3;
            break;
        }
        if (R < tol) {
            status = 0;
            break;
        }
    }
    if (status == 1 && n < max_steps) {
        orc_step(p, ft, max_steps - n);
        n = max_steps;
    }
    *steps_out = n;
    if (hist_len) *hist_len = nh;
    free(rho); free(uxp); free(uyp);
    return status;
}
