/*
 * FP64 reference ("oracle") for the preconditioned rectangular central-moment
 * lattice Boltzmann method (PRC-LBM) of Yahia & Premnath, arXiv 2208.03562.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; it is
 * called from the test suite, from the smoke check and from the CPU-baseline
 * leg of the benchmark, and from nothing else.  It shares no code, header,
 * table or constant with the HIP library and includes nothing from it.
 *
 * Everything is plain double precision, written for a reader to check against
 * the paper by eye: one function per algorithmic step, no blocking, no fusion.
 * Populations are stored as full values f_alpha (not deviations), in dense
 * arrays laid out [alpha][j][i] with i in [0,nx) along x and j in [0,ny) along y.
 *
 * Velocity ordering (Sec. 2, eq. 3a/3b): alpha = 0 rest, 1 E, 2 N, 3 W, 4 S,
 * 5 NE, 6 NW, 7 SW, 8 SE; e_x in {0,+-1}, e_y = r * (0,+-1).
 */
#ifndef PRC_ORACLE_H
#define PRC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_CAVITY = 0, ORC_BC_PERIODIC = 1, ORC_BC_CHANNEL = 2 };

/* correction switches (tests only; the method uses all of them) */
enum { ORC_CORR_THETA = 1,   /* velocity-gradient terms of k2s/k2d (eq. 38, 39) */
       ORC_CORR_LAMBDA = 2,  /* density-gradient terms of k2s/k2d (eq. 38, 39) */
       ORC_CORR_K11 = 4,     /* both correction terms of k11 (eq. 40) */
       ORC_CORR_ALL = 7 };

/* collision frame: the paper's central-moment scheme (Sec. 4.2) or the
 * raw-moment variant it compares against (Sec. 4.1, Sec. 6) */
enum { ORC_FRAME_CENTRAL = 0, ORC_FRAME_RAW = 1 };

typedef struct {
    int32_t nx, ny;
    double r;          /* grid aspect ratio dy/dx (Sec. 2) */
    double gamma;      /* preconditioning parameter (eq. 6) */
    double omega_nu;   /* shear rate: k2d and k11 */
    double omega_xi;   /* bulk rate: k2s */
    double omega_1;    /* first-order central moments */
    double omega_3;    /* k21, k12 */
    double omega_4;    /* k22 */
    double u_lid;      /* lid velocity along +x at the top wall */
    double fx, fy;     /* uniform body force */
    double rho0;       /* reference density (initial state, wall density) */
    int32_t bc;        /* ORC_BC_* */
    int32_t corrections; /* ORC_CORR_* bitmask */
    int32_t frame;     /* ORC_FRAME_* */
} orc_params;

/* number of per-node diagnostics written by orc_collide_node */
#define ORC_NDIAG 8

/* threads the loops over nodes may use (OpenMP), 1 without OpenMP */
int orc_threads(void);
/* Threads the parallel loops use from now on (n > 0; no effect without OpenMP). */
void orc_set_threads(int n);

/* Sec. 2, eq. 2: q = min(1, r), c_s^2 = q^2 c_*^2 with c_*^2 = 1/3 */
void orc_lattice(double r, double *q, double *c2);

/* Sec. 5 (Re = U H / nu) with eq. transport-coefficients:
 * shear relaxation rate for a cavity of height H = ny * r */
double orc_omega_nu_from_re(const orc_params *p, double re);

/* rest state rho0 * w_alpha (product of the two one-dimensional rest weights) */
void orc_rest_populations(const orc_params *p, double w[9]);

/* Appendix A transforms (each one algorithmic sub-step) */
void orc_raw_moments_square(const double f[9], double m[9]);          /* eq. 62 */
void orc_scale_rect(double r, double m[9]);                           /* S      */
void orc_central_from_raw(const double m[9], double ux, double uy, double k[9]);   /* F(u)  */
void orc_raw_from_central(const double k[9], double ux, double uy, double m[9]);  /* F(-u) */
void orc_unscale_rect(double r, double m[9]);                         /* S^-1   */
void orc_populations_from_square_raw(const double m[9], double f[9]); /* eq. 72 */

/* one node's collision: f -> f~ given the density gradient at the node.
 * diag (may be NULL): rho, ux, uy, dxux, dyuy, R2s, R2d, det */
void orc_collide_node(const orc_params *p, const double f[9], double drho_dx,
                      double drho_dy, double ft[9], double *diag);

/* equilibrium populations for given (rho, u) with zero gradients: the
 * post-collision state of a collision with every rate equal to one */
void orc_equilibrium_node(const orc_params *p, double rho, double ux, double uy,
                          double feq[9]);

/* streaming with boundaries: f(x) = f~(x - e_alpha), arrays [9][ny][nx] */
void orc_stream(const orc_params *p, const double *ft, double *f);

/* hydrodynamic fields of streamed populations */
void orc_macros(const orc_params *p, const double *f, double *rho, double *ux,
                double *uy);

/* density gradient from the rho field (isotropic second-order stencil) */
void orc_grad_rho(const orc_params *p, const double *rho, double *gx, double *gy);

/* advance nsteps time steps; ft holds post-collision populations in and out */
int orc_step(const orc_params *p, double *ft, int64_t nsteps);

/* fields of the state ft (streams first, then takes moments) */
int orc_velocity(const orc_params *p, const double *ft, double *rho, double *ux,
                 double *uy);

/* residual sums against a velocity snapshot, then refreshes the snapshot:
 * out = { sum |u-u_prev|^2, sum |u|^2, sum rho, max |u|^2 } */
int orc_residual(const orc_params *p, const double *ft, double *ux_prev,
                 double *uy_prev, double out[4]);

/* run until the relative velocity residual over check_every steps drops
 * below tol (0: converged, 1: step limit, -3: diverged, -1: bad input) */
int orc_solve(const orc_params *p, double *ft, double tol, int64_t check_every,
              int64_t max_steps, int64_t *steps_out, double *hist,
              int64_t hist_cap, int64_t *hist_len);

#ifdef __cplusplus
}
#endif

#endif
