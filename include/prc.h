/*
 * prc.h -- C ABI of the MI355X (gfx950) library for the preconditioned
 * rectangular central-moment lattice Boltzmann method (PRC-LBM) of
 * E. Yahia and K. N. Premnath, arXiv 2208.03562.
 *
 * The library solves the preconditioned Navier-Stokes equations (Sec. 3,
 * eq. 5-6) on a two-dimensional rectangular D2Q9 grid with aspect ratio
 * r = dy/dx (Sec. 2).  One time step is the algorithm of Appendix A: central
 * moments, relaxation to gamma-preconditioned equilibria extended by the
 * grid-anisotropy and cubic-velocity corrections (Sec. 3.5, eq. 38-40) whose
 * velocity gradients come from non-equilibrium moments (Sec. 3.6, eq. 41-48),
 * back to populations, then streaming with no-slip walls and a moving lid.
 *
 * Conventions for every entry point:
 *  - Every call returns prc_status; nothing throws across the ABI.  On an
 *    error, prc_last_error() returns a message for the calling thread.
 *  - All state buffers are device memory allocated and owned by the caller;
 *    the single-problem calls keep no pointer after they return and allocate
 *    no device memory of their own, except the cached launch graphs of
 *    prc_step (until prc_release_graphs or process exit), the scratch
 *    states prc_tune allocates and frees within the call, and, on a device
 *    where the resident sweep (tile 9) runs, its counters and exchange
 *    buffer (about 28 MB, allocated and cleared once), an 8-byte pinned host
 *    word and an event, kept until prc_release_resident or process exit.
 *    Process-wide state besides: the tile choices of prc_tune/prc_set_tile
 *    and the mode of prc_set_streamed.  A batch owns its
 *    small tables and graphs until prc_batch_destroy; prc_serve allocates its
 *    request pool for the duration of the call.
 *  - Calls are ordered on the HIP stream passed in (0 = null stream) and are
 *    asynchronous unless stated otherwise.
 *  - Arguments are validated on the host before anything is launched;
 *    invalid input returns PRC_EINVAL and launches nothing.
 *
 * State layout ("population state"): nine planes, plane a holding
 * population a in the velocity order of Sec. 2 eq. 3a/3b
 * (0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE).  Element (a, j, i)
 * -- node i along x in [0, nx), row j along y in [0, ny) -- sits at element
 * offset a * plane_stride + j * row_stride + i, with both strides from
 * prc_layout(); rows are padded to 256 bytes.  Elements not addressed by any
 * (a, j, i) are padding that the kernels never read.
 * The stored value is the DEVIATION f_a - rho0 * w_a of the post-collision
 * population from the rest state (w_a: product of the one-dimensional rest
 * weights of variance c_s^2 along x and c_s^2 / r^2 along y, c_s^2 = q^2/3,
 * q = min(1, r), eq. 2), in the element type given by prc_params.storage.
 * A buffer of all zeros is the fluid at rest with density rho0.
 */
#ifndef PRC_H
#define PRC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PRC_OK = 0,
    PRC_NOT_CONVERGED = 1, /* step limit reached; not an error */
    PRC_EINVAL = -1,       /* invalid argument; nothing launched */
    PRC_EHIP = -2,         /* a HIP call failed; message has hipGetErrorString */
    PRC_EDIVERGED = -3,    /* non-finite residual/mass or |u| >= 1 */
    PRC_ENOMEM = -4        /* host allocation failed */
} prc_status;

typedef enum {
    PRC_BC_CAVITY = 0,   /* walls on all four sides, lid on top (y = ny r) */
    PRC_BC_PERIODIC = 1, /* periodic in x and y */
    PRC_BC_CHANNEL = 2   /* periodic in x; wall at y = 0, lid at y = ny r */
} prc_bc;

typedef enum {
    PRC_F64 = 0,  /* double deviations, double arithmetic */
    PRC_F32 = 1,  /* float deviations, float arithmetic */
    PRC_F16 = 2,  /* IEEE half deviations, float arithmetic */
    PRC_BF16 = 3  /* bfloat16 deviations, float arithmetic */
} prc_storage;

typedef enum {
    PRC_CORR_THETA = 1,  /* velocity-gradient terms of k2s, k2d (eq. 38, 39) */
    PRC_CORR_LAMBDA = 2, /* density-gradient terms of k2s, k2d (eq. 38, 39) */
    PRC_CORR_K11 = 4,    /* correction terms of k11 (eq. 40) */
    PRC_CORR_ALL = 7     /* the method; the others exist for tests */
} prc_corrections;

typedef enum {
    PRC_FRAME_CENTRAL = 0, /* PRC-LBM: relax central moments (Sec. 4.2) */
    PRC_FRAME_RAW = 1      /* PRNR-LBM: relax raw moments (Sec. 4.1, Sec. 6) */
} prc_frame;

/* Problem description (Sec. 2-5).  Lattice units: dx = dt = 1, dy = r. */
typedef struct {
    int32_t nx, ny;     /* nodes along x and y, each >= 3 */
    double r;           /* grid aspect ratio dy/dx > 0 (Sec. 2) */
    double gamma;       /* preconditioning parameter, 0 < gamma <= 1 (eq. 6) */
    double omega_nu;    /* shear relaxation rate: k2d, k11 (Appendix A) */
    double omega_xi;    /* bulk relaxation rate: k2s; the paper uses 1 */
    double omega_1;     /* first-order central moments; the paper uses 1 */
    double omega_3;     /* k21, k12; the paper uses 1 */
    double omega_4;     /* k22; the paper uses 1 */
    double u_lid;       /* lid velocity along +x; |u_lid| < q / sqrt(3) */
    double fx, fy;      /* uniform body force (eq. 6) */
    double rho0;        /* reference density: rest state and wall density */
    int32_t bc;         /* prc_bc */
    int32_t storage;    /* prc_storage */
    int32_t corrections;/* prc_corrections bitmask, normally PRC_CORR_ALL */
    int32_t frame;      /* prc_frame, normally PRC_FRAME_CENTRAL */
} prc_params;

/* Fill *p with the method's defaults: rates omega_xi = omega_1 = omega_3 =
 * omega_4 = 1 (Appendix A, below the relaxation sub-step), omega_nu = 1,
 * gamma = 1, r = 1, rho0 = 1, no lid, no force, cavity, FP32 storage, all
 * corrections, central frame; nx, ny must still be set.  Host only. */
prc_status prc_params_default(prc_params *p);

/* Set p->omega_nu from the Reynolds number Re = U H / nu of Sec. 5 with the
 * cavity height H = ny * r (units of dx) and U = p->u_lid, inverting
 * nu = gamma q^2 c_*^2 (1/omega_nu - 1/2) (eq. transport-coefficients).
 * EINVAL if re <= 0, u_lid == 0 or the resulting omega_nu is not in (0, 2).
 * Host only. */
prc_status prc_params_from_re(prc_params *p, double re);

/* Check *p against the rules above without touching the GPU. Host only. */
prc_status prc_validate(const prc_params *p);

/* Element strides of the population state (see the layout above): from one
 * row to the next and from one population plane to the next.  Host only. */
prc_status prc_layout(const prc_params *p, int64_t *row_stride, int64_t *plane_stride);

/* Bytes of one population state buffer (at most 4 GiB: larger grids are
 * rejected by validation); 0 if *p is invalid. */
size_t prc_state_bytes(const prc_params *p);

/* Bytes of the scratch buffer that prc_residual and prc_solve need. */
size_t prc_scratch_bytes(const prc_params *p);

/* Write the rest state (all deviations zero, Sec. 5: fluid at rest with
 * density rho0) into f, padding included.  f: device, prc_state_bytes. */
prc_status prc_init(const prc_params *p, void *f, hipStream_t stream);

/* Advance nsteps >= 0 time steps of Appendix A.  Each step reads one state
 * buffer and writes the other: step k (k = 0, 1, ...) reads f_a when k is
 * even and f_b when k is odd, so after nsteps steps the newest state is in
 * f_a when nsteps is even and in f_b when it is odd (the other buffer holds
 * an earlier state; the resident sweep, which keeps the state in LDS between
 * steps, may leave it as it was).  Resident-sweep launches on one device
 * share its exchange buffer and need every compute unit: a launch on another
 * stream than the device's latest resident launch first waits for that one
 * (an event), so calls on several streams run one after the other.  Launches
 * captured into a graph are not ordered this way: replays of such graphs on
 * one device must not overlap.  A launch that nevertheless loses a
 * workgroup's wait (its state is then invalid) is reported by the next
 * prc_step, prc_macros, prc_residual, prc_solve or prc_resident_status on
 * the device (PRC_EHIP), before anything else runs.  One step = streaming
 * with boundaries (Appendix A, "stream"; moving-wall bounce-back as noted at
 * the end of Appendix A), the hydrodynamic fields of the streamed state
 * (eq. hydrodynamicfields), the density gradient, and the collision.  f_a and
 * f_b: distinct device buffers of prc_state_bytes, 256-byte aligned. */
prc_status prc_step(const prc_params *p, void *f_a, void *f_b, int64_t nsteps,
                    hipStream_t stream);

/* prc_step, timed: start and stop (events created by the caller, e.g. with
 * hipEventCreate; timing enabled) are recorded on `stream` before and after
 * the call's work; for the resident sweep stop is recorded by its last
 * launch itself (hipExtLaunchKernel), when that kernel ends.  With
 * kernel_only set, the resident sweep's dispatch records both: start when
 * the first launch of the call begins, stop when its last launch ends, so
 * hipEventElapsedTime gives kernel time alone (as a kernel trace reports it;
 * such a launch takes longer to dispatch); other shapes, and any call under
 * graph capture, record them around the call either way.  PRC_EINVAL if
 * either event is NULL. */
prc_status prc_step_timed(const prc_params *p, void *f_a, void *f_b, int64_t nsteps,
                          hipEvent_t start, hipEvent_t stop, int32_t kernel_only,
                          hipStream_t stream);

/* Convergence check (Sec. 5.2: L2 norm of the change of the velocity between
 * checks).  Computes, in double precision, from the fields of state f:
 *   out[0] = sum_nodes |u - u_prev|^2     out[1] = sum_nodes |u|^2
 *   out[2] = sum_nodes rho                out[3] = max_nodes |u|^2
 * then overwrites u_prev with u.  The relative residual is
 * sqrt(out[0] / out[1]).  u_prev: device double[2][ny][nx] (u_x plane, then
 * u_y plane); scratch: device, prc_scratch_bytes; out: host double[4].
 * Synchronises the stream.  The sums are reproduced bit for bit run to run.
 * Returns PRC_EHIP (and clears the report) if a resident sweep on this device
 * gave up waiting for a neighbouring subdomain since the last report (every
 * subdomain must have a compute unit at once; the state is then invalid). */
prc_status prc_residual(const prc_params *p, const void *f, double *u_prev,
                        void *scratch, double out[4], hipStream_t stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: graph-free serving loops, harnesses that forbid allocation):
 * prc_residual without the scratch argument.  Same sums, same order, same
 * results bit for bit, same u_prev update, same synchronisation and errors;
 * the block partials and the result live in a static device array of
 * 4 * 1024 + 4 doubles (32 KiB + 32 bytes) that the library holds on every
 * device it runs on until the process ends.  That array takes the largest
 * partition of any valid problem, so no valid problem exceeds it (the call
 * still checks and returns PRC_EINVAL if one did).  The call allocates
 * nothing: it launches two kernels, copies 32 bytes to `out` and
 * synchronises the stream.  Calls on one device share the array, so calls
 * that overlap in time on one device (several threads or streams at once)
 * race and may return each other's sums; every call overwrites all it reads,
 * so nothing needs clearing between calls.  u_prev: device
 * double[2][ny][nx]; out: host double[4] (as prc_residual). */
prc_status prc_residual_noalloc(const prc_params *p, const void *f, double *u_prev,
                                double out[4], hipStream_t stream);

/* The state f of problem *p (storage p->storage) in storage type storage_to,
 * written to f_to (device, prc_state_bytes of *p with storage_to, 256-byte
 * aligned, distinct from f), each in its own layout.  Deviations stay
 * deviations; widening (FP16/BF16 -> FP32 -> FP64) is exact, narrowing
 * rounds to nearest.  This is how a run started in 16-bit storage continues
 * in FP32 once the 16-bit residual has reached its floor: the velocity
 * snapshot of prc_residual does not depend on the storage and carries over.
 * Padding of f_to is not written. */
prc_status prc_convert(const prc_params *p, const void *f, int32_t storage_to, void *f_to,
                       hipStream_t stream);

/* Add drho * w_a to every population deviation of state f (w_a the rest
 * weights of the layout notes above): the density of every node changes by
 * drho and nothing else does (no momentum, the second moments of a fluid at
 * rest).  The collision conserves mass exactly, so a run keeps the mass it
 * starts with; rounding to 16-bit storage does not, and a run that goes on
 * in FP32 after a 16-bit phase restores the initial mass this way (drho =
 * (initial mass - mass) / (nx ny), the mass from prc_residual). */
prc_status prc_add_density(const prc_params *p, void *f, double drho, hipStream_t stream);

/* Hydrodynamic fields of state f (eq. hydrodynamicfields after streaming):
 * rho, u_x, u_y as device double[ny][nx] arrays (row j at offset j * nx).
 * Any of the three output pointers may be NULL. */
prc_status prc_macros(const prc_params *p, const void *f, double *rho,
                      double *ux, double *uy, hipStream_t stream);

/* Run from the state in f_a until the relative residual over check_every
 * steps falls below tol, or max_steps is reached.  u_prev is first set from
 * the initial state; after every check_every steps prc_residual is taken and
 * its relative residual appended to hist (host double[hist_cap]; may be NULL).
 * The newest state is in f_a when *steps_out is even, else in f_b.
 * Returns PRC_OK (converged), PRC_NOT_CONVERGED, or PRC_EDIVERGED when a
 * residual or the mass is not finite or max |u| >= 1 (lattice speed).
 * Synchronises the stream at every check. */
prc_status prc_solve(const prc_params *p, void *f_a, void *f_b, double *u_prev,
                     void *scratch, double tol, int64_t check_every,
                     int64_t max_steps, int64_t *steps_out, double *hist,
                     int64_t hist_cap, int64_t *hist_len, hipStream_t stream);

/* Autotuner: time every tile shape of the sweep kernel (threads along x by
 * along y: 0 = 64 x 4, 1 = 64 x 8, 2 = 128 x 4, 3 = 32 x 8, 4 = 32 x 16, one
 * time step per launch; 5 = 64 x 8, 6 = 32 x 16, 7 = 64 x 16, 8 = 32 x 32, two
 * time steps per launch with the intermediate state in LDS; 9 = the resident
 * sweep, 64 x 32-node subdomains of 1024 threads, one per compute unit, that
 * keep the state in LDS for all the steps of a prc_step call and exchange
 * only their edges through memory -- FP32 and 16-bit storage on grids of at
 * most one subdomain per compute unit, a periodic side a multiple of the
 * subdomain; see prc_tile_info) for this problem's storage,
 * boundaries and grid size, on two scratch state buffers that the call
 * allocates and frees itself (hipMalloc/hipFree; timing the resident sweep
 * also sets up its per-device counters and exchange buffer, which stay), and
 * use the fastest (per time step) for
 * every later sweep of a problem with the same storage, boundaries and grid
 * size in this process.  The tile shape changes only the speed, not the
 * results.  tile_out (host, may be NULL) receives the chosen index.  Without
 * a tuning call the library picks, for grids at least 256 x 64 nodes, the
 * resident sweep (9) where it can run the problem, else a
 * two-step shape: 64 x 16 (7) for FP32 when the two states fit 160 MB and for
 * 16-bit storage, 32 x 32 (8) for larger FP32 states, 64 x 8 (5) for FP64
 * states that fit 160 MB and 32 x 16 (6) for larger ones; for smaller grids
 * 128 x 4 (2) when at least 256 nodes wide and 64 x 4 (0) otherwise.  The environment variable PRC_TILE, read once, forces a shape
 * where it is allowed.  Synchronises the stream; PRC_EHIP if the scratch
 * allocation fails. */
prc_status prc_tune(const prc_params *p, int32_t *tile_out, hipStream_t stream);

/* Shape of tile index `tile` (0 .. 9): threads along x and y (for the
 * resident sweep, 9: nodes of a subdomain) and time steps per launch (0 for
 * the resident sweep: any number).  A two-step launch computes the
 * intermediate step on the tile plus two rings in LDS (temporal blocking, for
 * states that fit the cache or to halve the state traffic); its results, and
 * the resident sweep's, are bit for bit those of single steps.  Any output
 * pointer may be NULL.  Host only. */
prc_status prc_tile_info(int32_t tile, int32_t *tx, int32_t *ty, int32_t *steps);

/* Use tile shape `tile` (index as for prc_tune; -1 forgets any choice) for
 * problems with this storage, boundaries and grid size.  Host only; launches
 * nothing (for the resident sweep it reads the current device's compute
 * units and LDS size, and fails without a device or where the problem does
 * not fit).  Launch graphs already cached by prc_step keep the shape they
 * were captured with until prc_release_graphs. */
prc_status prc_set_tile(const prc_params *p, int32_t tile);

/* Drop the launch graphs cached by prc_step (they hold no user memory).
 * Waits for the devices they were captured on to finish their work first
 * (a replay may still be running).  A graph that another thread is
 * replaying at that moment is destroyed once that call has enqueued it. */
prc_status prc_release_graphs(void);

/* Free the current device's resident-sweep counters, exchange buffer,
 * pinned report word and ordering event (see the conventions above), after
 * synchronising the device.  The next resident launch on the device sets
 * them up again.  PRC_OK when nothing was set up. */
prc_status prc_release_resident(void);

/* Whether a resident-sweep launch on the current device lost a workgroup's
 * wait (a subdomain that got no compute unit while its neighbours waited for
 * it; its state is invalid) since the last report: PRC_EHIP, once per
 * report, else PRC_OK.  Reads a pinned host word that the failing launch
 * writes: it does not synchronise, so a launch still running is reported
 * only by a later call (prc_step, prc_macros, prc_residual and prc_solve
 * make the same check themselves before launching or after synchronising). */
prc_status prc_resident_status(void);

/* How long a workgroup of a later resident launch (in this process) waits
 * for a neighbour's value before it gives up and the launch is reported as
 * failed: ticks of the GPU's 100 MHz real-time clock, -1 for the default
 * (2^26 ticks, about 0.67 s; a neighbour that has a compute unit delivers
 * within microseconds).  A small value makes launches fail on purpose, for
 * tests of the report.  PRC_EINVAL below -1.  Host only. */
prc_status prc_set_resident_wait(int64_t ticks);

/* Cache policy for the two state buffers of every later sweep in the
 * process: -1 (default) by size (non-temporal stores, and the load order of
 * the 1024-thread two-step tiles meant for states streamed from HBM, when
 * the two states exceed 160 MB), 0 never, 1 always.  Changes speed only,
 * never a result; cached launch graphs keep the mode they were captured
 * with.  PRC_EINVAL for another value.  Host only. */
prc_status prc_set_streamed(int32_t mode);

/* ---- Batches: many independent problems advanced together -------------
 *
 * The collision and streaming of Appendix A are local to a node and its
 * neighbours, so problems of different sizes and parameters (grid, r, gamma,
 * Re, lid) can share one launch per time step: a batch keeps a list of the
 * tiles of all its members and sweeps them together, which fills the GPU
 * with problems far too small to fill it alone.  Every member gets exactly
 * the arithmetic of prc_step / prc_residual / prc_solve on its own: its
 * states and residuals are bit for bit those of the same problem run alone.
 *
 * All members of a batch share one storage type and one boundary type.  A
 * member's state buffers, u_prev and their memory stay owned by the caller
 * and must stay valid while it is a member.  Between calls the newest state
 * of every member is in its f_a (all steps are taken in even numbers).
 * The batch object owns small device tables (tile and reduction lists) and
 * launch graphs, allocated on first use and freed by prc_batch_destroy.
 * A batch is not thread safe: one thread and one stream at a time.
 */
typedef struct prc_batch prc_batch;

/* Status of a member after prc_batch_solve. */
typedef enum {
    PRC_MEMBER_ACTIVE = 2,      /* still being advanced */
    PRC_MEMBER_CONVERGED = 0,   /* relative residual fell below tol */
    PRC_MEMBER_MAX_STEPS = 1,   /* step limit reached without converging */
    PRC_MEMBER_DIVERGED = -3,   /* non-finite residual or mass, or max |u| >= 1 */
    PRC_MEMBER_REMOVED = -5     /* taken out by prc_batch_remove */
} prc_member_status;

/* Create an empty batch for problems with this storage (prc_storage) and
 * boundary type (prc_bc).  Host only. */
prc_status prc_batch_create(int32_t storage, int32_t bc, prc_batch **out);

/* Free the batch's own tables and graphs (not the members' buffers).
 * Synchronises the device if anything was allocated.  NULL is a no-op. */
prc_status prc_batch_destroy(prc_batch *b);

/* Add a problem.  p must pass prc_validate and match the batch's storage and
 * boundary type.  f_a (holding the current state), f_b: distinct device
 * buffers of prc_state_bytes(p), 256-byte aligned; u_prev: device
 * double[2][ny][nx].  The member joins the next prc_batch_step or
 * prc_batch_solve; prc_batch_solve first takes its velocity snapshot, as
 * prc_solve does.  *id_out receives the member's id: 0, 1, 2, ... in order
 * of addition, never reused.  Host only. */
prc_status prc_batch_add(prc_batch *b, const prc_params *p, void *f_a, void *f_b,
                         double *u_prev, int32_t *id_out);

/* Take member id out of the batch (its buffers are no longer touched by
 * later calls).  Host only. */
prc_status prc_batch_remove(prc_batch *b, int32_t id);

/* Number of members added so far (ids 0 .. n-1) and of active members. */
prc_status prc_batch_count(const prc_batch *b, int32_t *n_added, int32_t *n_active);

/* Advance every active member by nsteps (even, >= 0) time steps: one sweep
 * launch per step and variant (members with every correction and no body
 * force, and the others) covers all of their tiles.  Long runs replay
 * captured graphs.  Asynchronous on stream. */
prc_status prc_batch_step(prc_batch *b, int64_t nsteps, hipStream_t stream);

/* Convergence check of every active member, as prc_residual (same sums, same
 * order, same update of u_prev): out[4 * id + k] for each active id (host,
 * double[4 * n_added]; other entries untouched).  Synchronises the stream. */
prc_status prc_batch_residual(prc_batch *b, double *out, hipStream_t stream);

/* Solve every active member as prc_solve would, side by side: snapshot the
 * velocity of members that have none yet, then repeat { advance all active
 * members check_every (even) steps; check all }; after each check a member
 * leaves the batch as CONVERGED (relative residual < tol), DIVERGED, or
 * MAX_STEPS once it has taken max_steps (a multiple of check_every) steps.
 * Returns when no member is active.  Per id (host arrays of n_added
 * entries, any may be NULL): status (prc_member_status), steps (taken by the
 * member since it joined), hist[id * hist_cap + k] (relative residual of its
 * k-th check) and hist_len.  The newest state of each member is in its f_a.
 * Returns PRC_OK when every member has left, or an error. */
prc_status prc_batch_solve(prc_batch *b, double tol, int64_t check_every, int64_t max_steps,
                           int32_t *status, int64_t *steps, double *hist, int64_t hist_cap,
                           int64_t *hist_len, hipStream_t stream);

/* Autotuner for the batch sweep: time each tile shape a batch can use
 * (indices 0 .. 7 of prc_tune: the single-step shapes and the two-step 64 x 8,
 * 32 x 16 and 64 x 16) on the current members, sweeping f_a into f_b (f_a, which holds
 * the state, is only read), and keep the fastest for this batch.  tile_out
 * (may be NULL) receives it.  Synchronises the stream. */
prc_status prc_batch_tune(prc_batch *b, int32_t *tile_out, hipStream_t stream);

/* Use tile shape `tile` (0 .. 7, as for prc_batch_tune) for this batch's
 * sweeps.  Without it (or prc_batch_tune) a batch sweeps two steps per
 * launch on 32 x 16 tiles, or on 64 x 16 tiles once its members' states
 * together exceed 160 MB (FP32 and 16-bit storage).  Host only. */
prc_status prc_batch_set_tile(prc_batch *b, int32_t tile);

/* ---- Serving: steady-state solve requests with continuous batching -----
 *
 * prc_serve runs a stream of steady-state solve requests (Sec. 5: each a
 * problem driven to a converged state) that arrive over time.  Requests are
 * admitted in arrival order while their device memory fits a budget; every
 * admitted request joins one batch (prc_batch_*), which advances in
 * intervals of check_every steps; after each interval's check, requests that
 * converged, diverged or used up max_steps leave, their results are copied
 * to the host and their memory goes back to the pool, and waiting requests
 * join.  A request's arithmetic does not depend on the others: its result is
 * bit for bit that of prc_solve on the same problem with the same tol,
 * check_every and max_steps.
 */
typedef struct {
    double arrival_s;  /* seconds after the start of prc_serve; non-decreasing */
    prc_params p;      /* the problem; storage and bc must be the server's */
    double *ux, *uy;   /* host double[ny][nx] each for the final velocity, or NULL */
} prc_request;

typedef struct {
    int32_t status;    /* prc_member_status; PRC_EINVAL if the request was
                          rejected (invalid problem, or larger than the budget) */
    int32_t reserved;
    int64_t steps;     /* time steps taken */
    double residual;   /* relative residual of its last check */
    double admit_s;    /* when its state was set up on the GPU (seconds) */
    double done_s;     /* when its result was on the host (seconds) */
} prc_result;

typedef struct {
    int32_t storage, bc;  /* of every request */
    double tol;           /* convergence tolerance on the relative residual */
    int64_t check_every;  /* even, > 0 */
    int64_t max_steps;    /* multiple of check_every */
    size_t hbm_budget;    /* device bytes for the requests' buffers: two states
                             and a velocity snapshot (16 B/node) each */
    int32_t max_active;   /* at most this many requests in the batch; 0 = no
                             limit, 1 = one at a time */
    int32_t tile;         /* sweep tile shape (0 .. 7, as for prc_batch_tune),
                             -1 for the default */
} prc_serve_config;

/* Serve requests reqs[0 .. n) (host array, arrivals non-decreasing) and write
 * res[0 .. n) (host): a server (prc_server_create, below) to which the
 * calling thread submits each request at its arrival time (seconds after the
 * call) while collecting results.  Allocates one pool of cfg->hbm_budget
 * bytes (hipMalloc) for the requests' buffers and frees it before returning.
 * Blocks until every request has its result; synchronises the stream. */
prc_status prc_serve(const prc_serve_config *cfg, const prc_request *reqs, int32_t n,
                     prc_result *res, hipStream_t stream);

/* ---- Online serving: requests submitted while the server runs ----------
 *
 * prc_server_create starts a server on the current device: a pool of
 * cfg->hbm_budget device bytes (one hipMalloc), a batch, and a host worker
 * thread that runs the loop described above on `stream` -- admit submitted
 * requests whose buffers fit, advance the batch one interval, hand finished
 * results to the host, return their memory -- until prc_server_destroy; it
 * sleeps while nothing is submitted.  Requests are submitted at any time,
 * from any thread, and the call returns at once; finished ones are collected
 * with prc_server_poll.  Admission follows submission order, except that a
 * request that does not fit yet is passed by later ones that do, for at most
 * 8 intervals; after that nothing is admitted before it.  Each result is bit
 * for bit that of prc_solve on the same problem with the server's tol,
 * check_every and max_steps.  prc_serve above replays a trace of arrivals
 * through such a server.
 */
typedef struct prc_server prc_server;

typedef struct {
    int64_t ticket;    /* as returned by prc_server_submit */
    int32_t status;    /* prc_member_status, or PRC_EINVAL if rejected (invalid
                          problem, other storage or bc, larger than the pool) */
    int32_t reserved;
    int64_t steps;     /* time steps taken */
    double residual;   /* relative residual of its last check */
    double submit_s;   /* seconds since prc_server_create: submitted, */
    double admit_s;    /* its state set up on the GPU, */
    double done_s;     /* its result on the host */
} prc_server_result;

/* Start a server (see above); cfg as for prc_serve.  *out receives it.
 * Allocates the pool (PRC_EHIP if that fails) and starts the worker. */
prc_status prc_server_create(const prc_serve_config *cfg, hipStream_t stream,
                             prc_server **out);

/* Queue a steady-state solve of problem *p (copied).  ux, uy: host
 * double[ny][nx] each for the final velocity, or NULL; they must stay valid
 * until this request's result has been polled.  *ticket (may be NULL)
 * receives its id (0, 1, 2, ... per server).  Thread safe; returns at once.
 * Fails if the server has stopped or its worker failed. */
prc_status prc_server_submit(prc_server *srv, const prc_params *p, double *ux,
                             double *uy, int64_t *ticket);

/* Take up to cap finished results (host array out), oldest first; *n
 * receives how many.  Waits up to wait_s seconds for a first one if none is
 * ready (0: does not wait).  Thread safe.  Returns the worker's error once
 * it has failed and no result is left. */
prc_status prc_server_poll(prc_server *srv, double wait_s, prc_server_result *out,
                           int32_t cap, int32_t *n);

/* Requests waiting for admission, in the batch, and finished but not yet
 * polled (any pointer may be NULL). */
prc_status prc_server_status(prc_server *srv, int32_t *waiting, int32_t *active,
                             int32_t *unpolled);

/* Stop the worker after its current interval, synchronise the stream, free
 * the pool and the server.  Requests not finished by then are dropped (no
 * result).  NULL is allowed. */
prc_status prc_server_destroy(prc_server *srv);

/* Message of the last failed call on this thread ("" if none). */
const char *prc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PRC_H */
