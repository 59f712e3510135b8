/*
 * rlb.h -- C ABI of the MI355X library for the third-order relativistic
 * lattice Boltzmann scheme (RLBD) of Mendoza, Karlin, Succi and Herrmann,
 * "Relativistic Lattice Boltzmann Model with Improved Dissipation", and of
 * the second-order model of its Appendix A.
 *
 * What one step computes (Sec. II D, Eq. rlb:disc, time step delta t' = 1):
 *
 *   f_i(x + theta_i, t + 1) = f_i(x, t)
 *                             - (p_i^mu U_mu / (tau p_i^0)) (f_i - f_i^eq)
 *
 * on a periodic nx x ny x nz cubic lattice, with discrete 4-momenta
 * p_i = p0_i (1, theta_i / R): 128 of them with R = sqrt(41) for the
 * third-order model (Sec. II C, Eqs. dio, mrecon2), 66 with R = 3 for the
 * second-order model (Appendix A).  Per cell: the moments
 * N^mu = sum f_i p_i^mu and T^{mu nu} = sum f_i p_i^mu p_i^nu; the
 * Landau-Lifshitz eigenproblem T^{mu nu} U_nu = eps U^mu
 * (Eq. eigenproblem); n = U_mu N^mu; the equation of state eps = 3 n T,
 * P = eps / 3; the Maxwell-Juttner equilibrium projected on the orthonormal
 * polynomials of Table I up to third order (Eqs. coeff, disc1, equi3rd) or
 * up to second order (Eq. equi2nd); and the Anderson-Witting relaxation.
 *
 * Conventions
 *  - Every call returns RLB_OK (0) or a negative error code; no C++
 *    exception crosses this interface.  rlb_strerror() names a code and
 *    rlb_last_error() gives the last message of the calling thread.
 *  - Fields are float64 arrays of nx*ny*nz entries, x fastest:
 *    index = x + nx * (y + ny * z).
 *  - "stream" arguments are hipStream_t values passed as void*; NULL is the
 *    default stream.  The library never synchronises the device except
 *    where a call says so.
 *  - The caller owns every device buffer it passes (e.g. memory of a torch
 *    tensor) and must keep it alive until rlb_destroy; the library frees
 *    only its own small host allocations.
 *  - A solver is bound to one stream and one device and is not
 *    thread-safe; use one solver per thread.
 */
#ifndef RLB_H
#define RLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define RLB_OK 0
#define RLB_EINVAL (-1)   /* bad argument (sizes, modes, tau <= 1/2, NULL) */
#define RLB_ENOMEM (-2)   /* caller buffer smaller than rlb_state_bytes()   */
#define RLB_ENONPHYS (-3) /* init field with n<=0, eps<=0, |v|>=1 or NaN   */
#define RLB_EHIP (-4)     /* HIP runtime or launch error                    */
#define RLB_ESTATE (-5)   /* call out of order (e.g. step before init)      */
#define RLB_EIO (-6)      /* checkpoint file could not be written or read   */

/* ---- precision of the stored populations ------------------------------- */
#define RLB_FP64 0  /* populations, moments and equilibrium in float64       */
#define RLB_MIXED 1 /* populations stored and streamed as float32; moments
                       accumulated in float64 from the float32 values; the
                       Landau solve, gamma, tau and the equilibrium
                       coefficients in float64; equilibrium and relaxation of
                       each population in float32                            */

/* ---- model ----------------------------------------------------------------
 * The `order` argument or field selects the model; 0 means the default,
 * RLB_ORDER3.  Any other value is RLB_EINVAL. */
#define RLB_ORDER3 3 /* third-order model: 128 points, R^2 = 41, 4 shells */
#define RLB_ORDER2 2 /* second-order model: 66 points, R^2 = 9, 3 shells  */

/* ---- streaming pattern ----------------------------------------------------
 * RLB_PATTERN_AB: two population buffers; each step reads one and writes the
 * other (pull streaming).  RLB_PATTERN_AA: one buffer updated in place, the
 * "AA" pattern: even steps read and write each cell's own slots (storing
 * population i in the slot of its inverse), odd steps read the inverse slots
 * of the neighbours x - theta_i and write to x + theta_i, which restores the
 * natural layout.  Same arithmetic and results, half the population memory
 * (plus 56 bytes per cell of staging), so larger boxes fit: 576^3 in
 * float64 with the third-order model needs 206 GB with AA and 391 GB with
 * AB.  Walls need AB. */
#define RLB_PATTERN_AB 0
#define RLB_PATTERN_AA 1

/* ---- relaxation time ---------------------------------------------------- */
#define RLB_TAU_FIXED 0 /* tau is a constant (> 1/2)                         */
#define RLB_TAU_ETA_S 1 /* tau per cell and step from eta/s:
                           eta = n T (tau - 1/2) / (c R) and
                           s = 4 n - n ln(n / n_eq) with n_eq = T^3
                           (Sec. II D transport coefficients, Sec. III), i.e.
                           tau = 1/2 + (c R / T) (eta/s) (4 - ln(n/T^3)),
                           c = 3/2 for the third-order model and c = 7 for
                           the second-order one (the fit of Appendix A)     */

/* ---- status flags (sticky, OR-ed by the kernels) ----------------------- */
#define RLB_FLAG_NONFINITE 1u   /* a cell produced a NaN or infinity        */
#define RLB_FLAG_NONPHYSICAL 2u /* n <= 0, eps <= 0 or |v| >= 1 in a cell   */
#define RLB_FLAG_LANDAU 4u      /* the Landau-frame solve did not converge  */
#define RLB_FLAG_STALL 8u       /* a tube kernel gave up waiting for its     */
                                /* neighbouring work (never expected; the    */
                                /* tube's results are then invalid)          */

#define RLB_MAX_Q 128

/* The discrete velocity set of a model: q points (128 on 4 energy shells
 * for the third-order model, Sec. II C; 66 on 3 shells for the second-order
 * one, Appendix A); entries beyond q are zero.
 * theta: integer displacement per step; p0: energy; w: weight;
 * inv[i]: index of the point with theta = -theta_i on the same shell (the
 * library orders points so that inv[i] == i ^ 1); shell: 0..nshell-1.  The
 * weights were recomputed from the paper's conditions (Eqs. eqs:eqs, for
 * polynomials up to degree 6 in the third-order model and 5 in the
 * second-order one) because the paper lists them only in a supplement;
 * sha256 is that of the text table they come from. */
typedef struct rlb_lattice {
  int32_t q;
  int32_t r2;
  int32_t nshell;
  int8_t theta[RLB_MAX_Q][3];
  double p0[RLB_MAX_Q];
  double w[RLB_MAX_Q];
  int32_t inv[RLB_MAX_Q];
  int32_t shell[RLB_MAX_Q];
  char sha256[65];
} rlb_lattice_t;

/* Fills *out with the lattice of model `order` (0, RLB_ORDER2 or
 * RLB_ORDER3).  Read-only library data; RLB_EINVAL for NULL or a bad order. */
int rlb_lattice_info(int32_t order, rlb_lattice_t *out);

/* ---- one periodic box ---------------------------------------------------- */
typedef struct rlb_config {
  int32_t nx, ny, nz; /* lattice size, all periodic; each >= 1, and       */
                      /* nx*ny*nz <= 2^28 - 2^16 (268,369,920 cells)      */
  int32_t precision;  /* RLB_FP64 or RLB_MIXED                            */
  int32_t tau_mode;   /* RLB_TAU_FIXED or RLB_TAU_ETA_S                   */
  double tau;         /* relaxation time when tau_mode == RLB_TAU_FIXED   */
  double eta_s;       /* eta/s (> 0) when tau_mode == RLB_TAU_ETA_S        */
  int32_t order;      /* model: 0 or RLB_ORDER3, or RLB_ORDER2             */
  int32_t pattern;    /* RLB_PATTERN_AB (0) or RLB_PATTERN_AA              */
} rlb_config;

typedef struct rlb_solver rlb_solver;

/* Bytes of device memory a box of this size, model and pattern needs: two
 * population buffers (AB) or one buffer and a staging area of 7 doubles per
 * cell (AA), plus a 4 KiB status area.  Returns 0 for invalid sizes,
 * precision, order or pattern.  Pure function. */
size_t rlb_state_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t precision, int32_t order, int32_t pattern);

/* Creates a solver over caller-owned device memory d_buf of `bytes` bytes
 * (>= rlb_state_bytes, 256-byte aligned) on `stream` of the current device.
 * Errors: RLB_EINVAL (bad config / NULL / misaligned), RLB_ENOMEM (bytes too
 * small), RLB_EHIP.  No device work is issued. */
int rlb_create(rlb_solver **out, const rlb_config *cfg, void *d_buf, size_t bytes,
               void *stream);

/* Sets every cell to local equilibrium f_i = f_i^eq(n, T, U) with
 * T = eps / (3 n) and U = gamma (1, v) (initial states of Sec. III) and
 * resets t = 0 and the status flags.  n, eps, vx, vy, vz are nx*ny*nz
 * float64 values.  on_device = 0: host arrays, validated on the host
 * (RLB_ENONPHYS if any n <= 0, eps <= 0, |v| >= 1 or a value is not
 * finite; nothing is changed then) and copied through the idle population
 * buffer (AB) or the staging area (AA); the call returns after the copy.  on_device = 1: device arrays,
 * read on the stream; invalid cells raise RLB_FLAG_NONPHYSICAL instead.
 * The arrays may be released when the call returns (host) or when the
 * stream has passed this point (device). */
int rlb_init_fields(rlb_solver *s, const double *n, const double *eps, const double *vx,
                    const double *vy, const double *vz, int32_t on_device);

/* Advances nsteps >= 0 time steps of Eq. rlb:disc (Sec. II D): per cell
 * the moments, the Landau-Lifshitz frame (Eq. eigenproblem, Eq.
 * densitycal, eps = 3 n T), tau, the equilibrium (Eqs. coeff, disc1,
 * equi3rd / equi2nd), the Anderson-Witting relaxation and the exact
 * streaming by theta_i.  Asynchronous on the solver's stream.
 * RLB_ESTATE before rlb_init_fields, RLB_EHIP on a launch error. */
int rlb_step(rlb_solver *s, int64_t nsteps);

/* Macroscopic fields of the current (post-streaming, pre-collision) state,
 * the quantities Sec. III reports: n = U_mu N^mu (Eq. densitycal), eps and
 * U^mu from T^{mu nu} U_nu = eps U^mu (Eq. eigenproblem), P = eps / 3:
 * n, eps, P each nx*ny*nz values and U4 = 4*nx*ny*nz values laid out as
 * U^0 block, U^1 block, U^2 block, U^3 block.  Any output pointer may be
 * NULL.  on_device = 0: host arrays, the call synchronises the stream;
 * on_device = 1: device arrays written on the stream (no synchronisation). */
int rlb_read_fields(rlb_solver *s, double *n, double *eps, double *U4, double *P,
                    int32_t on_device);

/* Box totals of N^0 and T^{0 nu} (nu = 0..3) of the current state, the
 * quantities the scheme conserves (Eqs. conser1, conser2): out[0] = N^0,
 * out[1..4] = T^{00}, T^{01}, T^{02}, T^{03}.  Float64 sums with a fixed
 * reduction order; synchronises the stream. */
int rlb_conserved(rlb_solver *s, double out[5]);

/* rlb_conserved for callers that cannot allocate device memory or lend
 * the library a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same kernels, summation order and
 * results as rlb_conserved, but the partial sums go to a fixed device array
 * of the library (8 MiB per GPU, held until the process ends) instead of the
 * solver's idle buffer or staging area, which stay untouched.  Allocates
 * nothing.  Limits: at most 33,554,432 cells (2^25; e.g. 320^3), and no
 * walls (their per-cell sums need a cells-sized array): RLB_EINVAL
 * otherwise.  Synchronises the stream.  All calls on one GPU share that
 * array: calls that overlap on one GPU (from several threads) race. */
int rlb_conserved_noalloc(rlb_solver *s, double out[5]);

/* Sticky status flags (RLB_FLAG_*) and the current step count.  Either
 * pointer may be NULL.  Synchronises the stream. */
int rlb_status(rlb_solver *s, uint32_t *flags, int64_t *t);

/* Writes the raw population buffer as the library stores it (tiles of
 * 256 / element-size cells with 256-byte segments per population; for AA in
 * the layout of the current step's parity), t, the flags and the
 * configuration to a file (host I/O; synchronises the stream). */
int rlb_save(rlb_solver *s, const char *path);

/* Restores a state written by rlb_save into a solver with the same
 * configuration.  RLB_EINVAL if the file's configuration or lattice
 * differs, RLB_EIO on a short or unreadable file. */
int rlb_load(rlb_solver *s, const char *path);

/* Releases the solver's host allocations (not the caller's buffer). */
void rlb_destroy(rlb_solver *s);

/* ---- solid walls ------------------------------------------------------------
 * The paper asks for weights that are equal on inversion pairs so that
 * bounce-back can impose zero velocity on solid walls (Sec. II C).  The
 * library implements link-wise bounce-back: a population i whose source cell
 * x - theta_i is solid arrives at fluid cell x as the post-collision value of
 * the inverse population at x.  N^0 and T^{00} stay conserved; the walls
 * exchange momentum with the fluid.  solid[] holds nx*ny*nz bytes, x
 * fastest, non-zero = solid.  A population can jump over a wall thinner than
 * its displacement (up to 6 cells in the third-order model, 3 in the
 * second-order one), so walls meant to be impermeable must be at least that
 * thick.  Solid cells hold no fluid: rlb_read_fields reports zeros there, and
 * a cell that becomes solid loses its contents. */

/* Device bytes the walls of this mask need (the mask plus one 12-byte
 * bounce-back link per solid-cell/population pair that points into fluid);
 * 0 if the arguments are invalid or every cell is solid.  Pure host
 * function. */
size_t rlb_walls_bytes(int32_t order, int32_t nx, int32_t ny, int32_t nz, const uint8_t *solid);

/* Sets (solid != NULL) or removes (solid == NULL) the walls of a solver.
 * d_buf: caller-owned device memory of >= rlb_walls_bytes bytes, 256-byte
 * aligned, kept alive while the walls are set; the host mask may be released
 * when the call returns (it synchronises the solver's stream).  Takes effect
 * from the next step; rlb_save records the mask's hash and rlb_load requires
 * the same walls.  Errors: RLB_EINVAL (NULL solver or buffer, misaligned,
 * every cell solid), RLB_ENOMEM (buffer too small), RLB_EHIP. */
int rlb_set_walls(rlb_solver *s, const uint8_t *solid, void *d_buf, size_t bytes);

/* ---- many independent shock tubes (1 x 1 x n periodic lattices) ------------
 * The Riemann problems of Sec. III are one-dimensional: a tube is a periodic
 * 1 x 1 x n lattice on which only the z displacement of each point moves
 * anything.  A batch holds many tubes of one precision in one caller-owned
 * buffer and advances all of them in one persistent launch: one workgroup
 * per tube, launched longest-work-first, whose wavefronts take the tube's
 * (step, chunk) work in order and wait only for the neighbouring chunks'
 * previous step (float64 tubes above 786,432 cells: a workgroup barrier
 * between steps instead).  Every such wait is bounded: after about 0.1 s it
 * gives up and raises RLB_FLAG_STALL in its tube (never expected; the
 * environment variable RLB_TUBE_SPIN_LIMIT, read by rlb_batch_step, lowers
 * the bound to that many polls, for tests of that path).  Tubes never
 * interact; a failure (status flag) stays in its tube. */
typedef struct rlb_tube {
  int32_t n;        /* cells along z, 1 .. 4,194,304 (2^22)                */
  int32_t tau_mode; /* RLB_TAU_FIXED or RLB_TAU_ETA_S                       */
  double tau;       /* when tau_mode == RLB_TAU_FIXED (> 1/2)               */
  double eta_s;     /* when tau_mode == RLB_TAU_ETA_S (> 0)                 */
} rlb_tube;

typedef struct rlb_batch rlb_batch;

/* Device bytes for a batch of these tubes under model `order` (0 if any
 * tube, the precision or the order is invalid). */
size_t rlb_batch_bytes(const rlb_tube *tubes, int32_t ntubes, int32_t precision, int32_t order);

/* Creates a batch of one precision and one model over caller-owned device
 * memory (>= rlb_batch_bytes, 256-byte aligned) on `stream`.  The tube array
 * is copied.  Errors as for rlb_create. */
int rlb_batch_create(rlb_batch **out, const rlb_tube *tubes, int32_t ntubes, int32_t precision, int32_t order,
                     void *d_buf, size_t bytes, void *stream);

/* Initial fields of one tube (n values each, index = z); semantics and
 * errors as rlb_init_fields.  Resets that tube's t and flags. */
int rlb_batch_init(rlb_batch *b, int32_t tube, const double *n, const double *eps, const double *vx,
                   const double *vy, const double *vz, int32_t on_device);

/* One persistent launch: tube j advances steps[j] >= 0 steps (0 leaves it
 * untouched).  Every tube with steps[j] > 0 must have been initialised.
 * Asynchronous on the batch's stream. */
int rlb_batch_step(rlb_batch *b, const int64_t *steps);

/* Fields of one tube, as rlb_read_fields (U4 holds 4 n values). */
int rlb_batch_read(rlb_batch *b, int32_t tube, double *n, double *eps, double *U4, double *P,
                   int32_t on_device);

/* Status flags and step count of one tube (synchronises the stream). */
int rlb_batch_status(rlb_batch *b, int32_t tube, uint32_t *flags, int64_t *t);

/* Releases the batch's host allocations. */
void rlb_batch_destroy(rlb_batch *b);

/* ---- serving: continuous batching of tube and box solves -------------------
 * A server owns a worker thread and a caller-owned device pool.  Requests
 * (a shock tube or a periodic box, each with its own precision, relaxation,
 * step count and initial fields) are submitted at any time; the worker
 * admits them in arrival order as soon as their footprint fits in the pool
 * and their stream is idle (a box goes to the box stream with the least
 * work left); a request waiting for its stream lets later requests bound
 * for idle streams pass, one waiting for memory holds back all behind it.
 * Work runs on four streams (tubes of each precision, and two
 * for boxes), each advancing on its own: when a stream has finished its last
 * work, its finished requests are read back, freed and reported by
 * rlb_server_poll, and its next work is issued: each of its boxes by
 * 40 * chunk_steps * max(1, 262144 / cells) steps (replays of a hipGraph of
 * chunk_steps launches; the last issue may end with fewer; a long tube run
 * as a box by chunk_steps * max(1, 262144 / nz)), or each of its
 * tubes by max(chunk_steps, chunk_steps * 8192 / nz) steps, all resident
 * tubes of one precision and model in one persistent launch.  Tubes of 2048
 * cells or more run as 1 x 1 x nz boxes (box kernels, which spread a step
 * over many CUs, where a persistent tube launch gives a tube one CU), on
 * the tube stream of their precision.
 * The four streams should each have a hardware queue: a process that has
 * other busy streams should raise GPU_MAX_HW_QUEUES (HIP's default is 4).
 * A request's result does not depend on what else is resident (the kernels
 * never mix requests).  Times are seconds since the server was created. */
#define RLB_REQ_TUBE 0 /* 1 x 1 x nz lattice (nx = ny = 1)                */
#define RLB_REQ_BOX 1  /* nx x ny x nz periodic box                        */

typedef struct rlb_request {
  int32_t kind;       /* RLB_REQ_TUBE or RLB_REQ_BOX                          */
  int32_t nx, ny, nz; /* lattice size (a tube has nx = ny = 1)                */
  int32_t precision;  /* RLB_FP64 or RLB_MIXED                                */
  int32_t tau_mode;   /* RLB_TAU_FIXED or RLB_TAU_ETA_S                       */
  int32_t order;      /* model: 0 or RLB_ORDER3, or RLB_ORDER2                */
  double tau, eta_s;
  int64_t steps;      /* >= 0                                                  */
  /* initial fields, nx*ny*nz host values each; copied by rlb_server_submit  */
  const double *n, *eps, *vx, *vy, *vz;
  /* host outputs written before the completion is reported (may be NULL);
   * they must stay valid until then                                        */
  double *out_n, *out_eps, *out_U4, *out_P;
} rlb_request;

typedef struct rlb_completion {
  int64_t id;
  int32_t rc;         /* RLB_OK, or the error that ended the request          */
  uint32_t flags;     /* RLB_FLAG_* of this request                           */
  double t_submit, t_admit, t_done;
} rlb_completion;

typedef struct rlb_server rlb_server;

/* Device bytes one request occupies while resident (0 if invalid). */
size_t rlb_request_bytes(const rlb_request *req);

/* Starts a server on the current device over a caller-owned pool (256-byte
 * aligned).  chunk_steps: even, >= 2.  max_tubes: how many tubes may be
 * resident at once.  The pool must stay valid until rlb_server_destroy. */
int rlb_server_create(rlb_server **out, void *d_pool, size_t pool_bytes, int32_t chunk_steps, int32_t max_tubes);

/* Queues a request (thread-safe).  Validates it (RLB_EINVAL, RLB_ENONPHYS
 * for bad fields, RLB_ENOMEM if it can never fit in the pool) and copies the
 * initial fields; *id identifies it in completions. */
int rlb_server_submit(rlb_server *s, const rlb_request *req, int64_t *id);

/* Up to `max` completions into out (thread-safe); waits up to wait_ms for
 * the first one.  *count is the number returned. */
int rlb_server_poll(rlb_server *s, rlb_completion *out, int32_t max, int32_t *count, int32_t wait_ms);

/* Requests submitted and not yet reported, and the number of times work
 * has been issued to a stream so far. */
int rlb_server_pending(rlb_server *s, int64_t *pending, int64_t *rounds);

/* Stops the worker (pending requests are dropped) and releases the
 * server's host resources and streams. */
void rlb_server_destroy(rlb_server *s);

/* ---- diagnostics --------------------------------------------------------- */
const char *rlb_strerror(int code);
const char *rlb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RLB_H */
