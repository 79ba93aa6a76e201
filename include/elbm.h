/*
 * elbm.h -- C ABI of the MI355X (gfx950) entropic lattice Boltzmann library.
 *
 * The library advances the entropic lattice Boltzmann method (ELBM) of
 * Zhao & Yong, "Relaxation-rate formula for the entropic lattice Boltzmann
 * method": per time step and lattice site it
 *   1. pulls the streamed populations f_i(x,t) (Eq. (5b)),
 *   2. forms rho = sum_i f_i and rho u = sum_i c_i f_i (the conservation
 *      constraints stated after Eq. (3)),
 *   3. builds the entropic equilibrium f^eq, the minimiser of
 *      H(f) = sum_i f_i ln(f_i/W_i) (Eq. (3)) under those constraints,
 *   4. chooses alpha: alpha_max (definition after Eq. (7)), alpha_* = min(2,
 *      alpha_max) (Eq. (8)), alpha = alpha_* if H(f*(alpha_*)) <= H(f),
 *      otherwise the closed form Eq. (9),
 *   5. collides, f~_i = f_i + alpha beta (f_i^eq - f_i) (Eq. (1) = Eq. (5a)),
 *      and stores f~ for the next step's pull.
 * Beside it: the entropy balance Eq. (4) solved per site by Newton or by
 * bisection (stop window -tol <= H(f*) - H(f) <= 0 as in the double-shear
 * comparison), the modified secant iteration of the closing remark, and
 * LBGK (alpha = 2, polynomial equilibrium; the special case after Eq. (4)).
 *
 * Conventions
 *   - Lattice units: delta_x = delta_t = 1, c_s^2 = 1/3, so Eq. (2) reads
 *     beta = 1 / (6 nu + 1).  Periodic box nx * ny * nz (ny = nz = 1 for
 *     D1Q3, nz = 1 for D2Q9), N = nx*ny*nz sites, site index
 *     s = x + nx*(y + ny*z).
 *   - Directions: c_i in {-1,0,1}^D with i = d(c_x) + 3 d(c_y) + 9 d(c_z),
 *     d(0) = 0, d(+1) = 1, d(-1) = 2.  Weights W_i = prod_a w(c_ia),
 *     w(0) = 2/3, w(+-1) = 1/6 (D2Q9: 4/9, 1/9, 1/36).
 *   - D3Q19 (ELBM_D3Q19) keeps the D3Q27 directions with at most two
 *     nonzero components (no corners), in the order of their D3Q27 index,
 *     with W = 1/3 (rest), 1/18 (|c|^2 = 1), 1/36 (|c|^2 = 2).  Its weights
 *     do not factorise, so f^eq (the minimiser of Eq. (3) under the mass and
 *     momentum constraints) has no closed form: the step finds its Lagrange
 *     multipliers per site by Newton's method.  Its domain is the interior
 *     of the velocities' hull: |u_a| < 1 and |u_x| + |u_y| + |u_z| < 2.
 *   - Every array argument is a DEVICE pointer (hipMalloc'd or a torch
 *     tensor's data pointer) unless its comment says "host".  Population
 *     arrays are SoA float64: f[i*N + s]; velocity arrays are SoA u[a*N + s].
 *   - f(x,t) always means the paper's pre-collision populations at time t.
 *
 * Memory and streams
 *   - The caller owns all device memory.  elbm_init places the whole
 *     simulation state (two population buffers, the optional alpha field and
 *     the diagnostics area) in the caller's buffer of elbm_state_bytes()
 *     bytes, which must stay allocated and untouched until elbm_destroy.
 *     The state's internal layout is private (populations are kept in
 *     blocks of 64 sites); the calls below exchange plain SoA arrays.
 *     The library itself calls no hipMalloc; it allocates only the small
 *     host-side handle.
 *   - Every call enqueues work on the stream given to elbm_init and returns
 *     without waiting, except where its comment says it synchronises.
 *   - A handle may be used from one host thread at a time.
 *
 * Errors
 *   - Every function returns an elbm_status; nothing is thrown across the
 *     ABI.  elbm_last_error() returns a message for the calling thread's
 *     last failure.  Numerical events (negative or non-finite populations)
 *     are not errors: they are counted in elbm_stats.
 */
#ifndef ELBM_H
#define ELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELBM_ABI_VERSION 1

typedef struct elbm_sim elbm_sim; /* opaque; owned by the library */

typedef enum {
  ELBM_OK = 0,
  ELBM_EINVAL = -1,      /* invalid argument or configuration            */
  ELBM_EDEVICE = -2,     /* a HIP runtime call failed                    */
  ELBM_ENOMEM = -3,      /* caller buffer smaller than elbm_state_bytes  */
  ELBM_ESTATE = -4,      /* call not valid in the handle's current state */
  ELBM_EUNSUPPORTED = -5 /* combination not built into this library      */
} elbm_status;

/* Lattice codes: D1Q3, D2Q9 and D3Q27 carry their dimension, D3Q19 its
 * direction count. */
enum { ELBM_D1Q3 = 1, ELBM_D2Q9 = 2, ELBM_D3Q27 = 3, ELBM_D3Q19 = 19 };

enum {
  ELBM_ALPHA_CLOSED = 0, /* Eq. (8), acceptance test, Eq. (9)            */
  ELBM_ALPHA_NEWTON = 1, /* bracketed Newton root of Eq. (4), from
                            alpha_*, stop at a step below 1e-13 alpha     */
  ELBM_ALPHA_BISECT = 2, /* bisection root of Eq. (4), window root_tol   */
  ELBM_ALPHA_BGK = 3,    /* alpha = 2 with the polynomial equilibrium    */
  ELBM_ALPHA_SECANT = 4  /* modified secant, secant_iters iterations     */
};

/* Population storage.  *_DEV stores s_i = f_i / W_i - rho_ref ("deviation
 * from W_i rho"), decoded as f_i = W_i (rho_ref + s_i); FP16 is rounded to
 * nearest even. */
enum {
  ELBM_STORE_F64 = 0,
  ELBM_STORE_F32 = 1,
  ELBM_STORE_F32_DEV = 2,
  ELBM_STORE_F16_DEV = 3
};

/* Site arithmetic (elbm_config.alpha_fp64).  The paper computes in FP64
 * throughout.
 *   FP64:  moments, equilibrium, x_i = f_i / f^eq_i - 1, the entropy
 *          differences, alpha and the collision in FP64; one rounding into
 *          the storage format.  Every alpha mode, every storage format.
 *   FP32:  all of it in FP32 on f_i (closed-form alpha; FP32 and deviation
 *          storage).
 *   MIXED: FP32 arithmetic on the deviations s_i = f_i / W_i - rho_ref:
 *          moments, the equilibrium as s^eq_i = f^eq_i / W_i - rho_ref
 *          (formed without cancellation), x_i = (s_i - s^eq_i) /
 *          (rho_ref + s^eq_i) and the collision s~_i = s_i + alpha beta
 *          (s^eq_i - s_i); the entropy differences of Eqs. (7)-(9) and alpha
 *          in FP64.  Closed-form alpha; FP32 and deviation storage; D1Q3,
 *          D2Q9 and D3Q27 with the Boltzmann entropy. */
enum { ELBM_ARITH_FP32 = 0, ELBM_ARITH_FP64 = 1, ELBM_ARITH_MIXED = 2 };

/* Entropy function.  The paper states the scheme for the Boltzmann entropy
 * of Eq. (3) and remarks that the closed form (Eq. (9)) needs only a convex
 * entropy; the library also runs it with Burg's entropy
 *   H(f) = -sum_i W_i ln(f_i / W_i),
 * whose equilibrium f_i = W_i / (m0 + m.c_i) is found per site by Newton's
 * method on the multipliers (no closed form on any lattice).  Burg's entropy
 * is infinite at a zero population, so alpha_* = alpha_max < 2 gives
 * alpha = 1 (the limit of Eq. (9)).  Burg is built for the entropic alpha
 * modes (not LBGK, which uses no entropy), FP64 arithmetic, FP64 and FP32
 * storage. */
enum { ELBM_ENTROPY_BOLTZMANN = 0, ELBM_ENTROPY_BURG = 1 };

/* Diagnostics switches (bit mask). */
enum {
  ELBM_DIAG_ALPHA = 1u,  /* record alpha(x) of every step (8 B/site extra) */
  ELBM_DIAG_COUNTS = 2u, /* per-step site counts and the alpha range      */
  ELBM_DIAG_SUMS = 4u    /* also sum_x rho, rho u and H(f(x,t)) (Eq. (6)); */
                         /* needs COUNTS                                  */
};

typedef struct {
  int32_t lattice;       /* ELBM_D1Q3 / ELBM_D2Q9 / ELBM_D3Q27 / ELBM_D3Q19 */
  int32_t nx, ny, nz;    /* box, each in [1, 2^20 - 1]; nz = 1 for D2Q9,
                            ny = nz = 1 for D1Q3; N = nx ny nz at most
                            2^31 - 1 sites (32-bit site indices)        */
  double beta;           /* Eq. (2), 0 < beta < 1                         */
  int32_t alpha_mode;    /* ELBM_ALPHA_*                                  */
  int32_t storage;       /* ELBM_STORE_*                                  */
  int32_t alpha_fp64;    /* ELBM_ARITH_*: FP64 (the default; required
                            for STORE_F64 and the root and secant modes),
                            FP32 or MIXED (closed mode, FP32 and deviation
                            storage)                                      */
  int32_t secant_iters;  /* iterations of ELBM_ALPHA_SECANT (>= 1)        */
  double rho_ref;        /* reference density of *_DEV storage (> 0)      */
  double root_tol;       /* bisection window; the paper uses 1e-13        */
  int32_t root_max_iter; /* cap for Newton / bisection iterations (>= 1)  */
  uint32_t diag;         /* ELBM_DIAG_* mask                              */
  int32_t entropy;       /* ELBM_ENTROPY_*                                */
  int32_t reserved;      /* must be 0                                     */
} elbm_config;

/* Per-step diagnostics of the most recent step (ELBM_DIAG_COUNTS).  In
 * ELBM_ALPHA_BGK mode the entropic alpha rules are not evaluated, so the
 * alpha-rule counts (n_accept2 ... n_fallback, total_iters) stay 0. */
typedef struct {
  int64_t step;            /* t after the step that produced these         */
  int64_t n_sites;
  int64_t n_accept2;       /* sites with H(f*(2)) <= H(f) (Fig. 5's count) */
  int64_t n_alphastar_lt2; /* sites with alpha_max < 2                     */
  int64_t n_alpha_lt2;     /* sites with alpha < 2                         */
  int64_t n_guard;         /* sites with f = f^eq to rounding              */
  int64_t n_fallback;      /* sites evaluated with log1p, not the series   */
  int64_t n_negative;      /* sites with a post-collision population < 0   */
  int64_t n_nonfinite;     /* sites whose rho, u or alpha is NaN or inf    */
  int64_t total_iters;     /* root-solver / secant iterations, summed      */
  double alpha_min, alpha_max; /* range of alpha (float precision)        */
  double sum_rho;          /* sum_x rho(x,t)        (ELBM_DIAG_SUMS, else 0) */
  double sum_j[3];         /* sum_x rho u(x,t)      (ELBM_DIAG_SUMS, else 0) */
  double sum_H;            /* sum_x H(f(x,t))       (ELBM_DIAG_SUMS, else 0) */
} elbm_stats_t;

/* Default configuration for a lattice and box (closed-form alpha, FP32
 * storage, FP64 site arithmetic, beta = 0.95, root_tol = 1e-13, no
 * diagnostics). */
elbm_status elbm_config_default(elbm_config *cfg, int32_t lattice, int32_t nx,
                                int32_t ny, int32_t nz);

/* Bytes of device memory the simulation state needs (0 on invalid cfg). */
size_t elbm_state_bytes(const elbm_config *cfg);

/* Create a simulation in the caller's device buffer dev_state (>= bytes of
 * elbm_state_bytes, 256-byte aligned) and set f(x,0) = f^eq(rho0(x), u0(x))
 * with rho0[N] > 0 and u0[D*N], |u0| < 1 per component and on D3Q19 also
 * |u0_x| + |u0_y| + |u0_z| < 2 (the domain of the entropic equilibrium; D = 3
 * and Q = 19 for D3Q19).  hip_stream is a hipStream_t (NULL = the null
 * stream).  Synchronises the stream once to validate rho0 and u0; returns
 * ELBM_EINVAL if any value is out of range.  *out receives the handle. */
elbm_status elbm_init(const elbm_config *cfg, const double *rho0,
                      const double *u0, void *dev_state, size_t bytes,
                      void *hip_stream, elbm_sim **out);

/* Overwrite the state with arbitrary pre-collision populations f(x,t),
 * f[Q*N] float64 (non-negative for the entropic modes).  t is unchanged. */
elbm_status elbm_set_populations(elbm_sim *sim, const double *f);

/* Advance nsteps >= 0 time steps (Eq. (1) then Eq. (5b) per step). */
elbm_status elbm_step(elbm_sim *sim, int64_t nsteps);

/* The moments of the current f(x,t) that the equilibrium is constrained to
 * (the conditions of the minimisation of Eq. (3)): rho = sum_i f_i into
 * rho[N] and u = sum_i c_i f_i / rho into u[D*N], component-major (u[a*N +
 * s]); device pointers, float64, written on the simulation's stream. */
elbm_status elbm_moments(elbm_sim *sim, double *rho, double *u);

/* Current pre-collision populations f_i(x,t) (the streamed values of
 * Eq. (5b)) decoded from their storage format into f[Q*N] (device,
 * float64, direction-major: f[i*N + s]). */
elbm_status elbm_populations(elbm_sim *sim, double *f);

/* Gather at n sites (site indices sites[n], int64, device):
 *   which = 0: the pre-collision f(x,t) of those sites (Eq. (5b));
 *   which = 1: the post-collision f~(x,t-1) of Eq. (1) that the last step
 *              wrote there.
 * out[i*n + k] (device, float64). */
elbm_status elbm_gather(elbm_sim *sim, const int64_t *sites, int64_t n,
                        int32_t which, double *out);

/* alpha(x) of the collision Eq. (1) in the most recent step: Eq. (8)-(9)
 * for the closed form, the root of Eq. (4) for Newton and bisection, the
 * modified secant's last iterate, 2 for LBGK (requires ELBM_DIAG_ALPHA and
 * at least one step), copied into alpha[N] (device, float64). */
elbm_status elbm_alpha_field(elbm_sim *sim, double *alpha);

/* Diagnostics of the most recent step (requires ELBM_DIAG_COUNTS and at
 * least one step): the counts of elbm_stats_t (sites accepting alpha = 2,
 * the quantity of the Fig. 5 discussion; alpha_* < 2 by Eq. (8); ...) and,
 * with ELBM_DIAG_SUMS, sum_x H of Eq. (6).  stats is a HOST pointer;
 * synchronises the stream. */
elbm_status elbm_stats(elbm_sim *sim, elbm_stats_t *stats);

/* Time t of the current state (host value, no synchronisation). */
int64_t elbm_time(const elbm_sim *sim);

/* Release the handle (not the caller's device buffer).  Waits for the
 * handle's pending work first. */
elbm_status elbm_destroy(elbm_sim *sim);

/* ---- checkpoint / resume ------------------------------------------------
 * A checkpoint is the current populations bit for bit in their stored form
 * (an opaque blob of elbm_checkpoint_bytes() bytes) plus the time t.  The
 * step is a function of the stored populations only, so a simulation
 * restored from a checkpoint continues exactly as the original would
 * (bitwise).  A checkpoint is valid for simulations of the same lattice,
 * box and storage (other configuration fields may differ, e.g. beta or the
 * alpha mode). */

/* Bytes of a checkpoint (0 and ELBM_EINVAL for a NULL handle). */
size_t elbm_checkpoint_bytes(const elbm_sim *sim);

/* Copy the current populations into dst (device, >= bytes of
 * elbm_checkpoint_bytes) on the simulation's stream; *t (host) receives the
 * time of the state.  Asynchronous like elbm_step. */
elbm_status elbm_export(elbm_sim *sim, void *dst, size_t bytes, int64_t *t);

/* Replace the current populations with a checkpoint src (device, bytes ==
 * elbm_checkpoint_bytes) taken from a simulation of the same lattice, box
 * and storage, and set the time to t.  Asynchronous; the alpha field and
 * the diagnostics of the previous step are invalidated. */
elbm_status elbm_import(elbm_sim *sim, const void *src, size_t bytes, int64_t t);

/* Message of the calling thread's last error ("" if none). */
const char *elbm_last_error(void);

/* Advance several independent simulations that share one stream with ONE
 * kernel launch per step: sims[n] all created on the same stream with the
 * same lattice, storage, alpha mode and arithmetic; nsteps[n] (host) steps
 * each, sims with fewer steps drop out as they finish.  Results are
 * identical to stepping each simulation alone. */
elbm_status elbm_step_batch(elbm_sim *const *sims, const int64_t *nsteps,
                            int32_t n);

/* ---- a step with diagnostics that allocates nothing ---------------------
 *
 * For callers that cannot allocate device memory or hand the library a
 * workspace: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  It is elbm_step(sim, nsteps) followed by
 * elbm_stats for a handle whose state need not hold the diagnostics areas
 * (create it without ELBM_DIAG_COUNTS): the per-workgroup records of the
 * steps live in a device array the library holds for the life of the
 * process, one per GPU (7,340,032 bytes: records of at most 65,536
 * workgroups, i.e. boxes of at most 2^24 sites, or 2^26 for D1Q3 and D2Q9
 * with 2- or 4-byte storage, whose workgroups hold 1024 sites), and the
 * diagnostics of the last step are reduced into dev_stats.
 *   diag:      ELBM_DIAG_COUNTS, optionally | ELBM_DIAG_SUMS (the meaning of
 *              each field as for elbm_stats); the handle's own
 *              ELBM_DIAG_ALPHA setting still records alpha(x).
 *   dev_stats: DEVICE pointer to one elbm_stats_t, written on the handle's
 *              stream after the last step (no host copy, no synchronisation,
 *              no allocation, no memset).
 * Populations, alpha and the statistics are the same bits as elbm_step then
 * elbm_stats.  Afterwards elbm_stats on the handle returns ELBM_ESTATE until
 * an elbm_step has written the handle's own records.  All calls on one GPU
 * share its array: calls that overlap on that GPU (other streams, other
 * threads) race and corrupt each other's statistics; serialise them.
 * ELBM_EINVAL for nsteps < 1, a NULL pointer, other diag bits, or a box of
 * more than 65,536 workgroups (the message names the limit in sites). */
elbm_status elbm_step_noalloc(elbm_sim *sim, int64_t nsteps, uint32_t diag,
                              elbm_stats_t *dev_stats);

/* ---- serving: continuous batching of many simulations ------------------
 *
 * A server owns a scheduler thread and sub-allocates the states of the
 * simulations it admits from one caller-provided device memory pool.
 * Requests are admitted first come, first served, as soon as a slot is free
 * and the pool has room for the request's state (elbm_state_bytes) plus a
 * staging copy of its initial fields.  Each scheduling round advances every
 * resident simulation by up to round_steps steps with batched launches
 * (elbm_step_batch: one launch per step for all residents of the same
 * lattice, storage, alpha mode and arithmetic); a request arriving while a
 * round runs joins at the next round.  Two rounds are kept in flight on the
 * stream, so admission and completion work on the host overlaps the GPU.
 * Each resident simulation gives the same bits as stepping it alone.
 */
typedef struct elbm_server elbm_server;

typedef struct {
  void *pool;           /* device memory to sub-allocate (caller-owned,
                           256-byte aligned, kept until elbm_server_destroy) */
  size_t pool_bytes;
  void *hip_stream;     /* stream of all server work (NULL = null stream)   */
  int32_t max_active;   /* resident simulations at once, >= 1              */
  int32_t round_steps;  /* steps per scheduling round, >= 1                */
  int32_t preempt_rounds; /* 0: never preempt.  k >= 1: when the request at
                           the head of the queue cannot be admitted (no free
                           slot or no room in the pool), requests resident
                           for at least k rounds, with more than one round of
                           steps left and more than twice the head's
                           remaining work (steps x sites) are preempted, most
                           remaining work first, if that makes room:
                           their populations are copied to pinned host
                           memory (a checkpoint, see elbm_export), their pool
                           block is freed and they re-enter the queue at the
                           back; re-admitted, they continue from the
                           checkpoint bit for bit.  A victim for which no
                           pinned host memory can be had stays resident  */
  int32_t reserved;     /* must be 0                                         */
} elbm_server_config;

typedef struct {
  elbm_config cfg;      /* as for elbm_init                                  */
  const double *rho0;   /* HOST, N values; copied by elbm_server_submit      */
  const double *u0;     /* HOST, D*N values; copied by elbm_server_submit    */
  int64_t nsteps;       /* >= 0                                              */
  double *out_rho;      /* device, N values: rho at the end, or NULL         */
  double *out_u;        /* device, D*N values: u at the end, or NULL         */
  int32_t keep_state;   /* 1: keep the simulation resident after its last
                           step, for elbm_server_sim, until
                           elbm_server_release                               */
  int32_t reserved;     /* must be 0                                         */
} elbm_request;

enum { ELBM_REQ_QUEUED = 0, ELBM_REQ_RUNNING = 1, ELBM_REQ_DONE = 2,
       ELBM_REQ_FAILED = 3, ELBM_REQ_CANCELLED = 4 };

typedef struct {
  int32_t state;        /* ELBM_REQ_* (a preempted request is QUEUED)        */
  int32_t preemptions;  /* times the request was preempted                   */
  int64_t steps_done;
  double t_submit;      /* seconds on the server's monotonic clock          */
  double t_admit;       /* first admission (0 while queued)                  */
  double t_done;        /* completion observed on the host (0 until done)   */
  size_t footprint;     /* pool bytes held while resident                    */
} elbm_request_info;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t rounds, launches;
  int64_t site_updates; /* sum over completed steps of the box sizes         */
  int64_t max_resident; /* most simulations resident at once                 */
  double t_first_submit, t_last_done;
  int64_t preemptions;  /* requests moved out to host memory (preempt_rounds) */
  int64_t cancelled;    /* requests ended by elbm_server_cancel              */
} elbm_server_stats;

/* Create a server; starts its scheduler thread on the current device.
 * ELBM_EINVAL for a NULL or misaligned pool, max_active or round_steps < 1,
 * preempt_rounds < 0 or reserved != 0. */
elbm_status elbm_server_create(const elbm_server_config *cfg, elbm_server **out);

/* Queue a request (thread-safe, returns at once).  The configuration and the
 * host fields are checked here (ELBM_EINVAL); a request whose footprint can
 * never fit the pool is rejected with ELBM_ENOMEM.  *id receives its id. */
elbm_status elbm_server_submit(elbm_server *srv, const elbm_request *req,
                               int64_t *id);

/* State and times of a request (HOST info). */
elbm_status elbm_server_poll(elbm_server *srv, int64_t id, elbm_request_info *info);

/* Block until request id is done, failed or cancelled, or timeout_s seconds
 * pass (ELBM_ESTATE on timeout or cancellation; timeout_s < 0 waits without
 * limit; ELBM_EDEVICE if the request failed).  Done means its final rho/u
 * are in out_rho/out_u. */
elbm_status elbm_server_wait(elbm_server *srv, int64_t id, double timeout_s);

/* Cancel a queued or running request (thread-safe, returns at once).  The
 * scheduler ends it between rounds as ELBM_REQ_CANCELLED and frees its pool
 * block and host copies; out_rho/out_u are not written.  A request whose
 * last round is already enqueued completes as ELBM_REQ_DONE instead.
 * ELBM_EINVAL for an unknown id, ELBM_ESTATE if it has already finished. */
elbm_status elbm_server_cancel(elbm_server *srv, int64_t id);

/* The simulation of a completed keep_state request (valid until release). */
elbm_status elbm_server_sim(elbm_server *srv, int64_t id, elbm_sim **sim);

/* Free a completed keep_state request's state. */
elbm_status elbm_server_release(elbm_server *srv, int64_t id);

elbm_status elbm_server_get_stats(elbm_server *srv, elbm_server_stats *stats);

/* Stop accepting requests, finish every request that can still be admitted,
 * stop the scheduler and free the server and every kept state.  Requests
 * left queued because kept states hold the pool end as ELBM_REQ_FAILED.
 * The caller's pool may be freed after this returns. */
elbm_status elbm_server_destroy(elbm_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* ELBM_H */
