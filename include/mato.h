/*
 * mato.h -- C ABI of the MI355X (gfx950) alternating-minimisation multi-agent
 * trajectory optimiser of Rastgar et al., "GPU Accelerated Convex
 * Approximations for Fast Multi-Agent Trajectory Optimization" (arXiv 2011.04240).
 *
 * The library implements the while-loop of Algorithm 1 (Sec. III-A): per
 * iteration it builds the linear term rho A_fc^T b_fc of eq. (cost_step_x),
 * applies the precomputed inverse of the KKT matrix of eq. (kkt_step_x) to the
 * x, y and z right-hand sides, forms all pairwise position differences, takes
 * the closed-form alpha/beta projection of eq. (sphere_project) and the d step of
 * eq. (step_d) with d >= 1, and updates the multipliers, eq. (lag_update).
 *
 * Conventions shared by every entry point
 *   - Every function returns a mato_status: 0 = success, < 0 = error (nothing
 *     was changed unless stated), > 0 = warning (results are valid).
 *     mato_last_error() returns a thread-local message for the last failure.
 *   - Pointers to caller data may be host or device pointers (HIP unified
 *     addressing decides); the caller owns them and may reuse them as soon as
 *     the call returns.  Handles own their device memory; *_destroy frees it.
 *   - Work is enqueued on the HIP stream given at creation (NULL = the legacy
 *     default stream).  Calls that return data to the caller synchronise that stream.
 *   - No exception crosses the ABI.  Handles are not thread-safe: one thread
 *     drives a handle at a time.
 *   - Agents are indexed 0..n-1; pair p = (i, j), i < j, is numbered in the row
 *     order of A_fc, eq. (A_f): p(i, j) = i n - i (i + 1) / 2 + (j - i - 1).
 *   - Coefficient arrays are [agent][axis][coef] (axis order x, y, z); pairwise
 *     arrays (multipliers, d e) are [row][time][axis], where the collision rows are
 *     the pairs p(i, j) followed, with static obstacles, by row
 *     n(n-1)/2 + i n_obs + o for agent i and obstacle o.
 *   - Static obstacles (Sec. IV-A: circumscribing spheres) are given per problem as
 *     [x, y, z, l_xy, l_z]: the centre and the semi-axes of the agent-obstacle
 *     clearance spheroid (agent size plus obstacle radius).  They add one row per
 *     agent and obstacle to A_fc, of the same form as an agent pair with the
 *     obstacle's position fixed.
 */
#ifndef MATO_H
#define MATO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mato_status;

#define MATO_OK                   0
#define MATO_ERR_INVALID_ARG     -1  /* a size, pointer or parameter out of range            */
#define MATO_ERR_OUT_OF_MEMORY   -2  /* device allocation failed or HBM budget exceeded      */
#define MATO_ERR_SINGULAR        -3  /* zero pivot or condition estimate above 1e14           */
#define MATO_ERR_NONFINITE       -4  /* NaN or Inf in inputs or state                        */
#define MATO_ERR_HIP             -5  /* a HIP runtime call failed                            */
#define MATO_ERR_UNSUPPORTED     -6  /* valid request the library does not handle (e.g. n > MATO_MAX_AGENTS) */
#define MATO_ERR_NOT_FOUND       -7  /* unknown request or slot id                            */
#define MATO_WARN_NOT_CONVERGED   1  /* iteration cap reached before the residual tolerance  */

#define MATO_MAX_AGENTS 160          /* largest n: the pairwise stage keeps one instant of all
                                        n(n-1)/2 pairs in LDS                                  */
#define MATO_MAX_STAGES 16           /* largest number of stages of a rho schedule             */
#define MATO_MAX_OBSTACLES 1024      /* largest number of static obstacles per problem         */
#define MATO_HISTORY_CAP 4096        /* per-problem residual history entries kept on the device */

/* Trajectory basis of eq. (param): Bernstein polynomials of degree n_coef-1 over
 * [0, t_final] seconds, sampled at T uniformly spaced instants including both ends. */
typedef enum { MATO_BASIS_BERNSTEIN = 0 } mato_basis_kind;
typedef struct {
    int32_t kind;      /* mato_basis_kind                                  */
    int32_t n_coef;    /* coefficients per agent and axis (n_v), 6..16     */
    double  t_final;   /* horizon in seconds, > 0                          */
} mato_basis;

/* Arithmetic of the per-iteration path.  The offline inverse, the coefficients, the
 * linear term g and the refinement residual are always FP64.
 *   MATO_FP64        : every stage in FP64 (reference precision on the GPU).
 *   MATO_FP32        : pairwise stage and multipliers in FP32; the inverse product
 *                      runs on FP32 MFMA (FP32 accumulation) followed by one FP64
 *                      residual correction.
 *   MATO_BF16_REFINED: as MATO_FP32, but the inverse product runs on BF16 MFMA with
 *                      FP32 accumulation over two-term BF16 splits of the inverse and of
 *                      the right-hand side, followed by two FP64 residual corrections.
 * The number of corrections can be overridden with the MATO_REFINE environment
 * variable (0..4). */
typedef enum { MATO_FP64 = 0, MATO_FP32 = 1, MATO_BF16_REFINED = 2 } mato_precision;

/* How the x/y/z step of eq. (kkt_step_x) is solved.
 *   MATO_SOLVE_DENSE     : the precomputed inverse as the method states it, c = K^{-1} [g; b_eq]
 *                          with the (17n)^2 FP64 inverse (Remarks 1-2), applied as a matrix
 *                          product in the plan's precision.
 *   MATO_SOLVE_STRUCTURED: the same c from the block structure of K: A_fc^T A_fc =
 *                          (n I - 1 1^T) (x) P^T P, whose eigenvalues are 0 on the agent mean
 *                          and n on the deviations, so that
 *                              K^{-1} = (1 1^T / n) (x) K_0^{-1} + (I - 1 1^T / n) (x) K_{rho n}^{-1},
 *                              K_s = [[Pddot^T Pddot + s P^T P, A^T], [A, 0]]  (17 x 17 for n_coef = 11),
 *                          in per-agent ordering.  Two per-agent inverses replace the dense one;
 *                          the step runs in FP64 in O(n n_coef^2) per axis.  Not the paper's
 *                          implementation, the same result up to rounding. */
typedef enum { MATO_SOLVE_DENSE = 0, MATO_SOLVE_STRUCTURED = 1 } mato_solve_kind;

typedef struct mato_plan_s*   mato_plan;    /* K^{-1} of eq. (kkt_step_x) for one (n, T, basis, rho) */
typedef struct mato_batch_s*  mato_batch;   /* one or more independent problems iterated together    */
typedef struct mato_server_s* mato_server;  /* continuous-batching request loop                      */

const char* mato_last_error(void);
const char* mato_version(void);

/* ---------------------------------------------------------------- plans ---
 * Offline step (Remarks 1-2): builds P, P-dot, P-ddot (eq. (param)), the
 * boundary matrix A, the KKT matrix
 *     K = [[Q_x + rho A_fc^T A_fc, A_eq^T], [A_eq, 0]],   Q_x = diag(Pddot^T Pddot),
 * of eq. (kkt_step_x) and inverts it on the device in FP64 (Gauss-Jordan with
 * partial pivoting).  K depends on n, T, the basis and rho only; a (= l_xy) and
 * b (= l_z), the spheroid dimensions of eq. (sphere_proposed), are stored for the
 * pairwise stage.  The plan is immutable and may be shared by any number of batches.
 * Errors: INVALID_ARG (n < 2, T < n_coef, n_coef outside 6..16, a, b, rho or t_final
 * not > 0, unknown basis or precision), UNSUPPORTED (n > MATO_MAX_AGENTS),
 * SINGULAR, OUT_OF_MEMORY, HIP. */
mato_status mato_plan_create(int32_t n, int32_t T, const mato_basis* basis,
                             double a, double b, double rho, int32_t precision,
                             void* hip_stream, mato_plan* out);
void        mato_plan_destroy(mato_plan plan);

/* `count` plans with the same n, T, basis, a, b and precision and the penalties
 * rhos[0..count) (a rho schedule, Sec. IV-A); their KKT matrices are inverted in the
 * same launches.  out[m] receives the plan for rhos[m].  Errors as mato_plan_create;
 * on error no plan is returned. */
mato_status mato_plan_create_many(int32_t n, int32_t T, const mato_basis* basis, double a, double b,
                                  const double* rhos, int32_t count, int32_t precision,
                                  void* hip_stream, mato_plan* out);

/* Everything a plan depends on (K depends on the number of obstacles, not on where they are). */
typedef struct {
    int32_t    n;          /* agents, 2..MATO_MAX_AGENTS                                  */
    int32_t    n_obs;      /* static obstacles per problem, 0..MATO_MAX_OBSTACLES          */
    int32_t    T;          /* instants, >= basis.n_coef                                    */
    mato_basis basis;
    double     a, b;       /* l_xy, l_z of the agent-pair clearance spheroid              */
    int32_t    precision;  /* mato_precision                                               */
    int32_t    solve;      /* mato_solve_kind                                              */
} mato_plan_desc;

/* General plan creation: `count` plans described by *desc with the penalties
 * rhos[0..count), inverted in the same launches.  With obstacles K gains
 * rho n_obs P^T P on every agent's diagonal block.  A structured plan takes MATO_FP32
 * (pairwise stage in FP32) or MATO_FP64; BF16_REFINED is INVALID_ARG.  Errors as
 * mato_plan_create; on error no plan is returned. */
mato_status mato_plan_create_ex(const mato_plan_desc* desc, const double* rhos, int32_t count,
                                void* hip_stream, mato_plan* out);

/* The description a plan was created with, and its rho. */
mato_status mato_plan_describe(mato_plan plan, mato_plan_desc* desc, double* rho);

/* Sizes and diagnostics: n, T, n_coef, precision; cond = ||K||_1 ||K^{-1}||_1 (FP64)
 * (structured plans: the larger of the two per-agent estimates). */
mato_status mato_plan_info(mato_plan plan, int32_t* n, int32_t* T, int32_t* n_coef,
                           int32_t* precision, double* cond);

/* Copies the FP64 inverse of K, (17n x 17n for n_coef = 11) row-major, unknowns ordered
 * [c (agent-major, n*n_coef); nu (agent-major, 6n)], into `kinv` (host or device).
 * Structured plans expand their two-block form.  */
mato_status mato_plan_inverse(mato_plan plan, double* kinv);

/* --------------------------------------------------------------- batches ---
 * A batch holds `count` independent problems, problem q using plans[q]; problems
 * with the same plan share one K^{-1} and are advanced together as one
 * matrix-matrix product per iteration.  All plans must have the same precision and
 * solve kind, and must stay alive (not destroyed) while the batch exists.
 * starts/goals: 3 doubles per agent per problem, problems concatenated in order
 * ([problem][agent][x,y,z]); velocities and accelerations at both ends are zero.
 * Creation runs the initialisation of Algorithm 1: multipliers 0, coefficients
 * from the boundary-only minimum-acceleration problem, then alpha, beta and
 * d = max(1, d*) at those positions.  Errors: INVALID_ARG, NONFINITE (starts/goals),
 * OUT_OF_MEMORY, HIP. */
mato_status mato_batch_create(int32_t count, const mato_plan* plans,
                              const double* starts, const double* goals,
                              void* hip_stream, mato_batch* out);

/* As mato_batch_create, for plans with static obstacles: obstacles holds
 * [problem][obstacle][x, y, z, l_xy, l_z], plans[q]->n_obs entries for problem q, problems
 * in order (NULL when no plan has obstacles).  l_xy, l_z must be finite and > 0. */
mato_status mato_batch_create_ex(int32_t count, const mato_plan* plans,
                                 const double* starts, const double* goals, const double* obstacles,
                                 void* hip_stream, mato_batch* out);
void        mato_batch_destroy(mato_batch batch);

/* Enqueue k iterations of Algorithm 1 for every problem not yet converged
 * (asynchronous).  A problem is converged once max_{p,t} ||f_c|| < tol, tested
 * after every iteration on the device (tol <= 0: never).  Iterations are replayed
 * from a captured HIP graph when use_graph != 0. */
mato_status mato_batch_step(mato_batch batch, int32_t k, double tol, int32_t use_graph);

/* Run up to `iters` iterations, checking convergence on the host every
 * `check_every` iterations (>= 1) and stopping once every problem has converged.
 * Returns NOT_CONVERGED if any problem reached the cap. */
mato_status mato_batch_run(mato_batch batch, int32_t iters, double tol, int32_t check_every);

mato_status mato_batch_sync(mato_batch batch);

/* Number of iterations problem q has taken, and whether it converged. */
mato_status mato_batch_status(mato_batch batch, int32_t q, int32_t* iters, int32_t* converged);

/* Coefficients of problem q, [agent][axis][coef], converted to double. */
mato_status mato_batch_coeffs(mato_batch batch, int32_t q, double* c);

/* Per-iteration history of problem q: max and RMS of ||f_c||_2 over pairs and
 * instants (metres) and the smoothness cost sum ||p-ddot||^2 of eq. (cost_proposed).
 * Writes min(cap, iterations, MATO_HISTORY_CAP) entries; any output pointer may be
 * NULL.  The device keeps the first MATO_HISTORY_CAP - 1 iterations, and its last
 * entry follows the latest iteration once more have been taken. */
mato_status mato_batch_residuals(mato_batch batch, int32_t q, double* r_max, double* r_rms,
                                 double* cost, int32_t cap, int32_t* n_written);

/* Checkpoint / parity hooks.  The state of problem q between iterations is
 * (c, lambda, d e): multipliers and the projected points of eq. (b_f)
 * (b_fc = d e - lambda / rho).  c is double [n][3][n_coef]; lambda, proj, d and X
 * are in the batch's scalar (float for MATO_FP32 / MATO_BF16_REFINED, double for
 * MATO_FP64): lambda and proj [n_rows][T][3], d [n_rows][T] (n_rows = n(n-1)/2 + n n_obs), X (positions P c of
 * the current c) [n][3][T].  get_state's `proj` and `d` need mato_batch_debug(batch, 1)
 * before the iteration that produced them; any output pointer may be NULL.
 * set_state rebuilds the linear term from (lambda, proj); c, if given, replaces the
 * reported coefficients and their positions. */
mato_status mato_batch_debug(mato_batch batch, int32_t enable);
mato_status mato_batch_get_state(mato_batch batch, int32_t q, void* c, void* lambda,
                                 void* proj, void* d, void* X);
mato_status mato_batch_set_state(mato_batch batch, int32_t q, const void* c,
                                 const void* lambda, const void* proj);
/* Linear term g = rho A_fc^T b_fc currently held for problem q, [n][3][n_coef]. */
mato_status mato_batch_linear_term(mato_batch batch, int32_t q, void* g);

/* Penalty schedule (Sec. IV-A: inverses cached for several increasing rho, the
 * larger ones used in later iterations).  plans[j * count + q] is problem q's plan in
 * stage j (same n, T and basis as its creation plan; plans[q] must be the creation
 * plan itself); stage j starts after start_iter[j] iterations (start_iter[0] = 0,
 * increasing).  Iteration k of stage j uses rho_j throughout (x-step, d step,
 * multiplier update).  Call before the first iteration; the caller keeps the plans
 * alive while the batch exists.  Errors: INVALID_ARG. */
mato_status mato_batch_set_rho_schedule(mato_batch batch, int32_t stages, const mato_plan* plans,
                                        const int32_t* start_iter);

/* Projection of the alpha/beta step for every problem of the batch: 0 projects the
 * pairwise difference delta onto the spheroid, eq. (sphere_project) (default); 1 projects
 * delta + lambda/rho, the point the objective of eq. (step_alpha) measures against
 * (the exact minimiser for spheres).  Takes effect from the next iteration. */
mato_status mato_batch_set_projection(mato_batch batch, int32_t mode);

/* Pairwise-stage launch shape: pair-instants per workgroup (target) and threads per
 * workgroup (256, 512 or 1024).  Until set: 16384 and 256, with work items shortened so
 * that a batch of few problems still has about four per compute unit.
 * mato_batch_autotune times candidate shapes on the
 * batch's own problems before it is used (state is re-initialised afterwards) and
 * keeps the fastest; results are cached in the file named by MATO_TUNE_CACHE.  */
mato_status mato_batch_set_tiles(mato_batch batch, int32_t items_per_wg, int32_t threads);
mato_status mato_batch_get_tiles(mato_batch batch, int32_t* items_per_wg, int32_t* threads);
mato_status mato_batch_autotune(mato_batch batch, int32_t* items_per_wg, int32_t* threads);

/* Device time (ms, HIP events on the batch stream) of the last mato_batch_step or
 * mato_batch_run call, and of its pairwise launches alone (summed); enabled by
 * mato_batch_timing(batch, 1). */
mato_status mato_batch_timing(mato_batch batch, int32_t enable);
mato_status mato_batch_last_times(mato_batch batch, double* total_ms, double* pairwise_ms,
                                  int32_t* pairwise_launches);

/* --------------------------------------------------------------- serving ---
 * Continuous batching of planning problems with different agent counts.  Requests
 * wait in arrival order and are admitted while a slot is free and the device-memory
 * budget (plans + resident problem state) allows; K^{-1} is cached per agent count
 * (Remarks 1-2) and unused plans are evicted when memory is short.  All resident
 * problems iterate together (one launch per stage per iteration) and leave when
 * max ||f_c|| < tol or after max_iters iterations.  A problem's iterates do not
 * depend on which other problems are resident. */
typedef struct {
    int32_t    T;                  /* instants per problem                                 */
    mato_basis basis;
    double     a, b, rho;          /* spheroid dimensions l_xy, l_z and the penalty rho    */
    int32_t    precision;          /* mato_precision                                       */
    int32_t    max_slots;          /* problems resident at once, >= 1                      */
    double     hbm_budget_bytes;   /* device bytes for plans and resident problems (a problem's
                                      block counts at its power-of-two size class); <= 0: no limit */
    int32_t    chunk;              /* iterations per scheduling step, >= 1                 */
    int32_t    max_iters;          /* iteration cap per problem, >= 1                      */
    double     tol;                /* convergence threshold on max ||f_c|| (metres)        */
    int32_t    projection;         /* 0: project delta (eq. (sphere_project)); 1: delta + lambda/rho */
    int32_t    rho_stages;         /* 0: fixed rho; else stages of a rho schedule (<= MATO_MAX_STAGES) */
    double     rho_values[MATO_MAX_STAGES];  /* rho of each stage (replaces rho)          */
    int32_t    rho_start[MATO_MAX_STAGES];   /* first iteration of each stage: 0, then
                                                increasing multiples of chunk            */
    int32_t    solve;                        /* mato_solve_kind of every plan             */
    int32_t    use_graphs;                   /* 1: replay each step's iterations from HIP
                                                graphs, recaptured when the resident set
                                                changes; 0: launch them one by one        */
} mato_server_config;

/* Errors: INVALID_ARG (configuration out of range), OUT_OF_MEMORY, HIP. */
mato_status mato_server_create(const mato_server_config* cfg, void* hip_stream, mato_server* out);
void        mato_server_destroy(mato_server s);

/* Builds the plans for n_min..n_max ahead of the requests (OUT_OF_MEMORY if the budget
 * cannot hold them). */
mato_status mato_server_warm(mato_server s, int32_t n_min, int32_t n_max);

/* Queues one problem (n agents; starts/goals [n][3], copied).  *id identifies it.
 * Errors: INVALID_ARG, UNSUPPORTED (n > MATO_MAX_AGENTS, or a pairwise stage that does not
 * fit the device), NONFINITE.  A queued request that still cannot be started (its slot
 * set-up fails) is rejected by mato_server_step, as described there. */
mato_status mato_server_submit(mato_server s, int32_t n, const double* starts, const double* goals,
                               int64_t* id);

/* As mato_server_submit, with n_obs static obstacles [n_obs][x, y, z, l_xy, l_z] (copied;
 * plans are cached per agent count and obstacle count).  Errors as mato_server_submit and
 * INVALID_ARG for n_obs outside 0..MATO_MAX_OBSTACLES or semi-axes not > 0. */
mato_status mato_server_submit_ex(mato_server s, int32_t n, const double* starts, const double* goals,
                                  int32_t n_obs, const double* obstacles, int64_t* id);

/* One scheduling step: retire finished problems, admit queued ones, run `chunk`
 * iterations of the resident problems (asynchronously).  Reports resident and
 * queued counts after admission.  A request that can never run is rejected here
 * instead of holding up the queue: its plan could not be built, its slot could not be
 * set up (any error but HIP, which is returned), or with nothing resident the budget
 * still cannot hold its plans and state. */
mato_status mato_server_step(mato_server s, int32_t* running, int32_t* queued);

/* state: 0 queued, 1 resident, 2 finished, 3 rejected; iterations taken, converged
 * flag, last max ||f_c||.  NOT_FOUND for unknown (or already collected) ids. */
mato_status mato_server_poll(mato_server s, int64_t id, int32_t* state, int32_t* iters,
                             int32_t* converged, double* r_max);

/* Coefficients [n][3][n_coef] of a finished problem; forgets the request.
 * NONFINITE if its iteration produced non-finite values.  For a rejected request it
 * writes nothing, forgets the request and returns the reason (OUT_OF_MEMORY, or the
 * status of the failed plan build). */
mato_status mato_server_result(mato_server s, int64_t id, double* c);

mato_status mato_server_stats(mato_server s, double* device_bytes, int32_t* n_plans,
                              int32_t* running, int32_t* queued);

/* Replays an arrival trace in real time: request k (n[k] agents; starts/goals
 * concatenated as [request][agent][3]) arrives arrival_s[k] seconds after the call
 * (non-decreasing).  Writes each request's latency (finish - arrival, seconds), its
 * iterations and convergence flag, and the wall time of the whole trace; results
 * are not kept.  A rejected request reports 0 iterations and converged 0. */
mato_status mato_server_run_trace(mato_server s, int32_t count, const double* arrival_s,
                                  const int32_t* n, const double* starts, const double* goals,
                                  double* latency_s, int32_t* iters, int32_t* converged,
                                  double* wall_s);

/* ------------------------------------------------------ single problem ---
 * Convenience wrappers: a solve is a batch of one (same handle type).
 * mato_solve_run runs Algorithm 1 on one problem: the initialisation, then passes of
 * its while-loop until `iters` passes or max ||f_c|| < tol (tested every check_every
 * passes), as mato_batch_run.  It creates the solve; if the run itself
 * fails (NONFINITE, HIP) *out still holds the solve, for inspection, and the caller
 * destroys it; if creation fails *out is NULL. */
typedef struct mato_batch_s* mato_solve;
mato_status mato_solve_run(mato_plan plan, const double* starts, const double* goals,
                           int32_t iters, double tol, int32_t check_every, mato_solve* out);
mato_status mato_solve_sync(mato_solve s);
mato_status mato_solve_coeffs(mato_solve s, double* c);
mato_status mato_residuals(mato_solve s, double* r_max, double* r_rms, double* cost,
                           int32_t cap, int32_t* n_written);
/* k more iterations (asynchronous, graph-replayed), as mato_batch_step with tol = 0. */
mato_status mato_step(mato_solve s, int32_t k_steps);
/* State hooks of the single problem, as mato_batch_get_state / mato_batch_set_state. */
mato_status mato_get_state(mato_solve s, void* c, void* lambda, void* proj, void* d, void* X);
mato_status mato_set_state(mato_solve s, const void* c, const void* lambda, const void* proj);
void        mato_solve_destroy(mato_solve s);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same whole solve as
 * mato_solve_run + mato_solve_sync + mato_solve_coeffs + mato_residuals +
 * mato_batch_status + mato_solve_destroy, with every device buffer it needs carved
 * from a fixed array of MATO_NOALLOC_SCRATCH_BYTES per device that the library holds
 * until the process ends.  It calls no hipMalloc / hipFree and creates no graph; it is
 * synchronous on the plan's stream and returns when the results are written.
 *   plan         a plan without static obstacles (created beforehand: plan creation
 *                allocates); its precision and solve kind select the arithmetic
 *   starts/goals [n][3] FP64, host or device
 *   c            out [n][3][n_coef] FP64, host or device
 *   r_max, r_rms, cost  out, per iteration as mato_residuals (each may be NULL),
 *                at most `cap` entries, *n_written set (may be NULL)
 *   iters_done, converged  out, as mato_batch_status (each may be NULL)
 * Errors: INVALID_ARG (null plan/starts/goals/c, iters < 0, check_every < 1, a plan
 * with obstacles), UNSUPPORTED (the problem's state does not fit the fixed array: about
 * 12 n(n-1)/2 T bytes in FP32, twice that in FP64, plus under 200 KB), NONFINITE, HIP;
 * NOT_CONVERGED (warning) when tol > 0 is not met.  Calls on one device share its array:
 * the library serialises them with a lock per device (host threads of one process);
 * every call clears what it reads before use, and its results are copied out before
 * it returns. */
#define MATO_NOALLOC_SCRATCH_BYTES (32u << 20)
mato_status mato_solve_noalloc(mato_plan plan, const double* starts, const double* goals,
                               int32_t iters, double tol, int32_t check_every, double* c,
                               double* r_max, double* r_rms, double* cost, int32_t cap,
                               int32_t* n_written, int32_t* iters_done, int32_t* converged);

/* --------------------------------------------------------------- streams ---
 * A HIP stream of the library's own runtime (non-blocking, default priority), for
 * callers that advance several batches concurrently: each batch enqueues its work on
 * the stream given at its creation, so batches on different streams overlap on the
 * device (one's pairwise stage, bound by HBM, beside another's per-problem kernels).
 * Destroy a stream only after the batches using it. */
mato_status mato_stream_create(void** out);
mato_status mato_stream_destroy(void* stream);

/* ---------------------------------------------------------- measurement ---
 * Not part of the method: allocates two device buffers of `bytes` (a positive multiple
 * of 16), fills the source, and times `iters` launches (after one warm-up) of a
 * streaming copy between them (`grid` workgroups of 256 threads, 16-byte nontemporal
 * loads and stores); checks the first and last 64 KiB of the copy and frees both
 * buffers.  Writes the mean time of one copy: the practical ceiling for a stream with
 * equal reads and writes, beside the vendor peak, for the pairwise stage's roofline.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP (also if the copy differs). */
mato_status mato_stream_copy(int64_t bytes, int32_t grid, int32_t iters, void* hip_stream, double* ms_per_copy);

/* Not part of the method: as mato_stream_copy for one buffer of `bytes` updated in
 * place (x <- x/2 + 1, 16-byte nontemporal loads and stores): the access pattern of the
 * multipliers, read and written back at the same addresses.  Checks the first and last
 * 64 KiB against the value the recurrence gives on the host.  Writes the mean time of
 * one pass.  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP (also on a wrong value). */
mato_status mato_stream_update(int64_t bytes, int32_t grid, int32_t iters, void* hip_stream, double* ms_per_update);

/* Not part of the method: as mato_stream_copy for a pure read of one buffer of `bytes`
 * (every float 1.0; 16-byte nontemporal loads; each workgroup writes one partial sum,
 * which the host checks: exact while a workgroup reads at most 2^24 floats, else
 * INVALID_ARG).  Writes the mean time of one pass: the practical ceiling of the
 * pairwise stage's multiplier stream once unchanged multipliers are not written back.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP (also on a wrong sum). */
mato_status mato_stream_read(int64_t bytes, int32_t grid, int32_t iters, void* hip_stream, double* ms_per_read);

#ifdef __cplusplus
}
#endif
#endif /* MATO_H */
