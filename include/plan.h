/*
 * plan.h -- C ABI of the MI355X batched bi-level trajectory planner.
 *
 * The library implements the data-parallel hot path of the bi-level planner
 * of Singh, Shrestha and Albarella, "Bi-Level Optimization Augmented with
 * Conditional Variational Autoencoder for Autonomous Driving in Dense
 * Traffic" (arXiv 2212.02224):
 *
 *   Alg. 1 (Sec. III-B)   sample behavioural inputs p_j ~ N(mu, Sigma);
 *                         solve the lower level for every p_j; residual r_j;
 *                         ConstraintEliteSet (n lowest r), EliteSet (q lowest
 *                         c_u + r); update mu, Sigma (eqs. mean_update,
 *                         cov_update, s_formula); repeat; return the best.
 *   lower level           Step 1: equality-constrained QP (Sec. III-C,
 *                         eqs. over_2 / over_3), Step 2: projection onto the
 *                         constraints of Table ineq_list by the alternating
 *                         minimisation of Alg. 2 (App. "GPU Accelerated Batch
 *                         Projection", eqs. aug_lag .. update_lagrange).
 *
 * Every step runs in HIP kernels on the GPU. The host part only validates,
 * precomputes the sample-independent matrices in FP64 once (Sec. III-C: the
 * KKT inverse is computed once, irrespective of the batch size), and moves
 * a few hundred bytes per request.
 *
 * Conventions
 *   - Coordinates: x along the road (Frenet frame, Sec. II-C), y lateral.
 *   - xi = (c_x, c_y): 22 Bernstein coefficients of degree 10 on
 *     tau = t / t_f, c_x first (eq. param, Sec. V-A).
 *   - p = [y_d1..y_d4, v_d1..v_d4] (eq. behaviour_param, Sec. V-A): lateral
 *     offset and longitudinal velocity set-points of 4 equal horizon parts.
 *   - Time grid t_k = k t_f / (T - 1), k = 0..T-1.
 *   - All host arrays are row-major and owned by the caller unless stated.
 *   - Every function returns a plan_status; nothing throws across the ABI.
 *     plan_last_error() gives a message for the last failing call.
 *   - A handle is not thread-safe; one host thread drives it.
 */
#ifndef PLAN_H
#define PLAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLAN_NC 11      /* coefficients per axis (10th-order polynomial)  */
#define PLAN_NX 22      /* coefficients of xi                              */
#define PLAN_NP 8       /* behavioural inputs                              */
#define PLAN_MAX_T 256  /* horizon samples per request                    */
#define PLAN_MAX_M 32   /* neighbouring vehicles per request              */
#define PLAN_MAX_N 4096 /* behavioural samples per request                */
#define PLAN_MAX_L 16   /* upper-level iterations                         */
#define PLAN_MAX_ROAD 64 /* knots of a road profile                       */
#define PLAN_OBS_DIM 55    /* observation o of the decoder sampler (App. A) */
#define PLAN_LATENT_DIM 2  /* latent z of the decoder sampler               */
#define PLAN_DEC_HIDDEN 1024 /* outputs of decoder blocks 1-4               */
#define PLAN_DEC_HIDDEN5 256 /* outputs of decoder block 5                  */

typedef enum plan_status {
  PLAN_OK = 0,
  PLAN_E_INVALID = -1,     /* bad argument or request (NaN, T/M/N out of set) */
  PLAN_E_NOMEM = -2,       /* workspace / HBM budget too small               */
  PLAN_E_DEVICE = -3,      /* HIP runtime error                              */
  PLAN_E_BUSY = -4,        /* plan_poll: not finished yet                    */
  PLAN_E_UNSUPPORTED = -5, /* configuration the library does not implement   */
  PLAN_E_TIMEOUT = -6      /* a bounded device-side wait gave up (fused_iters) */
} plan_status;

/* plan_result.flags */
#define PLAN_F_INFEASIBLE 1u /* the returned trajectory has residual r > 0 */
#define PLAN_F_WARM 2u       /* iteration 0 sampled from a warm start       */

/*
 * Arithmetic of the lower level (Alg. 2 and the residual of each sample).
 *   PLAN_PREC_FP32        every product and evaluation in FP32 on the vector
 *                         ALUs.
 *   PLAN_PREC_FP16_SPLIT  the dense products (trajectory evaluation W xi, the
 *                         sums N^T g over the horizon and the xi-update
 *                         A^-1 rhs) on the matrix cores in FP16 with FP32
 *                         accumulation; every operand is split into a high
 *                         and a low FP16 half and three products recover
 *                         about 22 significant bits (the low x low term is
 *                         dropped). Tables are built in FP64; everything
 *                         between the products (projections, clips,
 *                         residual) stays FP32. Requires every T <= 128;
 *                         values beyond the FP16 range (|v| > 65504 after the
 *                         scalings) give NaN residuals, which rank last.
 *   PLAN_PREC_FP32_MFMA   the same dense products on the matrix cores in
 *                         FP32 (FP32 operands, FP32 accumulation; no
 *                         splitting), everything else as PLAN_PREC_FP32.
 *                         Groups of 16 samples per workgroup (8 for small
 *                         launches), so it pays on large batches (thousands
 *                         of samples in flight); requires every T <= 128.
 * All modes draw the same samples and use the same selection and update;
 * a request's results depend on the mode, never on what else runs with it.
 */
typedef enum plan_precision {
  PLAN_PREC_FP32 = 0,
  PLAN_PREC_FP16_SPLIT = 1,
  PLAN_PREC_FP32_MFMA = 2
} plan_precision;

/*
 * Behavioural inputs p (eq. behaviour_param, Sec. II-B). Both use the
 * 8 slots of p (and of mu, Sigma):
 *   PLAN_BEHAV_SETPOINTS  p = [y_d1..y_d4, v_d1..v_d4]: lateral offset and
 *                         velocity set-points of 4 equal horizon parts,
 *                         tracked by c_l and c_v of the lower-level cost
 *                         (Sec. V-A); the final boundary is ydot(t_f) = 0.
 *   PLAN_BEHAV_GOALS      p = [x_f - x0, y_f, 0, ..., 0]: a goal position
 *                         (the Batch-MPC baseline of Sec. V-A), x_f measured
 *                         from the ego like every position the planner sees;
 *                         the lower-level cost is the smoothness term c_s
 *                         alone and the final boundary is eq. final_boundary
 *                         (x, y, ydot)(t_f) = (x_f, y_f, 0). Only p[0], p[1]
 *                         are drawn; the other slots stay 0.
 * The initial sampler of a request without a warm start draws, per sample,
 * one lane centre of lane_c plus N(0, lane_sigma^2) for the lateral inputs
 * and U(vd_lo, vd_hi] for the velocities (goal: x_f - x0 = t_f times such a
 * velocity) (plan_sampler_t RANDOM), or takes sample j from a fixed grid
 * (GRID: lane centre j mod 3, velocity at the midpoint of bin floor(j/3) of
 * ceil(N/3) equal bins of (vd_lo, vd_hi], held over the horizon). With
 * upper_iters = 1 the grid gives the MPC-Grid baseline of Sec. V-A.
 * DECODER: the learned sampler of Sec. III-D / App. A at inference. Sample j
 * is the decoder MLP (weights from plan_set_decoder) applied to [o, z_j],
 * o the request's observation and z_j ~ N(0, I) (2-d: the Box-Muller pair of
 * Philox block (j, 0, 0, 0) under the request's seed); with goal positions
 * its p[2..7] are 0. The distribution before the first update is then the
 * sample mean and covariance (normalised by N) of the N decoder samples.
 */
typedef enum plan_behaviour { PLAN_BEHAV_SETPOINTS = 0, PLAN_BEHAV_GOALS = 1 } plan_behaviour;
typedef enum plan_sampler_t {
  PLAN_SAMPLER_RANDOM = 0,
  PLAN_SAMPLER_GRID = 1,
  PLAN_SAMPLER_DECODER = 2
} plan_sampler_t;

/*
 * Configuration. plan_config_init() fills the defaults; every point the paper
 * leaves open is a field here.
 *   T_set/M_set     horizon lengths and obstacle counts that get precomputed
 *                   matrices; a request must use one of each.
 *   t_f             horizon [s].
 *   max_N           largest sample count of a request (<= PLAN_MAX_N).
 *   max_requests    request slots resident on the device at once.
 *   sample_budget   rows of per-sample device memory (samples, coefficients,
 *                   residual, cost: 104 bytes each) shared by the resident
 *                   requests; a request takes N contiguous rows. With
 *                   max_requests this is the HBM budget of admission.
 *   served_run_ahead  served mode, 0..3: how many upper iterations the host
 *                   may enqueue beyond the one the GPU is running. 0 (the
 *                   default): plan_progress prepares the next iteration
 *                   while the GPU runs the current one and enqueues it when
 *                   that one has finished, so a request submitted meanwhile
 *                   joins it. Larger values keep the GPU busier (more
 *                   throughput) but a new request waits behind the
 *                   iterations already enqueued (more latency).
 *   fused_iters     PLAN_PREC_FP32 only, 0 (the default) or 1. 1: all L
 *                   upper iterations of a launch group in one launch; the
 *                   selection and update of each request run on the device
 *                   by the workgroup that finishes its last samples, and the
 *                   request's next iteration starts as soon as its update
 *                   has run (no per-iteration launches or host round trips).
 *                   Results are bitwise those of the per-iteration launches.
 *                   Measured on MI355X it is slower than back-to-back
 *                   per-iteration launches (whose gaps are about a
 *                   microsecond): the workgroups' device-scope release and
 *                   acquire across the eight L2 caches and the selection's
 *                   registers cost more than the launches save. In served
 *                   mode with fused_iters = 1 each plan_progress call
 *                   enqueues the whole solve of the requests it admits
 *                   (served_run_ahead is then unused).
 *   fused_wait_us   bound on how long a workgroup of a fused launch waits
 *                   for an update before it gives up (default 1 s, far
 *                   above any real wait); the requests whose updates did
 *                   not all run then fail with PLAN_E_TIMEOUT, and the
 *                   launch still ends.
 *   proj_iters      K, iterations of Alg. 2 (its maxiter).
 *   upper_iters     L, iterations of Alg. 1 (its N).
 *   frac_ces/es     n = max(q, round(frac_ces N)), q = max(1, round(frac_es N))
 *                   (150 and 50 of 1000 in Sec. V-A).
 *   eta, gamma      learning rate and temperature of eqs. mean_update,
 *                   cov_update, s_formula (gamma = 0.9 in Sec. V-A).
 *   rho             penalty of eq. aug_lag.
 *   k_p, k_v        PD gains and w_s, w_l, w_v weights of c_s, c_l, c_v
 *                   (Sec. II-C).
 *   cov_jitter      epsilon of chol(Sigma + eps I) before sampling.
 *   v_min .. y_ub   bounds of Table ineq_list; ell_a, ell_b the ellipse
 *                   denominators of its collision row; v_eps the speed floor
 *                   of the curvature residual.
 *   lane_c, lane_sigma, vd_lo, vd_hi   the structured initial sampler (used
 *                   when a request has no warm start).
 *   device_workspace/workspace_bytes   optional caller-owned device memory
 *                   (e.g. a torch tensor); NULL lets the library allocate.
 *                   The size is the HBM budget: see plan_workspace_bytes().
 *   stream          hipStream_t the library enqueues on (NULL: its own).
 */
typedef struct plan_config {
  int32_t T_set[4];
  int32_t n_T;
  int32_t M_set[8];
  int32_t n_M;
  double t_f;
  int32_t max_N;
  int32_t max_requests;
  int32_t proj_iters;
  int32_t upper_iters;
  double frac_ces, frac_es;
  double eta, gamma, rho;
  double k_p, k_v, w_s, w_l, w_v;
  double cov_jitter;
  double v_min, v_max, a_max, kappa_max, c_max, y_lb, y_ub;
  double ell_a, ell_b, v_eps;
  double lane_c[3];
  double lane_sigma, vd_lo, vd_hi;
  int32_t precision;
  int32_t trace; /* nonzero: keep per-iteration elite sets and mu, Sigma */
  int32_t behaviour; /* plan_behaviour */
  int32_t sampler;   /* plan_sampler_t: initial sampler */
  int32_t served_run_ahead; /* served mode: iterations enqueued ahead (0..3) */
  int32_t fused_iters;   /* 1: every upper iteration of a launch group in one launch */
  int32_t fused_wait_us; /* bound of a device-side wait of the fused launch [us] */
  int64_t sample_budget; /* sample rows resident at once (0: max_requests * max_N) */
  void *device_workspace;
  size_t workspace_bytes;
  void *stream;
} plan_config;

/*
 * One planning request (one call of Alg. 1).
 *   request_id   caller's tag, echoed nowhere but useful for logs.
 *   session_id   key of the device-resident warm start (0 = none): after a
 *                request of a session finishes, its mu, Sigma stay on the
 *                device and seed the next request of that session
 *                (warm start across planning cycles, Sec. IV).
 *   seed         64-bit key of the sample stream (Philox4x32-10).
 *   N, M, T      samples, neighbours, horizon samples.
 *   ego          b_0 = (x0, y0, vx0, vy0, ax0, ay0) (eq. boundary_cond_initial).
 *   obstacles    host, M x 4 doubles: (x, y, vx, vy) at t = 0; neighbours move
 *                at constant velocity x_o(t) = x + vx t (Fig. learned_sampler).
 *   kappa_road   road curvature (0: straight road) when no profile is given.
 *   n_road, road_x0, road_dx, road
 *                road profile along x (Table ineq_list: the centripetal row's
 *                kappa(x(t)) and the lane limits y_lb(x(t)), y_ub(x(t)), the
 *                bound e(xi) of eq. lane_reform, taken at each iterate's
 *                position): road is host, n_road x 3 doubles (kappa, y_lb,
 *                y_ub) at x = road_x0 + i road_dx, x in the same coordinate
 *                as ego[0] (not relative to it); linear between knots,
 *                constant beyond them. Copied at the call; the caller keeps
 *                ownership. n_road = 0: kappa_road and the config's y_lb,
 *                y_ub. n_road <= PLAN_MAX_ROAD, road_dx > 0 if n_road > 1,
 *                y_lb < y_ub at every knot, all finite; else the request
 *                fails with PLAN_E_INVALID. Requests with a profile run in
 *                lower-level launches of their own.
 *   mu0, sigma0  optional initial distribution (8, 8x8); if NULL the session
 *                warm start is used, else the structured initial sampler.
 *   first_iter   index of the first upper iteration (normally 0). It keys
 *                the sample stream, so a request started from the
 *                distribution of iteration l with first_iter = l draws the
 *                same samples as iteration l of a longer run.
 *   observation  host, PLAN_OBS_DIM doubles: the observation o the decoder
 *                sampler conditions on (Sec. V-A lists ego heading and
 *                speeds, the ten nearest neighbours and the road boundary;
 *                its layout and scaling are those the weights were trained
 *                with). Required, and finite, when the config's sampler is
 *                PLAN_SAMPLER_DECODER; ignored otherwise. Copied at the call.
 */
typedef struct plan_request {
  uint64_t request_id;
  uint64_t session_id;
  uint64_t seed;
  int32_t N, M, T;
  double ego[6];
  const double *obstacles;
  double kappa_road;
  const double *mu0;
  const double *sigma0;
  int32_t first_iter;
  int32_t n_road;
  double road_x0, road_dx;
  const double *road;
  const double *observation;
} plan_request;

/*
 * Result of one request (Alg. 1, return step): the sample of the final
 * EliteSet with the smallest augmented cost c_u + r (ties: lower index), its
 * behavioural input and projected trajectory, and the sampling distribution
 * after the last update (the warm start of the next planning cycle).
 * The selection ranks samples by the lower level's own residual and cost
 * (FP32, or FP16-split products with FP32 sums); the returned trajectory's
 * residual and upper cost are then evaluated again in FP64 (its Bernstein
 * polynomial, every row of Table ineq_list at every instant t_k), and
 * PLAN_F_INFEASIBLE is set from that FP64 residual.
 *   traj_xy   caller-owned, nullable: T x 2 doubles (x, y at t_k, k = 0..T-1,
 *             FP64 on the device) of the returned trajectory. Set it before
 *             the call that fills the result (plan_solve_batch, plan_collect,
 *             plan_poll, plan_mpc_run); the library keeps the pointer and
 *             writes T x 2 values there when the request succeeded.
 */
typedef struct plan_result {
  int32_t status;
  uint32_t flags;
  int32_t best_index;
  int32_t iterations;
  double p_best[PLAN_NP];
  double xi_best[PLAN_NX];
  double cost_upper; /* c_u of the returned trajectory (FP64 evaluation) */
  double residual;   /* r of the returned trajectory (FP64 evaluation)   */
  double mu[PLAN_NP];
  double sigma[PLAN_NP * PLAN_NP];
  double latency_s;  /* submit -> completion (served path), else solve time */
  double *traj_xy;   /* caller-owned T x 2 or NULL (see above)            */
} plan_result;

typedef struct plan_handle plan_handle; /* opaque, owned by the library */

/* Fill *cfg with the defaults (T_set {50, 100}, M_set {4, 10, 20}, t_f 5,
 * K 20, L 5, n/q fractions 0.15/0.05, gamma 0.9, eta 0.6, rho 1, ...). */
void plan_config_init(plan_config *cfg);

/* Device bytes the library needs for cfg (tables + max_requests slots). */
size_t plan_workspace_bytes(const plan_config *cfg);

/* Sizes of the ConstraintEliteSet (*n_ces) and EliteSet (*n_es) of Alg. 1
 * for a request of N samples under cfg: q = max(1, round(frac_es N)),
 * n = max(q, round(frac_ces N)), both at most N (150 and 50 at N = 1000,
 * Sec. V-A). PLAN_E_INVALID for a NULL argument or N outside [1, max_N]. */
plan_status plan_elite_sizes(const plan_config *cfg, int32_t N, int32_t *n_ces, int32_t *n_es);

/* Validate cfg, precompute the sample-independent matrices in FP64 (once,
 * Sec. III-C), and set up device memory. *out receives the handle.
 * Errors: PLAN_E_INVALID (cfg), PLAN_E_NOMEM (workspace too small),
 * PLAN_E_DEVICE (HIP). */
plan_status plan_create(const plan_config *cfg, plan_handle **out);

/* Release everything the handle owns (not the caller's workspace). */
void plan_destroy(plan_handle *h);

/* Message of the last failing call on h (or of plan_create if h is NULL). */
const char *plan_last_error(const plan_handle *h);

/* Solve n requests (Alg. 1 each) and wait. out[i] gets request i's result;
 * a bad request fails alone (its status: PLAN_E_INVALID, or PLAN_E_NOMEM for
 * an N beyond the sample budget), the call returns the worst status.
 * Requests beyond max_requests or the budget run in successive groups; if a
 * group cannot run (a device error), it and every later request get that
 * status. */
plan_status plan_solve_batch(plan_handle *h, const plan_request *reqs,
                             int32_t n, plan_result *out);

/* Device-resident form of plan_solve_batch for timing with inputs already in
 * HBM: plan_stage uploads n <= max_requests requests; plan_launch enqueues
 * the whole hot path of all staged requests on the stream and returns
 * without waiting (each call repeats the same work from the staged inputs);
 * plan_collect waits and copies the results out. */
plan_status plan_stage(plan_handle *h, const plan_request *reqs, int32_t n);
plan_status plan_launch(plan_handle *h);
plan_status plan_collect(plan_handle *h, plan_result *out);

/* Lower level only (Alg. 1 Steps 1-2 and the residual/cost) for the given
 * behavioural inputs p (host, N x 8), one request's scene. Outputs (host,
 * nullable): xi_bar, xi_star (N x 22), resid, cost_upper (N; the lower
 * level's own values, as the selection sees them). PLAN_E_INVALID for a bad
 * request or non-finite p, PLAN_E_NOMEM if N exceeds the sample budget. */
plan_status plan_lower_solve(plan_handle *h, const plan_request *req,
                             const double *p, int32_t N, double *xi_bar,
                             double *xi_star, double *resid,
                             double *cost_upper);

/* plan_lower_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels on the same inputs, with every array on the
 * device and the library's working memory for the call (the request
 * descriptor, the launch arrays and the free-coefficient rows of the
 * samples) in a static device array of about 260 KB, one per GPU, held until
 * the process ends; its address on the handle's device is looked up once, at
 * plan_create. The call allocates nothing, enqueues on the handle's stream
 * and waits for its own work before returning.
 *   p           device, N x 8 floats: the behavioural inputs (read only;
 *               not checked for finiteness: non-finite values give NaN
 *               outputs).
 *   xi_bar, xi_star   device, N x 22 doubles each, or both NULL.
 *   resid, cost_upper device, N floats each (the lower level's own values).
 * The caller's device arrays must be ready when the handle's stream reaches
 * the call (e.g. synchronise the stream that wrote them first).
 * N <= PLAN_MAX_N (the scratch array's row count; larger N: PLAN_E_NOMEM)
 * and N <= max_N. Every call rewrites the parts it uses, so nothing is
 * cleared between calls; two calls that overlap on one GPU (other host
 * threads or handles) share the array and race. Errors as plan_lower_solve
 * (PLAN_E_INVALID for a bad request or a NULL array, PLAN_E_BUSY while
 * served requests are in flight). Slot 0 of a staged batch is replaced. */
plan_status plan_lower_solve_static(plan_handle *h, const plan_request *req,
                                    const float *p, int32_t N, double *xi_bar,
                                    double *xi_star, float *resid,
                                    float *cost_upper);

/* Per-iteration record of the last plan_solve_batch / plan_collect for
 * staged request i (needs cfg.trace): samples p (L x N x 8), residuals and
 * costs (L x N), ConstraintEliteSet (L x n) and EliteSet (L x q) sample
 * indices (each list in increasing sample index), mu (L x 8) and Sigma
 * (L x 64) after each update. Any pointer may be NULL. */
plan_status plan_get_trace(plan_handle *h, int32_t i, double *p, double *resid,
                           double *cost_upper, int32_t *ces, int32_t *es,
                           double *mu, double *sigma);

/*
 * Served mode: continuous batching at the granularity of one upper iteration
 * of Alg. 1. plan_submit validates and queues a request (copying everything
 * it points to) and returns a ticket. Each plan_progress call admits queued
 * requests, first come first served, while a request slot and N contiguous
 * sample rows of the budget are free; and enqueues one upper iteration for
 * every resident request at once (whatever their sizes and iteration
 * indices, in the same kernel launches). The host waits for the GPU only
 * as far as plan_config.served_run_ahead asks, so its own work overlaps the
 * GPU's. A request whose L-th iteration is enqueued has its result copied
 * back; it is retired (result ready, slot and rows free) by the first
 * plan_progress or plan_poll call after the copy has arrived. A
 * plan_progress call with nothing to enqueue waits for the oldest pending
 * result instead, so every call makes progress. plan_poll returns
 * PLAN_E_BUSY until the ticket's request is done, then its result
 * (latency_s: submit to the call that saw it complete) and forgets the
 * ticket. A request's arithmetic does not depend on what else is resident,
 * so its result equals the one of plan_solve_batch bit for bit. A request
 * with a session_id is admitted only once no other request of its session is
 * in flight (it, and the queue behind it, wait for that one to retire), so
 * it starts from the distribution the session's previous request left,
 * whatever the timing. plan_submit fails with PLAN_E_NOMEM for an N beyond
 * the sample budget. *n_active / *n_queued (nullable) receive the
 * in-flight (resident or retiring) and waiting counts. plan_submit fails
 * with PLAN_E_INVALID for a bad request. The batch calls (plan_solve_batch,
 * plan_stage, plan_mpc_run, plan_set_decoder) return PLAN_E_BUSY while any
 * served request is queued or in flight.
 */
plan_status plan_submit(plan_handle *h, const plan_request *req, uint64_t *ticket);
plan_status plan_progress(plan_handle *h, int32_t *n_active, int32_t *n_queued);
plan_status plan_poll(plan_handle *h, uint64_t ticket, plan_result *out);

/* Every finished served request at once, for a serving loop that would
 * otherwise poll ticket by ticket: retires what has completed (as plan_poll
 * does), then moves up to max_n finished results, in ticket order, into
 * out[0..*n_done) with their tickets in tickets[0..*n_done), and forgets
 * those tickets; the rest stay for the next call. out[i].traj_xy, if set
 * before the call, must hold the longest horizon of the config (T x 2
 * doubles) and receives the returned trajectory. A ticket is returned by
 * exactly one of plan_poll and plan_poll_done. PLAN_E_INVALID for NULL
 * arrays with max_n > 0 or a negative max_n; *n_done = 0 when nothing has
 * finished. */
plan_status plan_poll_done(plan_handle *h, uint64_t *tickets, plan_result *out, int32_t max_n,
                           int32_t *n_done);

/*
 * Receding-horizon closed loop (MPC-Bi-Level, Sec. V-A "MPC Baselines").
 * Every episode replans with Alg. 1 once per cycle, executes the first
 * n_exec instants of the trajectory it got (5 in Sec. V-A), and replans
 * from the state reached. The first upper iteration of cycles 2.. draws
 * from (init):
 *   PLAN_MPC_SAMPLER  the initial sampler, as at the first cycle of a
 *                     request without a warm start. Sec. V-A feeds each
 *                     cycle's observation to the learned sampler; the
 *                     structured sampler of plan_config stands in for it.
 *   PLAN_MPC_WARM     the distribution the episode's previous cycle left
 *                     (warm start across planning cycles, Sec. IV "Trajectory
 *                     Sampling Approaches"), kept on the device in its
 *                     session. Sigma shrinks with every update, so over many
 *                     cycles the samples concentrate on one behaviour.
 * The loop runs on the library's stream without a
 * host round trip between cycles: after a cycle's L upper iterations an
 * advance kernel (one workgroup per episode, FP64) evaluates the returned
 * trajectory at t_0 .. t_{n_exec}, tests every executed instant against
 * every neighbour's ellipse (the collision row of Table ineq_list: a
 * collision when ((x - x_o) / a)^2 + ((y - y_o) / b)^2 < 1, a = ell_a,
 * b = ell_b), and writes the next cycle's request in place.
 *
 *   reqs      the first cycle's requests, one per episode (n <= max_requests);
 *             with PLAN_MPC_WARM each needs a distinct nonzero session_id
 *             (optional otherwise; nonzero ids must be distinct, and the
 *             last cycle's mu, Sigma stay in them). Episode i at cycle c
 *             plans from the state its cycle c - 1 reached at t_{n_exec}
 *             (held if that plan failed), with seed reqs[i].seed + c and the
 *             neighbours at scene time s = (c n_exec) t_f / (T - 1), the
 *             position of neighbour m formed as fma(v_m, s, p_m) from its
 *             first-cycle position p_m and velocity v_m (constant-velocity
 *             traffic, as in the collision row). Instant k of cycle c is
 *             tested against the neighbours at s = (c n_exec + k) t_f / (T - 1).
 *   cycles    planning cycles, >= 1.
 *   n_exec    instants executed per cycle, 1 <= n_exec <= T - 1.
 *   init      PLAN_MPC_SAMPLER or PLAN_MPC_WARM (above).
 *   log       caller-owned host arrays, each nullable, row-major:
 *               ego       n x (cycles + 1) x 6  b_0 of every cycle, then the
 *                                                final state
 *               xi        n x cycles x 22       trajectory returned by each cycle
 *               mu, sigma n x cycles x 8, x 64  distribution after each cycle
 *               cost      n x cycles x 2        (c_u, r) of the returned sample
 *               collided  n x cycles            1 if an executed instant
 *                                                meets a neighbour's ellipse
 *               status    n x cycles            the cycle's plan status
 *             A NULL log (or NULL members) records nothing; the call
 *             allocates device memory for the requested logs and frees it.
 *   out       nullable; n results of the last cycle (its mu, Sigma are the
 *             episodes' warm starts, kept in their sessions).
 * Errors: PLAN_E_INVALID for a bad request (the whole call fails), a missing
 * or repeated session_id, n, cycles, n_exec or init out of range; PLAN_E_BUSY
 * while served requests are in flight; PLAN_E_NOMEM if the log memory cannot
 * be allocated. A batch staged before the call is replaced.
 */
typedef enum plan_mpc_init { PLAN_MPC_SAMPLER = 0, PLAN_MPC_WARM = 1 } plan_mpc_init;

typedef struct plan_mpc_log {
  double *ego;
  double *xi;
  double *mu;
  double *sigma;
  double *cost;
  int32_t *collided;
  int32_t *status;
} plan_mpc_log;

plan_status plan_mpc_run(plan_handle *h, const plan_request *reqs, int32_t n,
                         int32_t cycles, int32_t n_exec, int32_t init,
                         plan_mpc_log *log, plan_result *out);

/*
 * Weights of the decoder sampler (App. A, decoder table: five blocks of
 * Linear, BatchNorm and ReLU with 1024, 1024, 1024, 1024 and 256 outputs,
 * then Linear to the PLAN_NP behavioural inputs; the input is [o, z],
 * PLAN_OBS_DIM + PLAN_LATENT_DIM values). All host, row-major doubles:
 *   W[i]   block i's Linear weights, out x in (W[0]: 1024 x 57, W[1..3]:
 *          1024 x 1024, W[4]: 256 x 1024, W[5]: PLAN_NP x 256)
 *   b[i]   its bias (out)
 *   bn_gamma[i], bn_beta[i], bn_mean[i], bn_var[i]   BatchNorm of blocks
 *          0..4 in inference form: gamma (h - mean) / sqrt(var + eps) + beta
 *   bn_eps eps of that form (PyTorch's default is 1e-5)
 */
typedef struct plan_decoder {
  const double *W[6];
  const double *b[6];
  const double *bn_gamma[5];
  const double *bn_beta[5];
  const double *bn_mean[5];
  const double *bn_var[5];
  double bn_eps;
} plan_decoder;

/* Load the decoder sampler's weights (needed before any request of a
 * handle whose config has sampler = PLAN_SAMPLER_DECODER). The library
 * folds each BatchNorm and bias into its Linear layer in FP64 and keeps the
 * layers on the device: blocks 1-5 as FP16 high/low pairs on the matrix
 * cores (block 1 with its 57 inputs padded to 64; three products recover
 * about 22 significant bits, as the lower level's FP16-split form does), the
 * output layer in FP32. The
 * arrays are copied; the call waits for the upload. PLAN_E_INVALID for a
 * handle without the decoder sampler, a missing or non-finite array, a
 * variance with var + eps <= 0, or weights beyond 1e30 in magnitude;
 * PLAN_E_BUSY while served requests are in flight. Hidden activations must
 * stay below 65504 in magnitude (FP16 range). */
plan_status plan_set_decoder(plan_handle *h, const plan_decoder *dec);

/* Kernel timing by HIP events recorded on the library's stream around every
 * launch of plan_launch / plan_solve_batch / plan_progress. enable != 0
 * starts recording (and clears the totals); plan_profile_read waits for the
 * stream and returns the summed milliseconds and launch counts per part:
 * [0] lower level (sampling, Steps 1-2, residual/cost), [1] selection /
 * update, [2] decoder sampler (all of its kernels for one upper iteration
 * count as one launch). */
plan_status plan_profile(plan_handle *h, int32_t enable);
plan_status plan_profile_read(plan_handle *h, double ms[3], int64_t count[3]);

#ifdef __cplusplus
}
#endif
#endif
