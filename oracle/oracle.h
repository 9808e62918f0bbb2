/*
 * oracle.h -- FP64 CPU oracle for the bi-level planner of arXiv 2212.02224
 * (Singh, Shrestha, Albarella, "Bi-Level Optimization Augmented with
 * Conditional Variational Autoencoder for Autonomous Driving in Dense
 * Traffic").
 *
 * TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU baseline of
 * the benchmark may load this library. It shares no code, header, table or
 * constant generator with the HIP path; the HIP path never calls it.
 *
 * Conventions
 *   xi      = (c_x, c_y): 22 polynomial coefficients (Sec. III-A), c_x first.
 *   p       = [y_d1..y_d4, v_d1..v_d4] (Sec. V-A, eq. behaviour_param).
 *   ego     = b_0 = (x0, y0, vx0, vy0, ax0, ay0) (eq. boundary_cond_initial).
 *   obs     = M rows of (x, y, vx, vy) at t = 0; neighbours move on straight
 *             lines at constant velocity.
 *   All arrays are row-major, caller-owned.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NC 11 /* coefficients per axis (10th-order polynomial) */
#define ORC_NX 22 /* coefficients of xi                              */
#define ORC_NP 8  /* behavioural inputs                              */
#define ORC_NEQ 7 /* equality rows: 3 initial per axis + final ydot   */
#define ORC_NEQ_MAX 9 /* plus x(t_f) = x_f, y(t_f) = y_f with goals    */

typedef struct orc_params {
  int T;          /* samples of the horizon, t_k = k t_f/(T-1)          */
  int M;          /* neighbouring vehicles                              */
  int K;          /* projection iterations (Alg. 2 maxiter)            */
  int L;          /* upper-level iterations (Alg. 1 N)                 */
  double t_f;     /* horizon [s]                                       */
  double k_p, k_v;          /* PD tracking gains (Sec. II-C)             */
  double w_s, w_l, w_v;     /* weights of c_s, c_l, c_v                  */
  double rho;               /* penalty of eq. aug_lag                    */
  double ell_a, ell_b;      /* ellipse denominators (Table ineq_list)    */
  double v_min, v_max, a_max, kappa_max, c_max, y_lb, y_ub;
  double v_eps;             /* speed floor of the curvature residual     */
  double eta, gamma;        /* eqs. mean_update, cov_update, s_formula   */
  double cov_jitter;        /* epsilon added before the Cholesky factor  */
  double frac_ces, frac_es; /* n = max(q, round(frac_ces N)), q = ...    */
  double lane_c[3];         /* initial sampler: lateral lane centres     */
  double lane_sigma;        /* initial sampler: offset noise (std)       */
  double vd_lo, vd_hi;      /* initial sampler: U(vd_lo, vd_hi]          */
  int behaviour; /* 0: p = [y_d1..4, v_d1..4] (set-points, Sec. V-A);
                    1: p = [x_f - x0, y_f, 0 ...] (goal positions, eq.
                    behaviour_param and eq. final_boundary)             */
  int sampler;   /* 0: random initial sampler; 1: fixed grid at the
                    first upper iteration                              */
} orc_params;

typedef struct orc_scene {
  double ego[6];
  double kappa_road;
  const double *obs; /* M x 4 */
  /* Road profile along x (Table ineq_list: kappa(x(t)) of the centripetal
   * row, lane limits y_lb(x(t)), y_ub(x(t))): n_road knots at road_x0 +
   * i road_dx holding (kappa, y_lb, y_ub), linear between knots and constant
   * beyond the ends. n_road = 0: the constant kappa_road and the parameters'
   * y_lb, y_ub. */
  int n_road;
  double road_x0, road_dx;
  const double *road; /* n_road x 3 */
} orc_scene;

/* Defaults of every reading the paper leaves open. */
void orc_default_params(orc_params *par);

/* Elite-set sizes for N samples. */
void orc_elite_sizes(const orc_params *par, int N, int *n_ces, int *n_es);

/* Basis of eq. param: W, Wd, Wdd are T x 11. */
void orc_basis(int T, double t_f, double *W, double *Wd, double *Wdd);

/* Lower-level cost c_s + c_l + c_v summed over t (eq. cost) of one xi. */
double orc_lower_cost(const orc_params *par, const double *p, const double *xi);

/* Step 1 of Alg. 1: equality-constrained QP, eq. over_2; N x 22 out. */
int orc_step1(const orc_params *par, const orc_scene *sc, const double *p,
              int N, double *xi_bar);

/* Step 2 of Alg. 1 by Alg. 2. p (N x 8) gives the goal positions of the
 * final boundary rows (needed with behaviour = 1, else nullable). xi_iter
 * (nullable) receives N x (K+1) x 22: the initial iterate and every
 * xi-update. */
int orc_project(const orc_params *par, const orc_scene *sc,
                const double *xi_bar, const double *p, int N, double *xi_star,
                double *xi_iter);

/* Alg. 2 for one sample with every intermediate, iterations k = 0..K (each
 * output nullable, row k of each array belongs to iteration k):
 *   xi   (K+1) x 22          xi^0 = xi_bar, xi^k the k-th xi-update (eq.
 *                            split_xy)
 *   h    (K+1) x 2(M+2)T     targets of the pass at xi^k (rows of F)
 *   s, e (K+1) x 2T          lane slack and lane bound e of that pass
 *   da   (K+1) x T           d_a of that pass
 *   lam  (K+1) x 22          lambda^0 = 0, lambda^k after the step
 *                            update_lagrange of iteration k
 * The xi-update of iteration k uses lambda^(k-1), h^(k-1), s^(k-1), e^(k-1).
 * p as for orc_project. The same code as orc_project computes it. */
int orc_project_dump(const orc_params *par, const orc_scene *sc,
                     const double *xi_bar, const double *p, double *xi,
                     double *h, double *s, double *e, double *da, double *lam);

/* One target pass of Alg. 2 (steps split_alpha_o .. update_slack) for one
 * xi. h is 2(M+2)T (rows of F), s is 2T, da_prev/da_out are T. */
void orc_targets(const orc_params *par, const orc_scene *sc, const double *xi,
                 const double *da_prev, double *h, double *s, double *da_out);

/* Residual r_j (Alg. 1, constraint residual) and upper cost c_u. */
void orc_residual_cost(const orc_params *par, const orc_scene *sc,
                       const double *xi, int N, double *r, double *cu);

/* ConstraintEliteSet / EliteSet of Alg. 1. ces: n indices, es: q indices,
 * c_es: the q augmented costs c_u + r, all sorted ascending (key, index). */
void orc_select(const double *r, const double *cu, int N, int n, int q,
                int *ces, int *es, double *c_es);

/* Distribution update, eqs. mean_update, cov_update, s_formula. */
void orc_update(const orc_params *par, const double *mu, const double *Sigma,
                const double *p, const int *es, const double *c_es, int q,
                double *mu_out, double *Sigma_out);

/* Lower Cholesky factor of A + jitter I (n x n). Returns 0 on success. */
int orc_cholesky(const double *A, int n, double jitter, double *Lout);

/* Philox4x32-10 (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* Moments of the structured initial sampler. */
void orc_initial_moments(const orc_params *par, double *mu, double *Sigma);

/* Draw N behavioural samples for upper iteration l (0-based).
 * structured != 0: the initial sampler; else p = mu + Lchol z. */
void orc_sample(const orc_params *par, uint64_t seed, int l, int N,
                int structured, const double *mu, const double *Lchol,
                double *p);

typedef struct orc_plan_out {
  int best_index;
  double p_best[ORC_NP];
  double xi_best[ORC_NX];
  double cost_upper, residual;
  double mu[ORC_NP];
  double Sigma[ORC_NP * ORC_NP];
} orc_plan_out;

/* Per-iteration record, all arrays sized for par->L iterations, nullable. */
typedef struct orc_plan_trace {
  double *p;       /* L x N x 8   */
  double *xi_bar;  /* L x N x 22  */
  double *xi_star; /* L x N x 22  */
  double *r;       /* L x N       */
  double *cu;      /* L x N       */
  int *ces;        /* L x n       */
  int *es;         /* L x q       */
  double *c_es;    /* L x q       */
  double *mu;      /* L x 8 (after the update of iteration l) */
  double *Sigma;   /* L x 64      */
} orc_plan_trace;

/* Alg. 1. mu0/Sigma0 NULL: iteration 0 draws from the structured sampler
 * and the update starts from its moments. */
int orc_plan(const orc_params *par, const orc_scene *sc, uint64_t seed, int N,
             const double *mu0, const double *Sigma0, orc_plan_out *out,
             orc_plan_trace *trace);

/* Alg. 1 whose first iteration evaluates the given samples p0 (N x 8, the
 * decoder sampler's output, App. A) and whose prior before the first update
 * is their sample moments (orc_sample_moments). */
int orc_plan_p0(const orc_params *par, const orc_scene *sc, uint64_t seed, int N,
                const double *p0, orc_plan_out *out, orc_plan_trace *trace);

/* Latent draws z (N x 2) of the decoder sampler: Box-Muller of words 0, 1 of
 * Philox block (sample j, iteration 0, block 0). */
void orc_decoder_latent(uint64_t seed, int N, double *z);

/* Sample mean and covariance (normalised by N) of p (N x 8). */
void orc_sample_moments(const double *p, int N, double *mu, double *Sigma);

/* Threads used by the OpenMP loops over samples (1 = serial). */
/* One step of the receding-horizon loop (MPC-Bi-Level, Sec. V-A): state of
 * xi at t_{n_exec} (x, y, xdot, ydot, xddot, yddot), the neighbours (M x 4,
 * first-cycle states obs0) at the start of cycle + 1, and whether an
 * executed instant of cycle `cycle` meets a neighbour's ellipse. */
int orc_advance(const orc_params *par, const double *xi, const double *obs0, int M, int cycle, int n_exec,
                double *ego_next, double *obs_next, int *collided);

void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
