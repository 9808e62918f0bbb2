/*
 * oracle.c -- plain FP64 CPU oracle of the bi-level planner hot path of
 * arXiv 2212.02224: Alg. 1 (upper level) around the two-step lower level
 * (Step 1: equality-constrained QP, eq. over_2; Step 2: projection by the
 * alternating minimisation of Alg. 2, App. "GPU Accelerated Batch
 * Projection").
 *
 * TEST INFRASTRUCTURE. This file exists to check the HIP path. Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares nothing with the HIP path.
 *
 * Style: slow and literal. Matrices of the paper (Q, A_eq, F, G, h, e, s,
 * lambda) are built explicitly; linear systems are solved with a textbook
 * LU factorisation with partial pivoting; the polar variables (alpha, d) are
 * obtained with atan2/hypot and turned back with cos/sin, as the paper writes
 * them. Points the paper leaves open follow the readings listed with the
 * build's design notes; each is marked "reading" below.
 *
 * Parity status: every function is pinned by CPU tests (closed forms,
 * invariants, brute force, known-answer vectors). In orc_project every
 * xi-update is pinned (its KKT system at each iteration, the first one by an
 * independent least-squares solve), the target pass by brute force, and the
 * multiplier step by the fixed point it must reach. The length of the
 * multiplier step (the printed rho/2 of eq. update_lagrange) is the one
 * factor no property fixes: any positive length has the same fixed points,
 * so the iterate values at finite K are "parity unpinned" in that factor.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NC ORC_NC
#define NX ORC_NX
#define NP ORC_NP
#define NEQ_MAX ORC_NEQ_MAX
#define NKKT_MAX (NX + NEQ_MAX)
#define DEG 10 /* polynomial order, Sec. V-A */
#define NSEG 4 /* set-points per axis, Sec. V-A */

static const double ORC_PI = 3.14159265358979323846;

static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return g_threads; }

void orc_default_params(orc_params *par) {
  memset(par, 0, sizeof(*par));
  par->T = 100;
  par->M = 10;
  par->K = 20;
  par->L = 5;
  par->t_f = 5.0;
  par->k_p = 1.0; /* reading: stable PD form, critically damped */
  par->k_v = 2.0;
  par->w_s = 1.0;
  par->w_l = 1.0;
  par->w_v = 1.0;
  par->rho = 1.0;
  par->ell_a = 4.5; /* reading: a, b are the denominators of Table ineq_list */
  par->ell_b = 2.0;
  par->v_min = 0.0;
  par->v_max = 30.0;
  par->a_max = 8.0;
  par->kappa_max = 0.2;
  par->c_max = 4.0;
  par->y_lb = -7.0;
  par->y_ub = 7.0;
  par->v_eps = 0.1;
  par->eta = 0.6;
  par->gamma = 0.9; /* Sec. V-A */
  par->cov_jitter = 1e-6;
  par->frac_ces = 0.15; /* 150 of 1000, Sec. V-A */
  par->frac_es = 0.05;  /* 50 of 1000, Sec. V-A */
  par->lane_c[0] = -3.5;
  par->lane_c[1] = 0.0;
  par->lane_c[2] = 3.5;
  par->lane_sigma = 0.3;
  par->vd_lo = 5.0;
  par->vd_hi = 25.0;
  par->behaviour = 0;
  par->sampler = 0;
}

/* Road at longitudinal position x: curvature and lane limits (see
 * orc_scene), linear interpolation between knots, constant beyond. */
static void road_at(const orc_params *par, const orc_scene *sc, double x, double *kappa,
                    double *y_lb, double *y_ub) {
  if (sc->n_road <= 0) {
    *kappa = sc->kappa_road;
    *y_lb = par->y_lb;
    *y_ub = par->y_ub;
    return;
  }
  const double *R = sc->road;
  if (sc->n_road == 1) {
    *kappa = R[0];
    *y_lb = R[1];
    *y_ub = R[2];
    return;
  }
  double u = (x - sc->road_x0) / sc->road_dx;
  int last = sc->n_road - 1;
  if (u <= 0.0) u = 0.0;
  if (u >= (double)last) u = (double)last;
  int i = (int)floor(u);
  if (i > last - 1) i = last - 1;
  double f = u - (double)i;
  *kappa = R[3 * i + 0] + f * (R[3 * (i + 1) + 0] - R[3 * i + 0]);
  *y_lb = R[3 * i + 1] + f * (R[3 * (i + 1) + 1] - R[3 * i + 1]);
  *y_ub = R[3 * i + 2] + f * (R[3 * (i + 1) + 2] - R[3 * i + 2]);
}

/* Equality rows: the 7 of the set-point reading, plus x(t_f) and y(t_f)
 * with goal positions. */
static int neq_of(const orc_params *par) { return par->behaviour ? 9 : 7; }

static int round_half_up(double v) { return (int)floor(v + 0.5); }

void orc_elite_sizes(const orc_params *par, int N, int *n_ces, int *n_es) {
  int q = round_half_up(par->frac_es * N);
  if (q < 1) q = 1;
  int n = round_half_up(par->frac_ces * N);
  if (n < q) n = q;
  if (n > N) n = N;
  if (q > n) q = n;
  *n_ces = n;
  *n_es = q;
}

/* ------------------------------------------------------------------ */
/* Basis of eq. param: Bernstein polynomials of order 10 on tau = t/t_f. */
/* (reading: the paper only says "10th order polynomial")              */

static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return r;
}

/* x^e with the convention that a term whose exponent is negative has a
 * zero multiplier everywhere it is used, and 0^0 = 1. */
static double ipow(double x, int e) {
  if (e < 0) return 0.0;
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

void orc_basis(int T, double t_f, double *W, double *Wd, double *Wdd) {
  const int n = DEG;
  for (int k = 0; k < T; ++k) {
    double tau = (T > 1) ? (double)k / (double)(T - 1) : 0.0;
    double u = 1.0 - tau;
    for (int i = 0; i <= n; ++i) {
      double C = binom(n, i);
      /* B_i = C tau^i u^(n-i) */
      double B = C * ipow(tau, i) * ipow(u, n - i);
      /* dB/dtau by the product rule */
      double dB = C * ((double)i * ipow(tau, i - 1) * ipow(u, n - i) -
                       (double)(n - i) * ipow(tau, i) * ipow(u, n - i - 1));
      /* d2B/dtau2 by the product rule applied twice */
      double d2B =
          C * ((double)i * (double)(i - 1) * ipow(tau, i - 2) * ipow(u, n - i) -
               2.0 * (double)i * (double)(n - i) * ipow(tau, i - 1) *
                   ipow(u, n - i - 1) +
               (double)(n - i) * (double)(n - i - 1) * ipow(tau, i) *
                   ipow(u, n - i - 2));
      W[k * NC + i] = B;
      Wd[k * NC + i] = dB / t_f;
      Wdd[k * NC + i] = d2B / (t_f * t_f);
    }
  }
}

/* ------------------------------------------------------------------ */
/* Dense linear algebra: LU with partial pivoting (Golub & Van Loan,
 * Alg. 3.4.1), solve, Cholesky.                                        */

static int lu_factor(int n, double *A, int *piv) {
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = fabs(A[i * n + k]);
      if (v > best) {
        best = v;
        pr = i;
      }
    }
    piv[k] = pr;
    if (best == 0.0) return -1;
    if (pr != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j];
        A[k * n + j] = A[pr * n + j];
        A[pr * n + j] = t;
      }
    }
    for (int i = k + 1; i < n; ++i) {
      double l = A[i * n + k] / A[k * n + k];
      A[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}

static void lu_solve(int n, const double *LU, const int *piv, double *b) {
  for (int k = 0; k < n; ++k) {
    if (piv[k] != k) {
      double t = b[k];
      b[k] = b[piv[k]];
      b[piv[k]] = t;
    }
  }
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= LU[i * n + j] * b[j];
    b[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= LU[i * n + j] * b[j];
    b[i] = s / LU[i * n + i];
  }
}

int orc_cholesky(const double *A, int n, double jitter, double *Lo) {
  memset(Lo, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j] + jitter;
    for (int k = 0; k < j; ++k) d -= Lo[j * n + k] * Lo[j * n + k];
    if (!(d > 0.0)) return -1;
    double ljj = sqrt(d);
    Lo[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= Lo[i * n + k] * Lo[j * n + k];
      Lo[i * n + j] = s / ljj;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Shared problem data for one (params, scene).                          */

typedef struct basis_t {
  int T;
  double *W, *Wd, *Wdd; /* T x 11 */
  double *t;            /* T     */
} basis_t;

static void basis_init(basis_t *B, const orc_params *par) {
  int T = par->T;
  B->T = T;
  B->W = (double *)malloc(sizeof(double) * T * NC);
  B->Wd = (double *)malloc(sizeof(double) * T * NC);
  B->Wdd = (double *)malloc(sizeof(double) * T * NC);
  B->t = (double *)malloc(sizeof(double) * T);
  orc_basis(T, par->t_f, B->W, B->Wd, B->Wdd);
  for (int k = 0; k < T; ++k)
    B->t[k] = (T > 1) ? par->t_f * (double)k / (double)(T - 1) : 0.0;
}

static void basis_free(basis_t *B) {
  free(B->W);
  free(B->Wd);
  free(B->Wdd);
  free(B->t);
}

/* Equality constraints A_eq xi = b (eqs. boundary_cond_initial and
 * final_boundary): x(0), xdot(0), xddot(0), y(0), ydot(0), yddot(0),
 * ydot(t_f) = 0, and with goal positions (behaviour 1) x(t_f) = x_f,
 * y(t_f) = y_f. (reading: the set-point experiments of Sec. V-A have no goal
 * positions, so there only the final lateral velocity is constrained.) */
static int build_Aeq(const basis_t *B, const orc_params *par, double *A) {
  int T = B->T, neq = neq_of(par);
  memset(A, 0, sizeof(double) * NEQ_MAX * NX);
  for (int i = 0; i < NC; ++i) {
    A[0 * NX + i] = B->W[0 * NC + i];
    A[1 * NX + i] = B->Wd[0 * NC + i];
    A[2 * NX + i] = B->Wdd[0 * NC + i];
    A[3 * NX + NC + i] = B->W[0 * NC + i];
    A[4 * NX + NC + i] = B->Wd[0 * NC + i];
    A[5 * NX + NC + i] = B->Wdd[0 * NC + i];
    A[6 * NX + NC + i] = B->Wd[(T - 1) * NC + i];
    if (neq == 9) {
      A[7 * NX + i] = B->W[(T - 1) * NC + i];
      A[8 * NX + NC + i] = B->W[(T - 1) * NC + i];
    }
  }
  return neq;
}

/* Right-hand side b of A_eq xi = b: the ego state b_0 and the final values;
 * with goals x_f = x0 + p[0] (measured from the ego, as all positions the
 * planner sees, Sec. V-A) and y_f = p[1]. */
static void eq_rhs(const orc_params *par, const orc_scene *sc, const double *p,
                   double *b) {
  b[0] = sc->ego[0];
  b[1] = sc->ego[2];
  b[2] = sc->ego[4];
  b[3] = sc->ego[1];
  b[4] = sc->ego[3];
  b[5] = sc->ego[5];
  b[6] = 0.0;
  if (par->behaviour) {
    b[7] = sc->ego[0] + p[0];
    b[8] = p[1];
  }
}

/* Segment of time index k: the horizon is cut into 4 equal parts and
 * each set-point repeated over its part (Sec. II-C; reading for T not a
 * multiple of 4: floor(4k/T)). */
static int segment_of(int k, int T) { return (NSEG * k) / T; }

/* ------------------------------------------------------------------ */
/* Lower-level cost, eq. cost with c_s, c_l, c_v of Sec. II-C.
 * (reading: c_l = (yddot + k_p (y - y_d) + k_v ydot)^2 and
 *  c_v = (xddot + k_p (xdot - v_d))^2, the stable PD / P forms.)       */

typedef struct cost_row {
  double a[NX];
  double beta;
  double w;
} cost_row;

/* Fill the 4T rows of the quadratic cost sum_rows w (a^T xi - beta)^2. */
static void cost_rows(const orc_params *par, const basis_t *B, const double *p,
                      cost_row *rows) {
  int T = B->T;
  for (int k = 0; k < T; ++k) {
    const double *W = B->W + k * NC, *Wd = B->Wd + k * NC,
                 *Wdd = B->Wdd + k * NC;
    int sg = segment_of(k, T);
    /* with goal positions p holds no set-points: c_l and c_v drop out */
    int setpoints = !par->behaviour;
    double y_d = setpoints ? p[sg] : 0.0;
    double v_d = setpoints ? p[NSEG + sg] : 0.0;
    cost_row *r;
    /* c_s, x part: xddot^2 */
    r = &rows[4 * k + 0];
    memset(r->a, 0, sizeof(r->a));
    for (int i = 0; i < NC; ++i) r->a[i] = Wdd[i];
    r->beta = 0.0;
    r->w = par->w_s;
    /* c_s, y part: yddot^2 */
    r = &rows[4 * k + 1];
    memset(r->a, 0, sizeof(r->a));
    for (int i = 0; i < NC; ++i) r->a[NC + i] = Wdd[i];
    r->beta = 0.0;
    r->w = par->w_s;
    /* c_l: (yddot + k_p (y - y_d) + k_v ydot)^2 */
    r = &rows[4 * k + 2];
    memset(r->a, 0, sizeof(r->a));
    for (int i = 0; i < NC; ++i)
      r->a[NC + i] = Wdd[i] + par->k_p * W[i] + par->k_v * Wd[i];
    r->beta = par->k_p * y_d;
    r->w = setpoints ? par->w_l : 0.0;
    /* c_v: (xddot + k_p (xdot - v_d))^2 */
    r = &rows[4 * k + 3];
    memset(r->a, 0, sizeof(r->a));
    for (int i = 0; i < NC; ++i) r->a[i] = Wdd[i] + par->k_p * Wd[i];
    r->beta = par->k_p * v_d;
    r->w = setpoints ? par->w_v : 0.0;
  }
}

double orc_lower_cost(const orc_params *par, const double *p, const double *xi) {
  basis_t B;
  basis_init(&B, par);
  cost_row *rows = (cost_row *)malloc(sizeof(cost_row) * 4 * B.T);
  cost_rows(par, &B, p, rows);
  double J = 0.0;
  for (int r = 0; r < 4 * B.T; ++r) {
    double v = -rows[r].beta;
    for (int i = 0; i < NX; ++i) v += rows[r].a[i] * xi[i];
    J += rows[r].w * v * v;
  }
  free(rows);
  basis_free(&B);
  return J;
}

/* ------------------------------------------------------------------ */
/* Step 1 of Alg. 1: min 1/2 xi^T Q xi + q(p)^T xi s.t. A_eq xi = b,
 * solved through the KKT system of eq. over_2. With J = sum w (a^T xi -
 * beta)^2: Q = sum 2 w a a^T, q = -sum 2 w beta a; the KKT right-hand
 * side is (-q, b) (reading of the sign printed in eq. over_2).          */

int orc_step1(const orc_params *par, const orc_scene *sc, const double *p,
              int N, double *xi_bar) {
  basis_t B;
  basis_init(&B, par);
  int T = B.T;
  double Aeq[NEQ_MAX * NX];
  int neq = build_Aeq(&B, par, Aeq);
  int nk = NX + neq;
  double *K = (double *)calloc((size_t)nk * nk, sizeof(double));
  int *piv = (int *)malloc(sizeof(int) * nk);

  /* Q does not depend on p: build it with any p. */
  double pz[NP] = {0};
  cost_row *rows = (cost_row *)malloc(sizeof(cost_row) * 4 * T);
  cost_rows(par, &B, pz, rows);
  for (int r = 0; r < 4 * T; ++r)
    for (int i = 0; i < NX; ++i)
      for (int j = 0; j < NX; ++j)
        K[i * nk + j] += 2.0 * rows[r].w * rows[r].a[i] * rows[r].a[j];
  for (int e = 0; e < neq; ++e)
    for (int i = 0; i < NX; ++i) {
      K[(NX + e) * nk + i] = Aeq[e * NX + i];
      K[i * nk + NX + e] = Aeq[e * NX + i];
    }
  free(rows);
  int rc = lu_factor(nk, K, piv);
  if (rc != 0) {
    free(K);
    free(piv);
    basis_free(&B);
    return rc;
  }

  int nthreads = g_threads;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int j = 0; j < N; ++j) {
    const double *pj = p + (size_t)j * NP;
    cost_row *rw = (cost_row *)malloc(sizeof(cost_row) * 4 * T);
    cost_rows(par, &B, pj, rw);
    double rhs[NKKT_MAX], beq[NEQ_MAX];
    memset(rhs, 0, sizeof(rhs));
    for (int r = 0; r < 4 * T; ++r)
      for (int i = 0; i < NX; ++i)
        rhs[i] += 2.0 * rw[r].w * rw[r].beta * rw[r].a[i]; /* -q */
    eq_rhs(par, sc, pj, beq);
    for (int e = 0; e < neq; ++e) rhs[NX + e] = beq[e];
    lu_solve(nk, K, piv, rhs);
    memcpy(xi_bar + (size_t)j * NX, rhs, sizeof(double) * NX);
    free(rw);
  }
  free(K);
  free(piv);
  basis_free(&B);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Projection (App. "GPU Accelerated Batch Projection").                 */

typedef struct proj_t {
  const orc_params *par;
  const orc_scene *sc;
  basis_t B;
  int T, M, nF; /* nF = 2 (M+2) T rows of F */
  double *F;    /* nF x 22, eq. for F: blkdiag([F_o; Wd; Wdd]) */
  double *G;    /* 2T x 22, lane rows G xi <= e (eq. lane_reform) */
  double *xo, *yo; /* M x T neighbour trajectories */
  double *KP;   /* LU of [[I + rho F^T F + rho G^T G, A^T], [A, 0]] */
  int *piv;
  int neq, nk;  /* equality rows, KKT size NX + neq */
} proj_t;

static void proj_init(proj_t *P, const orc_params *par, const orc_scene *sc) {
  P->par = par;
  P->sc = sc;
  basis_init(&P->B, par);
  int T = par->T, M = par->M;
  P->T = T;
  P->M = M;
  P->nF = 2 * (M + 2) * T;
  int rows_axis = (M + 2) * T;
  P->F = (double *)calloc((size_t)P->nF * NX, sizeof(double));
  /* F_o stacks W once per neighbour, then Wd, then Wdd; the y block
   * repeats the structure on c_y. */
  for (int ax = 0; ax < 2; ++ax) {
    int r0 = ax * rows_axis, c0 = ax * NC;
    for (int i = 0; i < M; ++i)
      for (int k = 0; k < T; ++k)
        for (int c = 0; c < NC; ++c)
          P->F[(size_t)(r0 + i * T + k) * NX + c0 + c] = P->B.W[k * NC + c];
    for (int k = 0; k < T; ++k)
      for (int c = 0; c < NC; ++c) {
        P->F[(size_t)(r0 + M * T + k) * NX + c0 + c] = P->B.Wd[k * NC + c];
        P->F[(size_t)(r0 + (M + 1) * T + k) * NX + c0 + c] =
            P->B.Wdd[k * NC + c];
      }
  }
  /* Lane bounds y_lb(x) <= y <= y_ub(x) as G xi <= e with G = [W; -W] on
   * c_y; e = [y_ub; -y_lb] at each instant, taken at x(t_k) of the iterate
   * of the target pass (constant on a road without a profile). */
  P->G = (double *)calloc((size_t)2 * T * NX, sizeof(double));
  for (int k = 0; k < T; ++k) {
    for (int c = 0; c < NC; ++c) {
      P->G[(size_t)k * NX + NC + c] = P->B.W[k * NC + c];
      P->G[(size_t)(T + k) * NX + NC + c] = -P->B.W[k * NC + c];
    }
  }
  /* Neighbour trajectories x_o,i(t), y_o,i(t): constant velocity. */
  P->xo = (double *)malloc(sizeof(double) * (M > 0 ? M : 1) * T);
  P->yo = (double *)malloc(sizeof(double) * (M > 0 ? M : 1) * T);
  for (int i = 0; i < M; ++i)
    for (int k = 0; k < T; ++k) {
      const double *o = sc->obs + 4 * i;
      P->xo[i * T + k] = o[0] + o[2] * P->B.t[k];
      P->yo[i * T + k] = o[1] + o[3] * P->B.t[k];
    }
  /* KKT matrix of eq. split_xy: stationarity of eq. aug_lag in xi gives
   * (I + rho F^T F + rho G^T G) xi + A^T nu = xi_bar + lambda + rho F^T h
   * + rho G^T (e - s). */
  double Aeq[NEQ_MAX * NX];
  P->neq = build_Aeq(&P->B, par, Aeq);
  int nk = P->nk = NX + P->neq;
  P->KP = (double *)calloc((size_t)nk * nk, sizeof(double));
  for (int i = 0; i < NX; ++i) P->KP[i * nk + i] = 1.0;
  for (int r = 0; r < P->nF; ++r)
    for (int i = 0; i < NX; ++i) {
      double fi = P->F[(size_t)r * NX + i];
      if (fi == 0.0) continue;
      for (int j = 0; j < NX; ++j)
        P->KP[i * nk + j] += par->rho * fi * P->F[(size_t)r * NX + j];
    }
  for (int r = 0; r < 2 * T; ++r)
    for (int i = 0; i < NX; ++i) {
      double gi = P->G[(size_t)r * NX + i];
      if (gi == 0.0) continue;
      for (int j = 0; j < NX; ++j)
        P->KP[i * nk + j] += par->rho * gi * P->G[(size_t)r * NX + j];
    }
  for (int e2 = 0; e2 < P->neq; ++e2)
    for (int i = 0; i < NX; ++i) {
      P->KP[(NX + e2) * nk + i] = Aeq[e2 * NX + i];
      P->KP[i * nk + NX + e2] = Aeq[e2 * NX + i];
    }
  P->piv = (int *)malloc(sizeof(int) * nk);
  lu_factor(nk, P->KP, P->piv);
}

static void proj_free(proj_t *P) {
  free(P->F);
  free(P->G);
  free(P->xo);
  free(P->yo);
  free(P->KP);
  free(P->piv);
  basis_free(&P->B);
}

static double clip(double v, double lo, double hi) {
  /* reading: with lo > hi the upper bound wins */
  double r = v < lo ? lo : v;
  return r > hi ? hi : r;
}

/* Target pass: given xi, compute (alpha, d) in closed form, clip d
 * (steps split_alpha_o, clip_d_o, clip_d_v, clip_d_a), assemble h of
 * eq. for h_j, and the lane slack of step update_slack.
 *   - obstacles: alpha_o = atan2(dy/b, dx/a), d_o = max(1, hypot(dx/a,
 *     dy/b)); h_o = (x_o + a d_o cos alpha_o, y_o + b d_o sin alpha_o)
 *     (reading: the ellipse axes scale the polar form on both rows).
 *   - velocity / acceleration: alpha = atan2 of the vector, d = its norm
 *     clipped to the bounds of clip_d_v / clip_d_a; the curvature bound
 *     d_a |sin(alpha_a - alpha_v)| / d_v^2 <= kappa_max gives
 *     vbar_min = max(v_min, sqrt(d_a_prev |sin| / kappa_max)) and
 *     abar_max = min(a_max, d_v^2 kappa_max / |sin|) (a_max if sin = 0);
 *     the centripetal bound gives vbar_max = min(v_max, sqrt(c_max /
 *     (|kappa| cos^2 alpha_v))) (v_max where the denominator is 0).
 *   - slack: s = max(0, e - G xi) from G xi - e + s = 0, s >= 0. */
static void targets(const proj_t *P, const double *xi, const double *da_prev,
                    double *h, double *s, double *e, double *da_out) {
  const orc_params *par = P->par;
  int T = P->T, M = P->M;
  int rows_axis = (M + 2) * T;
  const double *cx = xi, *cy = xi + NC;
  for (int k = 0; k < T; ++k) {
    const double *W = P->B.W + k * NC, *Wd = P->B.Wd + k * NC,
                 *Wdd = P->B.Wdd + k * NC;
    double x = 0, y = 0, xd = 0, yd = 0, xdd = 0, ydd = 0;
    for (int c = 0; c < NC; ++c) {
      x += W[c] * cx[c];
      y += W[c] * cy[c];
      xd += Wd[c] * cx[c];
      yd += Wd[c] * cy[c];
      xdd += Wdd[c] * cx[c];
      ydd += Wdd[c] * cy[c];
    }
    for (int i = 0; i < M; ++i) {
      double dx = x - P->xo[i * T + k];
      double dy = y - P->yo[i * T + k];
      double alpha = atan2(dy / par->ell_b, dx / par->ell_a);
      double d = hypot(dx / par->ell_a, dy / par->ell_b);
      d = d < 1.0 ? 1.0 : d; /* clip(1, inf) */
      h[i * T + k] = P->xo[i * T + k] + par->ell_a * d * cos(alpha);
      h[rows_axis + i * T + k] = P->yo[i * T + k] + par->ell_b * d * sin(alpha);
    }
    double alpha_v = atan2(yd, xd);
    double alpha_a = atan2(ydd, xdd);
    double sabs = fabs(sin(alpha_a - alpha_v));
    double vbar_min = par->v_min;
    double vcurv = sqrt(da_prev[k] * sabs / par->kappa_max);
    if (vcurv > vbar_min) vbar_min = vcurv;
    double kappa, y_lb, y_ub;
    road_at(par, P->sc, x, &kappa, &y_lb, &y_ub);
    e[k] = y_ub; /* lane rows G xi <= e at this iterate's x(t_k) */
    e[T + k] = -y_lb;
    double cva = cos(alpha_v);
    double den = fabs(kappa) * cva * cva;
    double vbar_max = par->v_max;
    if (den > 0.0) {
      double vc = sqrt(par->c_max / den);
      if (vc < vbar_max) vbar_max = vc;
    }
    double d_v = clip(hypot(xd, yd), vbar_min, vbar_max);
    double abar_max = par->a_max;
    if (sabs > 0.0) {
      double ac = d_v * d_v * par->kappa_max / sabs;
      if (ac < abar_max) abar_max = ac;
    }
    double d_a = clip(hypot(xdd, ydd), 0.0, abar_max);
    da_out[k] = d_a;
    h[M * T + k] = d_v * cos(alpha_v);
    h[rows_axis + M * T + k] = d_v * sin(alpha_v);
    h[(M + 1) * T + k] = d_a * cos(alpha_a);
    h[rows_axis + (M + 1) * T + k] = d_a * sin(alpha_a);
  }
  for (int r = 0; r < 2 * T; ++r) {
    double g = 0;
    for (int c = 0; c < NX; ++c) g += P->G[(size_t)r * NX + c] * xi[c];
    double v = e[r] - g;
    s[r] = v > 0.0 ? v : 0.0;
  }
}

void orc_targets(const orc_params *par, const orc_scene *sc, const double *xi,
                 const double *da_prev, double *h, double *s, double *da_out) {
  proj_t P;
  proj_init(&P, par, sc);
  double *e = (double *)malloc(sizeof(double) * 2 * par->T);
  targets(&P, xi, da_prev, h, s, e, da_out);
  free(e);
  proj_free(&P);
}

static void acc_norm_clip(const proj_t *P, const double *xi, double *da) {
  const double *cx = xi, *cy = xi + NC;
  for (int k = 0; k < P->T; ++k) {
    const double *Wdd = P->B.Wdd + k * NC;
    double xdd = 0, ydd = 0;
    for (int c = 0; c < NC; ++c) {
      xdd += Wdd[c] * cx[c];
      ydd += Wdd[c] * cy[c];
    }
    da[k] = clip(hypot(xdd, ydd), 0.0, P->par->a_max);
  }
}

/* Alg. 2 for one sample (reading of the unprinted initialisation: xi^0 =
 * xi_bar, lambda^0 = 0, targets from xi_bar with d_a^{-1} = clip(|a|, 0,
 * a_max); the returned iterate is the last xi-update). */
/* Every intermediate of Alg. 2 for one sample, iterations k = 0..K (each
 * array nullable): the iterate xi^k (xi^0 = xi_bar), the target pass taken
 * at it (h^k, s^k, the lane bound e^k, d_a^k) and the multiplier lambda^k
 * after the step update_lagrange of iteration k (lambda^0 = 0). */
typedef struct proj_dump {
  double *xi, *h, *s, *e, *da, *lam;
} proj_dump;

static void dump_step(const proj_t *P, const proj_dump *D, int k, const double *xi,
                      const double *h, const double *s, const double *e,
                      const double *da, const double *lam) {
  if (!D) return;
  int T = P->T, nF = P->nF;
  if (D->xi) memcpy(D->xi + (size_t)k * NX, xi, sizeof(double) * NX);
  if (D->h) memcpy(D->h + (size_t)k * nF, h, sizeof(double) * nF);
  if (D->s) memcpy(D->s + (size_t)k * 2 * T, s, sizeof(double) * 2 * T);
  if (D->e) memcpy(D->e + (size_t)k * 2 * T, e, sizeof(double) * 2 * T);
  if (D->da) memcpy(D->da + (size_t)k * T, da, sizeof(double) * T);
  if (D->lam) memcpy(D->lam + (size_t)k * NX, lam, sizeof(double) * NX);
}

static void project_one(const proj_t *P, const double *xi_bar, const double *p,
                        double *xi_out, double *xi_iter, const proj_dump *dump) {
  const orc_params *par = P->par;
  int T = P->T, nF = P->nF, K = par->K;
  double rho = par->rho;
  double *h = (double *)malloc(sizeof(double) * nF);
  double *s = (double *)malloc(sizeof(double) * 2 * T);
  double *da = (double *)malloc(sizeof(double) * T);
  double *da_prev = (double *)malloc(sizeof(double) * T);
  double *Fx = (double *)malloc(sizeof(double) * nF);
  double *e = (double *)malloc(sizeof(double) * 2 * T);
  double xi[NX], lam[NX], rhs[NKKT_MAX], beq[NEQ_MAX];
  eq_rhs(par, P->sc, p, beq);

  memcpy(xi, xi_bar, sizeof(xi));
  memset(lam, 0, sizeof(lam));
  acc_norm_clip(P, xi, da_prev);
  targets(P, xi, da_prev, h, s, e, da);
  memcpy(da_prev, da, sizeof(double) * T);
  if (xi_iter) memcpy(xi_iter, xi, sizeof(xi));
  dump_step(P, dump, 0, xi, h, s, e, da, lam);

  for (int k = 1; k <= K; ++k) {
    /* eq. split_xy */
    for (int i = 0; i < NX; ++i) rhs[i] = xi_bar[i] + lam[i];
    for (int r = 0; r < nF; ++r) {
      double hr = rho * h[r];
      const double *Fr = P->F + (size_t)r * NX;
      for (int i = 0; i < NX; ++i) rhs[i] += Fr[i] * hr;
    }
    for (int r = 0; r < 2 * T; ++r) {
      double er = rho * (e[r] - s[r]);
      const double *Gr = P->G + (size_t)r * NX;
      for (int i = 0; i < NX; ++i) rhs[i] += Gr[i] * er;
    }
    for (int e2 = 0; e2 < P->neq; ++e2) rhs[NX + e2] = beq[e2];
    lu_solve(P->nk, P->KP, P->piv, rhs);
    memcpy(xi, rhs, sizeof(xi));
    if (xi_iter) memcpy(xi_iter + (size_t)k * NX, xi, sizeof(xi));

    /* steps split_alpha_o .. update_slack */
    targets(P, xi, da_prev, h, s, e, da);
    memcpy(da_prev, da, sizeof(double) * T);

    /* step update_lagrange (reading: the two penalty gradients are both
     * subtracted with the printed factor rho/2) */
    for (int r = 0; r < nF; ++r) {
      double v = 0;
      const double *Fr = P->F + (size_t)r * NX;
      for (int i = 0; i < NX; ++i) v += Fr[i] * xi[i];
      Fx[r] = v - h[r];
    }
    for (int r = 0; r < nF; ++r) {
      const double *Fr = P->F + (size_t)r * NX;
      for (int i = 0; i < NX; ++i) lam[i] -= 0.5 * rho * Fr[i] * Fx[r];
    }
    for (int r = 0; r < 2 * T; ++r) {
      const double *Gr = P->G + (size_t)r * NX;
      double v = 0;
      for (int i = 0; i < NX; ++i) v += Gr[i] * xi[i];
      v = v - e[r] + s[r];
      for (int i = 0; i < NX; ++i) lam[i] -= 0.5 * rho * Gr[i] * v;
    }
    dump_step(P, dump, k, xi, h, s, e, da, lam);
  }
  memcpy(xi_out, xi, sizeof(xi));
  free(e);
  free(h);
  free(s);
  free(da);
  free(da_prev);
  free(Fx);
}

int orc_project(const orc_params *par, const orc_scene *sc,
                const double *xi_bar, const double *p, int N, double *xi_star,
                double *xi_iter) {
  if (par->behaviour && p == NULL) return -1;
  proj_t P;
  proj_init(&P, par, sc);
  int nthreads = g_threads;
  size_t stride_it = (size_t)(par->K + 1) * NX;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int j = 0; j < N; ++j)
    project_one(&P, xi_bar + (size_t)j * NX, p ? p + (size_t)j * NP : NULL,
                xi_star + (size_t)j * NX,
                xi_iter ? xi_iter + (size_t)j * stride_it : NULL, NULL);
  proj_free(&P);
  return 0;
}

int orc_project_dump(const orc_params *par, const orc_scene *sc,
                     const double *xi_bar, const double *p, double *xi,
                     double *h, double *s, double *e, double *da, double *lam) {
  if (par->behaviour && p == NULL) return -1;
  proj_t P;
  proj_init(&P, par, sc);
  proj_dump D = {xi, h, s, e, da, lam};
  double xs[NX];
  project_one(&P, xi_bar, p, xs, NULL, &D);
  proj_free(&P);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Constraint residual r = sum max(0, g) over Table ineq_list and the
 * upper-level driving cost c_u = sum_t (|v| - v_max)^2 (Sec. V-A, task
 * "drive as fast as possible"; reading: summed over the T instants).
 * The curvature row uses max(|v|, v_eps)^3 in its denominator.          */

void orc_residual_cost(const orc_params *par, const orc_scene *sc,
                       const double *xi, int N, double *r, double *cu) {
  basis_t B;
  basis_init(&B, par);
  int T = B.T, M = par->M;
  int nthreads = g_threads;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int j = 0; j < N; ++j) {
    const double *cx = xi + (size_t)j * NX, *cy = cx + NC;
    double res = 0.0, cost = 0.0;
    for (int k = 0; k < T; ++k) {
      const double *W = B.W + k * NC, *Wd = B.Wd + k * NC,
                   *Wdd = B.Wdd + k * NC;
      double x = 0, y = 0, xd = 0, yd = 0, xdd = 0, ydd = 0;
      for (int c = 0; c < NC; ++c) {
        x += W[c] * cx[c];
        y += W[c] * cy[c];
        xd += Wd[c] * cx[c];
        yd += Wd[c] * cy[c];
        xdd += Wdd[c] * cx[c];
        ydd += Wdd[c] * cy[c];
      }
      for (int i = 0; i < M; ++i) {
        const double *o = sc->obs + 4 * i;
        double xo = o[0] + o[2] * B.t[k], yo = o[1] + o[3] * B.t[k];
        double g = -((x - xo) * (x - xo)) / (par->ell_a * par->ell_a) -
                   ((y - yo) * (y - yo)) / (par->ell_b * par->ell_b) + 1.0;
        res += g > 0 ? g : 0;
      }
      double v = sqrt(xd * xd + yd * yd);
      double a = sqrt(xdd * xdd + ydd * ydd);
      double g;
      g = v - par->v_max;
      res += g > 0 ? g : 0;
      g = par->v_min - v;
      res += g > 0 ? g : 0;
      g = a - par->a_max;
      res += g > 0 ? g : 0;
      double vd = v > par->v_eps ? v : par->v_eps;
      g = fabs(ydd * xd - xdd * yd) / (vd * vd * vd) - par->kappa_max;
      res += g > 0 ? g : 0;
      double kappa, y_lb, y_ub;
      road_at(par, sc, x, &kappa, &y_lb, &y_ub);
      g = fabs(xd * xd * kappa) - par->c_max;
      res += g > 0 ? g : 0;
      g = y - y_ub;
      res += g > 0 ? g : 0;
      g = y_lb - y;
      res += g > 0 ? g : 0;
      cost += (v - par->v_max) * (v - par->v_max);
    }
    r[j] = res;
    cu[j] = cost;
  }
  basis_free(&B);
}

/* ------------------------------------------------------------------ */
/* Elite selection of Alg. 1: the n samples of lowest residual form the
 * ConstraintEliteSet; on them the cost c_u + r is formed and the q lowest
 * form the EliteSet. (reading: ties broken by the lower sample index.)  */

typedef struct keyidx {
  double key;
  int idx;
} keyidx;

static int cmp_keyidx(const void *a, const void *b) {
  const keyidx *x = (const keyidx *)a, *y = (const keyidx *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

void orc_select(const double *r, const double *cu, int N, int n, int q,
                int *ces, int *es, double *c_es) {
  keyidx *a = (keyidx *)malloc(sizeof(keyidx) * N);
  for (int j = 0; j < N; ++j) {
    a[j].key = r[j];
    a[j].idx = j;
  }
  qsort(a, N, sizeof(keyidx), cmp_keyidx);
  keyidx *b = (keyidx *)malloc(sizeof(keyidx) * n);
  for (int i = 0; i < n; ++i) {
    ces[i] = a[i].idx;
    b[i].key = cu[a[i].idx] + r[a[i].idx];
    b[i].idx = a[i].idx;
  }
  qsort(b, n, sizeof(keyidx), cmp_keyidx);
  for (int i = 0; i < q; ++i) {
    es[i] = b[i].idx;
    c_es[i] = b[i].key;
  }
  free(a);
  free(b);
}

/* ------------------------------------------------------------------ */
/* Update of the sampling distribution, eqs. mean_update, cov_update and
 * s_formula. (reading: the exponent is shifted by the minimum cost of the
 * EliteSet, which leaves the normalised weights unchanged.)             */

void orc_update(const orc_params *par, const double *mu, const double *Sigma,
                const double *p, const int *es, const double *c_es, int q,
                double *mu_out, double *Sigma_out) {
  double cmin = c_es[0];
  for (int i = 1; i < q; ++i)
    if (c_es[i] < cmin) cmin = c_es[i];
  double *s = (double *)malloc(sizeof(double) * q);
  double ssum = 0.0;
  for (int i = 0; i < q; ++i) {
    s[i] = exp(-(c_es[i] - cmin) / par->gamma);
    ssum += s[i];
  }
  double m[NP] = {0};
  for (int i = 0; i < q; ++i)
    for (int a = 0; a < NP; ++a) m[a] += s[i] * p[(size_t)es[i] * NP + a];
  double mu_new[NP];
  for (int a = 0; a < NP; ++a)
    mu_new[a] = (1.0 - par->eta) * mu[a] + par->eta * m[a] / ssum;
  double C[NP * NP] = {0};
  for (int i = 0; i < q; ++i) {
    const double *pj = p + (size_t)es[i] * NP;
    for (int a = 0; a < NP; ++a)
      for (int b = 0; b < NP; ++b)
        C[a * NP + b] += s[i] * (pj[a] - mu_new[a]) * (pj[b] - mu_new[b]);
  }
  double S2[NP * NP];
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b)
      S2[a * NP + b] =
          (1.0 - par->eta) * Sigma[a * NP + b] + par->eta * C[a * NP + b] / ssum;
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b)
      Sigma_out[a * NP + b] = 0.5 * (S2[a * NP + b] + S2[b * NP + a]);
  memcpy(mu_out, mu_new, sizeof(mu_new));
  free(s);
}

/* ------------------------------------------------------------------ */
/* Random numbers. Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64
 * multiplications with multipliers 0xD2511F53 and 0xCD9E8D57; the key is
 * bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
 * (reading: the paper only says "draw samples"; counter = (sample,
 * iteration, block, 0), key = (seed low word, seed high word).)          */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 24 high bits -> (0, 1]. */
static double unit_open0(uint32_t x) {
  return ((double)(x >> 8) + 1.0) * (1.0 / 16777216.0);
}

/* Box-Muller: two uniforms in (0, 1] -> two standard normals. */
static void box_muller(uint32_t a, uint32_t b, double *n0, double *n1) {
  double u1 = unit_open0(a), u2 = unit_open0(b);
  double rad = sqrt(-2.0 * log(u1));
  *n0 = rad * cos(2.0 * ORC_PI * u2);
  *n1 = rad * sin(2.0 * ORC_PI * u2);
}

static void philox_block(uint64_t seed, int j, int l, int blk, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)j, (uint32_t)l, (uint32_t)blk, 0u};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* Initial sampler, a stand-in for the learned CVAE sampler of Sec. III-D.
 * Set-points: one lane centre per sample (uniform over 3) plus
 * N(0, lane_sigma^2) on each of the 4 lateral set-points; each velocity
 * set-point U(vd_lo, vd_hi]. Goal positions: y_f the same lane draw (one
 * set-point's worth), x_f - x0 = t_f U(vd_lo, vd_hi] (the distance covered at
 * a velocity drawn like a set-point). Its exact moments seed the first
 * update; the fixed grid (sampler 1) discretises the same distribution and
 * uses the same moments. */
void orc_initial_moments(const orc_params *par, double *mu, double *Sigma) {
  double mc = (par->lane_c[0] + par->lane_c[1] + par->lane_c[2]) / 3.0;
  double vc = 0.0;
  for (int i = 0; i < 3; ++i) vc += (par->lane_c[i] - mc) * (par->lane_c[i] - mc);
  vc /= 3.0;
  double vm = 0.5 * (par->vd_lo + par->vd_hi);
  double vv = (par->vd_hi - par->vd_lo) * (par->vd_hi - par->vd_lo) / 12.0;
  memset(Sigma, 0, sizeof(double) * NP * NP);
  memset(mu, 0, sizeof(double) * NP);
  if (par->behaviour) {
    mu[0] = par->t_f * vm;
    Sigma[0] = par->t_f * par->t_f * vv;
    mu[1] = mc;
    Sigma[1 * NP + 1] = vc + par->lane_sigma * par->lane_sigma;
    return;
  }
  for (int a = 0; a < NSEG; ++a) {
    mu[a] = mc;
    mu[NSEG + a] = vm;
    for (int b = 0; b < NSEG; ++b)
      Sigma[a * NP + b] = vc + (a == b ? par->lane_sigma * par->lane_sigma : 0.0);
    Sigma[(NSEG + a) * NP + NSEG + a] = vv;
  }
}

/* Fixed grid of the first upper iteration (MPC-Grid of Sec. V-A samples a
 * pre-specified grid): sample j takes lane centre j mod 3 and the velocity
 * vd_lo + (vd_hi - vd_lo) (floor(j/3) + 1/2) / ceil(N/3), held over the
 * whole horizon (set-points) or as the goal t_f v ahead in that lane. */
static void grid_point(const orc_params *par, int j, int N, double *pj) {
  int nb = (N + 2) / 3;
  double lane = par->lane_c[j % 3];
  double v = par->vd_lo + (par->vd_hi - par->vd_lo) * ((double)(j / 3) + 0.5) / (double)nb;
  memset(pj, 0, sizeof(double) * NP);
  if (par->behaviour) {
    pj[0] = par->t_f * v;
    pj[1] = lane;
    return;
  }
  for (int m = 0; m < NSEG; ++m) {
    pj[m] = lane;
    pj[NSEG + m] = v;
  }
}

void orc_sample(const orc_params *par, uint64_t seed, int l, int N,
                int structured, const double *mu, const double *Lc, double *p) {
  for (int j = 0; j < N; ++j) {
    uint32_t w[12];
    double *pj = p + (size_t)j * NP;
    if (structured && par->sampler == 1) {
      grid_point(par, j, N, pj);
      continue;
    }
    philox_block(seed, j, l, 0, w);
    philox_block(seed, j, l, 1, w + 4);
    if (structured) {
      philox_block(seed, j, l, 2, w + 8);
      double n[4];
      box_muller(w[0], w[1], &n[0], &n[1]);
      box_muller(w[2], w[3], &n[2], &n[3]);
      int lane = (int)(((uint64_t)w[8] * 3u) >> 32);
      if (par->behaviour) {
        memset(pj, 0, sizeof(double) * NP);
        pj[0] = par->t_f * (par->vd_lo + (par->vd_hi - par->vd_lo) * unit_open0(w[4]));
        pj[1] = par->lane_c[lane] + par->lane_sigma * n[0];
        continue;
      }
      for (int m = 0; m < NSEG; ++m) {
        pj[m] = par->lane_c[lane] + par->lane_sigma * n[m];
        pj[NSEG + m] =
            par->vd_lo + (par->vd_hi - par->vd_lo) * unit_open0(w[4 + m]);
      }
    } else {
      double z[NP];
      for (int m = 0; m < NP; m += 2) box_muller(w[m], w[m + 1], &z[m], &z[m + 1]);
      /* with goal positions only the first two inputs are drawn */
      int nd = par->behaviour ? 2 : NP;
      for (int a = 0; a < NP; ++a) {
        double v = 0.0;
        if (a < nd) {
          v = mu[a];
          for (int b = 0; b <= a; ++b) v += Lc[a * NP + b] * z[b];
        }
        pj[a] = v;
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Alg. 1.                                                               */

/* Latent draws of the decoder sampler (App. A: z ~ N(0, I), 2-d): z_j is
 * the Box-Muller pair of words 0, 1 of Philox block (j, 0, 0, 0), the block
 * the structured sampler takes its first two normals from. */
void orc_decoder_latent(uint64_t seed, int N, double *z) {
  for (int j = 0; j < N; ++j) {
    uint32_t w[4];
    philox_block(seed, j, 0, 0, w);
    box_muller(w[0], w[1], &z[2 * j], &z[2 * j + 1]);
  }
}

/* Mean and covariance (normalised by N) of N samples p (N x 8), in two
 * passes: the distribution the samples of a learned sampler come from, as
 * far as N draws show it. */
void orc_sample_moments(const double *p, int N, double *mu, double *Sigma) {
  for (int a = 0; a < NP; ++a) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += p[(size_t)j * NP + a];
    mu[a] = s / (double)N;
  }
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) {
      double s = 0.0;
      for (int j = 0; j < N; ++j)
        s += (p[(size_t)j * NP + a] - mu[a]) * (p[(size_t)j * NP + b] - mu[b]);
      Sigma[a * NP + b] = s / (double)N;
    }
}

static int plan_impl(const orc_params *par, const orc_scene *sc, uint64_t seed, int N,
                     const double *mu0, const double *Sigma0, const double *p0,
                     orc_plan_out *out, orc_plan_trace *tr);

int orc_plan(const orc_params *par, const orc_scene *sc, uint64_t seed, int N,
             const double *mu0, const double *Sigma0, orc_plan_out *out,
             orc_plan_trace *tr) {
  return plan_impl(par, sc, seed, N, mu0, Sigma0, NULL, out, tr);
}

/* Alg. 1 started from given samples p0 (N x 8) instead of a draw: the first
 * iteration evaluates p0 (the decoder sampler's output, App. A), and the
 * distribution before the first update is their sample moments. */
int orc_plan_p0(const orc_params *par, const orc_scene *sc, uint64_t seed, int N,
                const double *p0, orc_plan_out *out, orc_plan_trace *tr) {
  if (p0 == NULL) return -1;
  return plan_impl(par, sc, seed, N, NULL, NULL, p0, out, tr);
}

static int plan_impl(const orc_params *par, const orc_scene *sc, uint64_t seed, int N,
                     const double *mu0, const double *Sigma0, const double *p0,
                     orc_plan_out *out, orc_plan_trace *tr) {
  int n, q;
  orc_elite_sizes(par, N, &n, &q);
  double mu[NP], Sigma[NP * NP], Lc[NP * NP];
  int structured = p0 == NULL && (mu0 == NULL || Sigma0 == NULL);
  if (p0 != NULL) {
    orc_sample_moments(p0, N, mu, Sigma);
  } else if (structured) {
    orc_initial_moments(par, mu, Sigma);
  } else {
    memcpy(mu, mu0, sizeof(mu));
    memcpy(Sigma, Sigma0, sizeof(Sigma));
  }
  double *p = (double *)malloc(sizeof(double) * N * NP);
  double *xb = (double *)malloc(sizeof(double) * N * NX);
  double *xs = (double *)malloc(sizeof(double) * N * NX);
  double *r = (double *)malloc(sizeof(double) * N);
  double *cu = (double *)malloc(sizeof(double) * N);
  int *ces = (int *)malloc(sizeof(int) * n);
  int *es = (int *)malloc(sizeof(int) * q);
  double *c_es = (double *)malloc(sizeof(double) * q);
  int rc = 0;
  for (int l = 0; l < par->L; ++l) {
    int draw_structured = structured && l == 0;
    if (p0 != NULL && l == 0) {
      memcpy(p, p0, sizeof(double) * N * NP);
    } else {
      if (!draw_structured) {
        if (orc_cholesky(Sigma, NP, par->cov_jitter, Lc) != 0) {
          rc = -2;
          break;
        }
      }
      orc_sample(par, seed, l, N, draw_structured, mu, Lc, p);
    }
    orc_step1(par, sc, p, N, xb);
    orc_project(par, sc, xb, p, N, xs, NULL);
    orc_residual_cost(par, sc, xs, N, r, cu);
    orc_select(r, cu, N, n, q, ces, es, c_es);
    double mu_n[NP], S_n[NP * NP];
    orc_update(par, mu, Sigma, p, es, c_es, q, mu_n, S_n);
    memcpy(mu, mu_n, sizeof(mu));
    memcpy(Sigma, S_n, sizeof(Sigma));
    if (tr) {
      if (tr->p) memcpy(tr->p + (size_t)l * N * NP, p, sizeof(double) * N * NP);
      if (tr->xi_bar)
        memcpy(tr->xi_bar + (size_t)l * N * NX, xb, sizeof(double) * N * NX);
      if (tr->xi_star)
        memcpy(tr->xi_star + (size_t)l * N * NX, xs, sizeof(double) * N * NX);
      if (tr->r) memcpy(tr->r + (size_t)l * N, r, sizeof(double) * N);
      if (tr->cu) memcpy(tr->cu + (size_t)l * N, cu, sizeof(double) * N);
      if (tr->ces) memcpy(tr->ces + (size_t)l * n, ces, sizeof(int) * n);
      if (tr->es) memcpy(tr->es + (size_t)l * q, es, sizeof(int) * q);
      if (tr->c_es) memcpy(tr->c_es + (size_t)l * q, c_es, sizeof(double) * q);
      if (tr->mu) memcpy(tr->mu + (size_t)l * NP, mu, sizeof(mu));
      if (tr->Sigma) memcpy(tr->Sigma + (size_t)l * NP * NP, Sigma, sizeof(Sigma));
    }
    if (l == par->L - 1) {
      /* Return: lowest c_u + r in the final EliteSet (ties: lower index). */
      int b = es[0];
      out->best_index = b;
      memcpy(out->p_best, p + (size_t)b * NP, sizeof(double) * NP);
      memcpy(out->xi_best, xs + (size_t)b * NX, sizeof(double) * NX);
      out->cost_upper = cu[b];
      out->residual = r[b];
    }
  }
  memcpy(out->mu, mu, sizeof(mu));
  memcpy(out->Sigma, Sigma, sizeof(Sigma));
  free(p);
  free(xb);
  free(xs);
  free(r);
  free(cu);
  free(ces);
  free(es);
  free(c_es);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Receding-horizon loop (MPC-Bi-Level, Sec. V-A "MPC Baselines"): the ego
 * executes the first n_exec instants of its trajectory, then replans from
 * the state reached. Neighbours keep their velocities (the constant-velocity
 * motion of the collision row of Table ineq_list). Scene time of instant m
 * of an episode: s_m = m t_f / (T - 1); cycle c starts at m = c n_exec. A
 * neighbour with first-cycle position p and velocity v is at fma(v, s, p)
 * (the exactly rounded p + v s). An executed instant k = 0..n_exec collides
 * with a neighbour when ((x - x_o)/a)^2 + ((y - y_o)/b)^2 < 1. */

static double scene_time(long m, double t_f, int T) {
  return ((double)m * t_f) / (double)(T - 1);
}

int orc_advance(const orc_params *par, const double *xi, const double *obs0, int M, int cycle, int n_exec,
                double *ego_next, double *obs_next, int *collided) {
  const int T = par->T;
  if (n_exec < 1 || n_exec > T - 1 || cycle < 0) return -1;
  double *W = (double *)malloc(sizeof(double) * T * NC);
  double *Wd = (double *)malloc(sizeof(double) * T * NC);
  double *Wdd = (double *)malloc(sizeof(double) * T * NC);
  orc_basis(T, par->t_f, W, Wd, Wdd);
  /* trajectory of eq. param at instant k: rows of W, Wd, Wdd times the
   * coefficients of each axis */
  int hit = 0;
  for (int k = 0; k <= n_exec; ++k) {
    double x = 0.0, y = 0.0;
    for (int i = 0; i < NC; ++i) {
      x += W[k * NC + i] * xi[i];
      y += W[k * NC + i] * xi[NC + i];
    }
    const double s = scene_time((long)cycle * n_exec + k, par->t_f, T);
    for (int m = 0; m < M; ++m) {
      const double xo = fma(obs0[4 * m + 2], s, obs0[4 * m + 0]);
      const double yo = fma(obs0[4 * m + 3], s, obs0[4 * m + 1]);
      const double u = (x - xo) / par->ell_a, v = (y - yo) / par->ell_b;
      if (u * u + v * v < 1.0) hit = 1;
    }
  }
  const int k = n_exec;
  double st[6] = {0, 0, 0, 0, 0, 0}; /* x, y, xdot, ydot, xddot, yddot */
  for (int i = 0; i < NC; ++i) {
    st[0] += W[k * NC + i] * xi[i];
    st[1] += W[k * NC + i] * xi[NC + i];
    st[2] += Wd[k * NC + i] * xi[i];
    st[3] += Wd[k * NC + i] * xi[NC + i];
    st[4] += Wdd[k * NC + i] * xi[i];
    st[5] += Wdd[k * NC + i] * xi[NC + i];
  }
  memcpy(ego_next, st, sizeof(st));
  const double sn = scene_time((long)(cycle + 1) * n_exec, par->t_f, T);
  for (int m = 0; m < M; ++m) {
    obs_next[4 * m + 0] = fma(obs0[4 * m + 2], sn, obs0[4 * m + 0]);
    obs_next[4 * m + 1] = fma(obs0[4 * m + 3], sn, obs0[4 * m + 1]);
    obs_next[4 * m + 2] = obs0[4 * m + 2];
    obs_next[4 * m + 3] = obs0[4 * m + 3];
  }
  *collided = hit;
  free(W);
  free(Wd);
  free(Wdd);
  return 0;
}
