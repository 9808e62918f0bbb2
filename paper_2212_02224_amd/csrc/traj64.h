// traj64.h -- FP64 evaluation of a returned trajectory on the device: the
// Bernstein polynomial of eq. param and its derivatives, and the constraint
// residual and upper cost of Table ineq_list / Sec. V-A at one instant.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_internal.h"

namespace plan {

// Position, velocity and acceleration of one axis at tau = t / t_f from its
// 11 Bernstein coefficients (FP64): the derivatives are Bernstein sums of
// degree 9 and 8 over the forward differences of the coefficients.
__device__ inline void bernstein_state(const double *c, double tau, double t_f, double &pos, double &vel,
                                       double &acc) {
  const double b10[11] = {1, 10, 45, 120, 210, 252, 210, 120, 45, 10, 1};
  const double b9[10] = {1, 9, 36, 84, 126, 126, 84, 36, 9, 1};
  const double b8[9] = {1, 8, 28, 56, 70, 56, 28, 8, 1};
  double tp[11], up[11];
  tp[0] = up[0] = 1.0;
  for (int i = 1; i <= 10; ++i) {
    tp[i] = tp[i - 1] * tau;
    up[i] = up[i - 1] * (1.0 - tau);
  }
  double p = 0.0, v = 0.0, a = 0.0;
  for (int i = 0; i <= 10; ++i) p += b10[i] * tp[i] * up[10 - i] * c[i];
  for (int i = 0; i <= 9; ++i) v += b9[i] * tp[i] * up[9 - i] * (c[i + 1] - c[i]);
  for (int i = 0; i <= 8; ++i) a += b8[i] * tp[i] * up[8 - i] * (c[i + 2] - 2.0 * c[i + 1] + c[i]);
  pos = p;
  vel = 10.0 * v / t_f;
  acc = 90.0 * a / (t_f * t_f);
}

// The request's road at position x (same coordinate as ego[0]): curvature
// and lane limits, linear between the knots of its profile and constant
// beyond; without a profile the constant curvature and the configured limits.
__device__ inline void road64(const ReqDesc &D, const MethodParams &P, double x, double &kappa, double &y_lb,
                              double &y_ub) {
  if (D.n_road <= 0) {
    kappa = D.kappa;
    y_lb = P.y_lb;
    y_ub = P.y_ub;
    return;
  }
  if (D.n_road == 1) {
    kappa = D.road[0][0];
    y_lb = D.road[0][1];
    y_ub = D.road[0][2];
    return;
  }
  const int last = D.n_road - 1;
  const double u = fmin(fmax((x - D.road_x0) / D.road_dx, 0.0), (double)last);
  const int i = min((int)floor(u), last - 1);
  const double f = u - (double)i;
  kappa = D.road[i][0] + f * (D.road[i + 1][0] - D.road[i][0]);
  y_lb = D.road[i][1] + f * (D.road[i + 1][1] - D.road[i][1]);
  y_ub = D.road[i][2] + f * (D.road[i + 1][2] - D.road[i][2]);
}

// Residual terms (Table ineq_list, summed max(0, g)) and upper cost
// (|v| - v_max)^2 (Sec. V-A) of trajectory xi (22 FP64 coefficients) at
// instant k of the request's horizon; also its position (x, y).
__device__ inline void residual_cost64(const ReqDesc &D, const MethodParams &P, const double *xi, int k,
                                       double &res, double &cost, double &x, double &y) {
  const int T = D.T;
  const double tk = P.t_f * (double)k / (double)(T - 1);
  const double tau = (double)k / (double)(T - 1);
  double xd, xdd, yd, ydd;
  bernstein_state(xi, tau, P.t_f, x, xd, xdd);
  bernstein_state(xi + 11, tau, P.t_f, y, yd, ydd);
  double r = 0.0;
  for (int i = 0; i < D.M; ++i) {
    const double dx = (x - (D.obs[i][0] + D.obs[i][2] * tk)) / P.ell_a;
    const double dy = (y - (D.obs[i][1] + D.obs[i][3] * tk)) / P.ell_b;
    r += fmax(0.0, 1.0 - dx * dx - dy * dy);
  }
  const double v = sqrt(xd * xd + yd * yd), a = sqrt(xdd * xdd + ydd * ydd);
  r += fmax(0.0, v - P.v_max) + fmax(0.0, P.v_min - v) + fmax(0.0, a - P.a_max);
  const double vd = fmax(v, P.v_eps);
  r += fmax(0.0, fabs(ydd * xd - xdd * yd) / (vd * vd * vd) - P.kappa_max);
  double kappa, y_lb, y_ub;
  road64(D, P, x, kappa, y_lb, y_ub);
  r += fmax(0.0, fabs(xd * xd * kappa) - P.c_max);
  r += fmax(0.0, y - y_ub) + fmax(0.0, y_lb - y);
  res = r;
  cost = (v - P.v_max) * (v - P.v_max);
}

}  // namespace plan
