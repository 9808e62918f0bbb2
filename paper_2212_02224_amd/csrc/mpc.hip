// mpc.hip -- receding-horizon closed loop of the batched bi-level planner
// (MPC-Bi-Level of Sec. V-A; optionally with the warm start of Sec. IV).
//
//   advance_kernel  after a planning cycle's L upper iterations, one 64-lane
//                   workgroup per episode executes the first n_exec instants
//                   of the returned trajectory (FP64), tests them against
//                   every neighbour's ellipse (collision row of Table
//                   ineq_list) and writes the next cycle's descriptor in
//                   place, so consecutive cycles need no host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_internal.h"
#include "traj64.h"

namespace plan {

// Scene time of absolute instant m of an episode (cycle c starts at
// m = c n_exec): m t_f / (T - 1), one rounding per operation.
__device__ __forceinline__ double scene_time(int64_t m, double t_f, int T) {
  return ((double)m * t_f) / (double)(T - 1);
}

__global__ void __launch_bounds__(kWave) advance_kernel(AdvArgs A, MethodParams P) {
  __shared__ double s_xi[22];
  __shared__ double s_ego[6];
  const int e = blockIdx.x, lane = threadIdx.x;
  ReqDesc &D = A.desc[e];
  const ResultRec &R = A.result[e];
  const DistState &Sd = A.dist[e];
  const int T = D.T, M = D.M, ne = A.n_exec, c = A.cycle;
  const bool ok = R.status == 0;
  const size_t ec = (size_t)e * A.cycles + c;
  if (lane < 22) s_xi[lane] = R.xi[lane];
  if (lane < 6) s_ego[lane] = D.ego[lane];
  __syncthreads();

  if (A.xi && lane < 22) A.xi[ec * 22 + lane] = s_xi[lane];
  if (A.mu && lane < 8) A.mu[ec * 8 + lane] = Sd.mu[lane];
  if (A.sigma) A.sigma[ec * 64 + lane] = Sd.sigma[lane];
  if (lane == 0) {
    if (A.cost) {
      A.cost[ec * 2] = R.cost_upper;
      A.cost[ec * 2 + 1] = R.residual;
    }
    if (A.status) A.status[ec] = R.status;
  }

  // Executed instants k = 0..n_exec against every neighbour's ellipse (the
  // collision row of Table ineq_list), neighbours at constant velocity from
  // their first-cycle positions.
  const double *o0 = A.obs0 + (size_t)e * PLAN_MAX_M * 2;
  bool hit = false;
  if (ok) {
    for (int k = lane; k <= ne; k += kWave) {
      const double tau = (double)k / (double)(T - 1);
      double x, xd, xdd, y, yd, ydd;
      bernstein_state(s_xi, tau, P.t_f, x, xd, xdd);
      bernstein_state(s_xi + 11, tau, P.t_f, y, yd, ydd);
      const double sm = scene_time((int64_t)c * ne + k, P.t_f, T);
      for (int i = 0; i < M; ++i) {
        const double dx = (x - fma(D.obs[i][2], sm, o0[2 * i])) / P.ell_a;
        const double dy = (y - fma(D.obs[i][3], sm, o0[2 * i + 1])) / P.ell_b;
        if (dx * dx + dy * dy < 1.0) hit = true;
      }
    }
  }
  const bool any_hit = __any(hit);

  // Next cycle: the state reached at t_{n_exec} (held if the plan failed),
  // the neighbours moved on, a fresh sample stream, and the initial
  // distribution: the structured sampler, or the warm start.
  if (lane == 0 && ok) {
    const double tau = (double)ne / (double)(T - 1);
    double st[6];
    bernstein_state(s_xi, tau, P.t_f, st[0], st[2], st[4]);
    bernstein_state(s_xi + 11, tau, P.t_f, st[1], st[3], st[5]);
    for (int a = 0; a < 6; ++a) s_ego[a] = st[a];
  }
  __syncthreads();
  const double sn = scene_time((int64_t)(c + 1) * ne, P.t_f, T);
  if (lane < M) {
    D.obs[lane][0] = fma(D.obs[lane][2], sn, o0[2 * lane]);
    D.obs[lane][1] = fma(D.obs[lane][3], sn, o0[2 * lane + 1]);
  }
  if (lane < 6) {
    D.ego[lane] = s_ego[lane];
    if (A.ego) A.ego[((size_t)e * (A.cycles + 1) + c + 1) * 6 + lane] = s_ego[lane];
  }
  if (lane == 0) {
    if (A.collided) A.collided[ec] = any_hit ? 1 : 0;
    D.seed += 1;
    if (!A.warm) {
      D.init_mode = kInitStructured;
    } else if (ok && D.session_wb >= 0) {
      D.init_mode = kInitSession;
      D.session = D.session_wb;
    }
  }
}

hipError_t launch_advance(const AdvArgs &a, const MethodParams &p, int n, hipStream_t st) {
  hipLaunchKernelGGL(advance_kernel, dim3(n), dim3(kWave), 0, st, a, p);
  return hipGetLastError();
}

}  // namespace plan
