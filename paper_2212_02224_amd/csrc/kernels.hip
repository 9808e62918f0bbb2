// kernels.hip -- CDNA4 (gfx950) kernels of the batched bi-level planner.
//
//   lower_kernel          Alg. 1 Steps 1-2 and the residual for every sample
//                         of every resident request: the Step-1 QP through
//                         its precomputed affine map (Sec. III-C, eq. over_3),
//                         K iterations of Alg. 2, then r_j and c_u,j.
//   init_kernel           sampling distribution of iteration 0 and its draw.
//   select_update_kernel  ConstraintEliteSet / EliteSet (Alg. 1), the update
//                         of eqs. mean_update, cov_update, s_formula (FP64),
//                         the Cholesky factor and the next iteration's draw.
//
// Lower-level algebra (mathematically identical to Alg. 2; the oracle does it
// the literal way). With the boundary conditions of eqs.
// boundary_cond_initial / final_boundary the coefficients are xi = N z +
// xi_f(b_0), N a 0/1 selection (x: c3..c10 free; y: c3..c8 free, c9 = c10
// free). The xi-update of eq. split_xy in these coordinates reads
//     z <- z + A^-1 (N^T N (z_bar - z) + N^T lambda + rho N^T g),
//     A = N^T N + rho N^T (F^T F + G^T G) N,
// where g = F^T (h - F xi) + G^T (e - s - G xi) is built only from the
// differences between the targets of the (alpha, d) step and the current
// trajectory (zero when a constraint is inactive), and the multiplier step of
// eq. update_lagrange is N^T lambda <- N^T lambda + (rho / 2) N^T g.
// F_o^T F_o = M W^T W and F_o^T h_o = W^T sum_i h_o,i, so the neighbours are
// summed per instant before the single W^T product.
//
// The x axis is carried relative to the line x0 + vx0 t (exact in the basis),
// which keeps FP32 magnitudes small; obstacle positions are shifted alike.
//
// Layout: a workgroup of 4 waves serves one request; each sample takes
// ceil(T/64) waves, one horizon instant per lane. The neighbours' positions
// at every instant are staged in LDS once per workgroup. The 15 sums over
// time of N^T g are formed by a transpose-reduction across the wave (17
// shuffles), the small A^-1 product by broadcasting through scalar
// registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_internal.h"

namespace plan {

// ---------------------------------------------------------------------------
// Fast scalar helpers (hardware rcp / rsq / sqrt, ~1 ulp).
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ float bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

__device__ __forceinline__ float xorf(float v, int m) { return __shfl_xor(v, m, 64); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += xorf(v, m);
  return v;
}

// Sum over the 64 lanes of 16 per-lane values; lane l returns value l >> 2.
__device__ __forceinline__ float reduce16(const float (&v)[16], int lane) {
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
  float a[8], b[4], c[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float keep = h5 ? v[i + 8] : v[i];
    float send = h5 ? v[i] : v[i + 8];
    a[i] = keep + xorf(send, 32);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float keep = h4 ? a[i + 4] : a[i];
    float send = h4 ? a[i] : a[i + 4];
    b[i] = keep + xorf(send, 16);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    float keep = h3 ? b[i + 2] : b[i];
    float send = h3 ? b[i] : b[i + 2];
    c[i] = keep + xorf(send, 8);
  }
  float keep = h2 ? c[1] : c[0];
  float send = h2 ? c[0] : c[1];
  float d = keep + xorf(send, 4);
  d += xorf(d, 2);
  d += xorf(d, 1);
  return d;
}

// ---------------------------------------------------------------------------
// Lower level.

struct Lane {
  // basis rows of this lane's instant (free columns)
  float bx[8], bdx[8], bddx[8];
  float by7, bdy7, bddy7;
  // fixed part of the trajectory (relative x frame)
  float xf, xdf, xddf, yf, ydf, yddf;
};

struct Scal {
  float vx0, rho, ia2, ib2, ell_a;
  float v_min, v_max, a_max, kmax, inv_kmax, c_max, kappa_abs, y_lb, y_ub, v_eps;
};

struct State6 {
  float x, xd, xdd, y, yd, ydd;
};

__device__ __forceinline__ State6 eval_traj(const Lane &L, const float (&zs)[15], float vx0) {
  State6 s;
  s.x = L.xf;
  s.xd = vx0 + L.xdf;
  s.xdd = L.xddf;
  s.y = L.yf;
  s.yd = L.ydf;
  s.ydd = L.yddf;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    s.x = fmaf(L.bx[c], zs[c], s.x);
    s.xd = fmaf(L.bdx[c], zs[c], s.xd);
    s.xdd = fmaf(L.bddx[c], zs[c], s.xdd);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    s.y = fmaf(L.bx[c], zs[8 + c], s.y);
    s.yd = fmaf(L.bdx[c], zs[8 + c], s.yd);
    s.ydd = fmaf(L.bddx[c], zs[8 + c], s.ydd);
  }
  s.y = fmaf(L.by7, zs[14], s.y);
  s.yd = fmaf(L.bdy7, zs[14], s.yd);
  s.ydd = fmaf(L.bddy7, zs[14], s.ydd);
  return s;
}

// One target pass (steps split_alpha_o .. update_slack of Alg. 2) at this
// lane's instant, accumulated into the lane's share of N^T g.
__device__ __forceinline__ void target_pass(const Lane &L, const Scal &S, const float (&zs)[15],
                                            const float2 *__restrict__ obs, int M, int T,
                                            int t, bool tv, float &da_prev, float (&g)[16]) {
  State6 s = eval_traj(L, zs, S.vx0);
  // neighbours: target minus trajectory, summed over i
  float dox = 0.f, doy = 0.f;
  for (int i = 0; i < M; ++i) {
    float2 o = obs[i * T + t];
    float dx = s.x - o.x, dy = s.y - o.y;
    float q = fmaf(dx * dx, S.ia2, dy * dy * S.ib2);
    if (q < 1.f) {
      if (q > 0.f) {
        float f = frsq(q) - 1.f;
        dox = fmaf(f, dx, dox);
        doy = fmaf(f, dy, doy);
      } else {
        dox += S.ell_a;  // centre: alpha = 0, d = 1
      }
    }
  }
  // velocity / acceleration polar variables and their clips
  float v2 = fmaf(s.xd, s.xd, s.yd * s.yd);
  float a2 = fmaf(s.xdd, s.xdd, s.ydd * s.ydd);
  float rv = v2 > 0.f ? frsq(v2) : 0.f;
  float ra = a2 > 0.f ? frsq(a2) : 0.f;
  float vn = v2 * rv, an = a2 * ra;
  float cv = v2 > 0.f ? s.xd * rv : 1.f, sv = s.yd * rv;
  float ca = a2 > 0.f ? s.xdd * ra : 1.f, sa = s.ydd * ra;
  float sig = fabsf(sa * cv - ca * sv);
  float vlo = fmaxf(S.v_min, fsqrt(da_prev * sig * S.inv_kmax));
  float vhi = S.v_max;
  if (S.kappa_abs > 0.f) {
    float den = S.kappa_abs * cv * cv;
    if (den > 0.f) vhi = fminf(vhi, fsqrt(S.c_max * frcp(den)));
  }
  float dv = fminf(fmaxf(vn, vlo), vhi);
  float ahi = S.a_max;
  if (sig > 0.f) ahi = fminf(ahi, dv * dv * S.kmax * frcp(sig));
  float dan = fminf(fmaxf(an, 0.f), ahi);
  float dvx, dvy, dax, day;
  if (v2 > 0.f) {
    float k = (dv - vn) * rv;
    dvx = k * s.xd;
    dvy = k * s.yd;
  } else {
    dvx = dv;
    dvy = 0.f;
  }
  if (a2 > 0.f) {
    float k = (dan - an) * ra;
    dax = k * s.xdd;
    day = k * s.ydd;
  } else {
    dax = dan;
    day = 0.f;
  }
  if (tv) da_prev = dan;
  // lane bounds: e - s - G xi = clip(y, y_lb, y_ub) - y
  float dl = fminf(fmaxf(s.y, S.y_lb), S.y_ub) - s.y;
  float wy = doy + dl;
  if (!tv) {
    dox = wy = dvx = dvy = dax = day = 0.f;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    g[c] = fmaf(L.bx[c], dox, fmaf(L.bdx[c], dvx, L.bddx[c] * dax));
#pragma unroll
  for (int c = 0; c < 6; ++c)
    g[8 + c] = fmaf(L.bx[c], wy, fmaf(L.bdx[c], dvy, L.bddx[c] * day));
  g[14] = fmaf(L.by7, wy, fmaf(L.bdy7, dvy, L.bddy7 * day));
  g[15] = 0.f;
}

// Residual r (sum of max(0, g) over Table ineq_list) and upper cost c_u at
// this lane's instant.
__device__ __forceinline__ void residual_pass(const Lane &L, const Scal &S, const float (&zs)[15],
                                              const float2 *__restrict__ obs, int M, int T, int t,
                                              bool tv, float &res, float &cost) {
  State6 s = eval_traj(L, zs, S.vx0);
  float r = 0.f;
  for (int i = 0; i < M; ++i) {
    float2 o = obs[i * T + t];
    float dx = s.x - o.x, dy = s.y - o.y;
    float q = fmaf(dx * dx, S.ia2, dy * dy * S.ib2);
    r += fmaxf(0.f, 1.f - q);
  }
  float vn = fsqrt(fmaf(s.xd, s.xd, s.yd * s.yd));
  float an = fsqrt(fmaf(s.xdd, s.xdd, s.ydd * s.ydd));
  r += fmaxf(0.f, vn - S.v_max) + fmaxf(0.f, S.v_min - vn) + fmaxf(0.f, an - S.a_max);
  float vd = fmaxf(vn, S.v_eps);
  float curv = fabsf(s.ydd * s.xd - s.xdd * s.yd) * frcp(vd * vd * vd);
  r += fmaxf(0.f, curv - S.kmax);
  r += fmaxf(0.f, fabsf(s.xd * s.xd * S.kappa_abs) - S.c_max);
  r += fmaxf(0.f, s.y - S.y_ub) + fmaxf(0.f, S.y_lb - s.y);
  float e = vn - S.v_max;
  res = tv ? r : 0.f;
  cost = tv ? e * e : 0.f;
}

__global__ void __launch_bounds__(kBlock) lower_kernel(LowerArgs A, MethodParams P) {
  extern __shared__ float2 s_obs[];
  __shared__ float s_red[2][4][16];

  const int2 bi = A.blocks[blockIdx.x];
  const ReqDesc &D = A.desc[bi.x];
  const int T = D.T, M = D.M, N = D.N;
  const int NW = (T + kWave - 1) / kWave;
  const int spb = 4 / NW;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int sl = wave / NW;
  const int wi = wave - sl * NW;
  const int j = bi.y + sl;
  const bool active = (sl < spb) && (j < N);
  const int t = wi * kWave + lane;
  const bool tv = active && t < T;
  const int tt = t < T ? t : T - 1;
  const size_t slot_off = (size_t)bi.x * A.max_N;

  const double x0 = D.ego[0], y0 = D.ego[1], vx0 = D.ego[2], vy0 = D.ego[3];
  const double ax0 = D.ego[4], ay0 = D.ego[5];

  const float *Bt = A.basis + A.basis_off[D.t_idx];
  const int Tp = A.basis_tpad[D.t_idx];

  // Neighbour positions relative to the reference line, per instant.
  for (int idx = threadIdx.x; idx < M * T; idx += kBlock) {
    int i = idx / T, k = idx - i * T;
    double tk = (double)P.t_f * (double)k / (double)(T - 1);
    double ox = (D.obs[i][0] - x0) + (D.obs[i][2] - vx0) * tk;
    double oy = D.obs[i][1] + D.obs[i][3] * tk;
    s_obs[idx] = make_float2((float)ox, (float)oy);
  }

  Scal S;
  S.vx0 = (float)vx0;
  S.rho = (float)P.rho;
  S.ia2 = (float)(1.0 / (P.ell_a * P.ell_a));
  S.ib2 = (float)(1.0 / (P.ell_b * P.ell_b));
  S.ell_a = (float)P.ell_a;
  S.v_min = (float)P.v_min;
  S.v_max = (float)P.v_max;
  S.a_max = (float)P.a_max;
  S.kmax = (float)P.kappa_max;
  S.inv_kmax = (float)(1.0 / P.kappa_max);
  S.c_max = (float)P.c_max;
  S.kappa_abs = (float)fabs(D.kappa);
  S.y_lb = (float)P.y_lb;
  S.y_ub = (float)P.y_ub;
  S.v_eps = (float)P.v_eps;

  // Basis rows of this lane's instant and the fixed part of the trajectory.
  Lane L;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    L.bx[c] = Bt[(kColW + c) * Tp + tt];
    L.bdx[c] = Bt[(kColWd + c) * Tp + tt];
    L.bddx[c] = Bt[(kColWdd + c) * Tp + tt];
  }
  L.by7 = Bt[(kColY7 + 0) * Tp + tt];
  L.bdy7 = Bt[(kColY7 + 1) * Tp + tt];
  L.bddy7 = Bt[(kColY7 + 2) * Tp + tt];
  {
    const double n = 10.0, tf = P.t_f;
    // relative x frame: c0 = c1 = 0, c2 = ax0 t_f^2 / (n (n - 1))
    const double cx2 = ax0 * tf * tf / (n * (n - 1.0));
    const double cy0 = y0, cy1 = y0 + vy0 * tf / n;
    const double cy2 = y0 + 2.0 * vy0 * tf / n + ay0 * tf * tf / (n * (n - 1.0));
    float W0 = Bt[(kColFix + 0) * Tp + tt], W1 = Bt[(kColFix + 1) * Tp + tt],
          W2 = Bt[(kColFix + 2) * Tp + tt];
    float Wd0 = Bt[(kColFix + 3) * Tp + tt], Wd1 = Bt[(kColFix + 4) * Tp + tt],
          Wd2 = Bt[(kColFix + 5) * Tp + tt];
    float Wdd0 = Bt[(kColFix + 6) * Tp + tt], Wdd1 = Bt[(kColFix + 7) * Tp + tt],
          Wdd2 = Bt[(kColFix + 8) * Tp + tt];
    float fx2 = (float)cx2, fy0 = (float)cy0, fy1 = (float)cy1, fy2 = (float)cy2;
    L.xf = W2 * fx2;
    L.xdf = Wd2 * fx2;
    L.xddf = Wdd2 * fx2;
    L.yf = fmaf(W0, fy0, fmaf(W1, fy1, W2 * fy2));
    L.ydf = fmaf(Wd0, fy0, fmaf(Wd1, fy1, Wd2 * fy2));
    L.yddf = fmaf(Wdd0, fy0, fmaf(Wdd1, fy1, Wdd2 * fy2));
  }

  // Step 1 (eq. over_3 through its affine map): z_bar = S p' + R b'.
  const int v = lane >> 2;
  float pin[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) pin[m] = active ? A.p[(slot_off + j) * 8 + m] : 0.f;
  float zb;
  {
    const float *S1 = A.step1 + (size_t)D.t_idx * kStep1Floats;
    const float *R1 = S1 + 16 * 8;
    float pp[8];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      pp[m] = pin[m];
      pp[4 + m] = (float)((double)pin[4 + m] - vx0);
    }
    const float bb[4] = {(float)ax0, (float)y0, (float)vy0, (float)ay0};
    zb = 0.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) zb = fmaf(S1[v * 8 + m], pp[m], zb);
#pragma unroll
    for (int m = 0; m < 4; ++m) zb = fmaf(R1[v * 4 + m], bb[m], zb);
  }
  float arow[16];
  float Dv;
  {
    const float *Pj = A.proj + (size_t)D.tm_idx * kProjFloats;
#pragma unroll
    for (int c = 0; c < 16; ++c) arow[c] = Pj[v * 16 + c];
    Dv = Pj[256 + v];
  }
  __syncthreads();  // obstacle table ready

  float z = zb, mu = 0.f;
  float zs[15];
#pragma unroll
  for (int c = 0; c < 15; ++c) zs[c] = bcast(z, 4 * c);

  // Initial d_a: clip(|a(xi_bar)|, 0, a_max).
  float da_prev;
  {
    State6 s = eval_traj(L, zs, S.vx0);
    da_prev = fminf(fsqrt(fmaf(s.xdd, s.xdd, s.ydd * s.ydd)), S.a_max);
  }

  const float2 *obs = s_obs;
  int buf = 0;
  auto reduce_sample = [&](const float (&g)[16]) -> float {
    float r = reduce16(g, lane);
    if (NW > 1) {
      if ((lane & 3) == 0) s_red[buf][wave][v] = r;
      __syncthreads();
      r = 0.f;
      if (sl < spb)  // a wave beyond the last sample of the group only syncs
        for (int w = 0; w < NW; ++w) r += s_red[buf][sl * NW + w][v];
      buf ^= 1;
    }
    return r;
  };

  float g[16];
  target_pass(L, S, zs, obs, M, T, tt, tv, da_prev, g);
  float Gv = reduce_sample(g);

  const int K = P.K;
  for (int k = 1; k <= K; ++k) {
    // xi-update (eq. split_xy) in the free coordinates
    float rhs = fmaf(Dv, zb - z, fmaf(S.rho, Gv, mu));
    float rs[15];
#pragma unroll
    for (int c = 0; c < 15; ++c) rs[c] = bcast(rhs, 4 * c);
    float dz = 0.f;
#pragma unroll
    for (int c = 0; c < 15; ++c) dz = fmaf(arow[c], rs[c], dz);
    z += dz;
#pragma unroll
    for (int c = 0; c < 15; ++c) zs[c] = bcast(z, 4 * c);
    if (k < K) {
      target_pass(L, S, zs, obs, M, T, tt, tv, da_prev, g);
      Gv = reduce_sample(g);
      mu = fmaf(0.5f * S.rho, Gv, mu);  // eq. update_lagrange
    }
  }

  // Residual and upper cost of xi* = xi^K.
  float rr, cc;
  residual_pass(L, S, zs, obs, M, T, tt, tv, rr, cc);
  rr = wave_sum(rr);
  cc = wave_sum(cc);
  if (NW > 1) {
    if (lane == 0) {
      s_red[buf][wave][0] = rr;
      s_red[buf][wave][1] = cc;
    }
    __syncthreads();
    rr = 0.f;
    cc = 0.f;
    if (sl < spb)
      for (int w = 0; w < NW; ++w) {
        rr += s_red[buf][sl * NW + w][0];
        cc += s_red[buf][sl * NW + w][1];
      }
  }

  if (!active) return;
  const size_t row = slot_off + j;
  if ((lane & 3) == 0 && v < 15) A.zs[row * kZ + v] = z;
  if (wi == 0 && lane == 0) {
    A.resid[row] = rr;
    A.cost[row] = cc;
  }
  if (A.xi_star_out != nullptr && wi == 0) {
    // absolute coefficients in FP64: add back the reference line on x
    const double n = 10.0, tf = P.t_f;
    double *xs = A.xi_star_out + (size_t)j * 22;
    double *xb = A.xi_bar_out + (size_t)j * 22;
    if ((lane & 3) == 0 && v < 8) {
      double ref = x0 + vx0 * tf * (double)(3 + v) / n;
      xs[3 + v] = (double)z + ref;
      xb[3 + v] = (double)zb + ref;
    } else if ((lane & 3) == 0 && v >= 8 && v < 14) {
      xs[11 + 3 + (v - 8)] = (double)z;
      xb[11 + 3 + (v - 8)] = (double)zb;
    } else if ((lane & 3) == 0 && v == 14) {
      xs[11 + 9] = xs[11 + 10] = (double)z;
      xb[11 + 9] = xb[11 + 10] = (double)zb;
    } else if (lane == 61) {
      double c0 = x0, c1 = x0 + vx0 * tf / n;
      double c2 = x0 + 2.0 * vx0 * tf / n + ax0 * tf * tf / (n * (n - 1.0));
      double e0 = y0, e1 = y0 + vy0 * tf / n;
      double e2 = y0 + 2.0 * vy0 * tf / n + ay0 * tf * tf / (n * (n - 1.0));
      xs[0] = xb[0] = c0;
      xs[1] = xb[1] = c1;
      xs[2] = xb[2] = c2;
      xs[11] = xb[11] = e0;
      xs[12] = xb[12] = e1;
      xs[13] = xb[13] = e2;
    }
  }
}

// ---------------------------------------------------------------------------
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the request
// seed; counter (sample, iteration, block, 0). Box-Muller turns pairs of
// uniforms in (0, 1] into normals.

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c[0];
    uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2];
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void rng_block(uint64_t seed, int j, int l, int blk, uint32_t w[4]) {
  w[0] = (uint32_t)j;
  w[1] = (uint32_t)l;
  w[2] = (uint32_t)blk;
  w[3] = 0u;
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ float u01(uint32_t x) {
  return (float)((x >> 8) + 1u) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ void normals2(uint32_t a, uint32_t b, float &n0, float &n1) {
  float rad = sqrtf(-2.0f * logf(u01(a)));
  float s, c;
  sincospif(2.0f * u01(b), &s, &c);
  n0 = rad * c;
  n1 = rad * s;
}

// Draw sample j of upper iteration l into p (8 floats).
__device__ void draw_sample(const MethodParams &P, const ReqDesc &D, const DistState &Sd, int j,
                            int l, bool structured, float *p) {
  uint32_t w[12];
  rng_block(D.seed, j, l, 0, w);
  rng_block(D.seed, j, l, 1, w + 4);
  if (structured) {
    rng_block(D.seed, j, l, 2, w + 8);
    float n[4];
    normals2(w[0], w[1], n[0], n[1]);
    normals2(w[2], w[3], n[2], n[3]);
    int lane = (int)(((uint64_t)w[8] * 3u) >> 32);
    double lc = P.lane_c[lane];
    for (int m = 0; m < 4; ++m) {
      p[m] = (float)(lc + P.lane_sigma * (double)n[m]);
      double u = (double)((w[4 + m] >> 8) + 1u) * (1.0 / 16777216.0);
      p[4 + m] = (float)(P.vd_lo + (P.vd_hi - P.vd_lo) * u);
    }
  } else {
    float zf[8];
    for (int m = 0; m < 8; m += 2) normals2(w[m], w[m + 1], zf[m], zf[m + 1]);
    for (int a = 0; a < 8; ++a) {
      double s = Sd.mu[a];
      for (int b = 0; b <= a; ++b) s += Sd.chol[a * 8 + b] * (double)zf[b];
      p[a] = (float)s;
    }
  }
}

// Lower Cholesky factor of A + jitter I (8x8, FP64). Returns false if not
// positive definite.
__device__ bool chol8(const double *A, double jitter, double *Lo) {
  for (int i = 0; i < 64; ++i) Lo[i] = 0.0;
  for (int jc = 0; jc < 8; ++jc) {
    double d = A[jc * 8 + jc] + jitter;
    for (int k = 0; k < jc; ++k) d -= Lo[jc * 8 + k] * Lo[jc * 8 + k];
    if (!(d > 0.0)) return false;
    double l = sqrt(d);
    Lo[jc * 8 + jc] = l;
    for (int i = jc + 1; i < 8; ++i) {
      double s = A[i * 8 + jc];
      for (int k = 0; k < jc; ++k) s -= Lo[i * 8 + k] * Lo[jc * 8 + k];
      Lo[i * 8 + jc] = s / l;
    }
  }
  return true;
}

// Iteration-0 distribution and draw: one workgroup per request.
__global__ void __launch_bounds__(kSelBlock) init_kernel(SelArgs A, MethodParams P) {
  const int slot = A.slots[blockIdx.x];
  ReqDesc &D = A.desc[slot];
  DistState &Sd = A.dist[slot];
  __shared__ int s_ok;
  if (D.init_mode == kInitForced) return;
  if (threadIdx.x == 0) {
    double *mu = Sd.mu, *sg = Sd.sigma;
    if (D.init_mode == kInitStructured) {
      // exact moments of the structured sampler
      double mc = (P.lane_c[0] + P.lane_c[1] + P.lane_c[2]) / 3.0;
      double vc = 0.0;
      for (int i = 0; i < 3; ++i) vc += (P.lane_c[i] - mc) * (P.lane_c[i] - mc);
      vc /= 3.0;
      double vm = 0.5 * (P.vd_lo + P.vd_hi);
      double vv = (P.vd_hi - P.vd_lo) * (P.vd_hi - P.vd_lo) / 12.0;
      for (int i = 0; i < 64; ++i) sg[i] = 0.0;
      for (int a = 0; a < 4; ++a) {
        mu[a] = mc;
        mu[4 + a] = vm;
        for (int b = 0; b < 4; ++b) sg[a * 8 + b] = vc + (a == b ? P.lane_sigma * P.lane_sigma : 0.0);
        sg[(4 + a) * 8 + 4 + a] = vv;
      }
      s_ok = 1;
    } else {
      const double *m0 = D.mu0, *s0 = D.sigma0;
      if (D.init_mode == kInitSession) {
        m0 = A.sess + (size_t)D.session * 72;
        s0 = m0 + 8;
      }
      for (int a = 0; a < 8; ++a) mu[a] = m0[a];
      for (int i = 0; i < 64; ++i) sg[i] = s0[i];
      s_ok = chol8(sg, P.cov_jitter, Sd.chol) ? 1 : 0;
    }
    ResultRec &R = A.result[slot];
    R.status = s_ok ? 0 : PLAN_E_INVALID;
    R.iterations = 0;
  }
  __syncthreads();
  if (!s_ok) return;
  const bool structured = D.init_mode == kInitStructured;
  for (int j = threadIdx.x; j < D.N; j += kSelBlock)
    draw_sample(P, D, Sd, j, D.first_iter, structured, A.p + ((size_t)slot * A.max_N + j) * 8);
}

// ---------------------------------------------------------------------------
// Selection and update.

__device__ __forceinline__ uint32_t order_key(float f) {
  uint32_t b = __float_as_uint(f);
  if (f != f) return 0xFFFFFFFFu;  // NaN sorts last
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ void bitonic_sort(uint64_t *s, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = threadIdx.x; i < n; i += kSelBlock) {
        int ixj = i ^ jj;
        if (ixj > i) {
          uint64_t a = s[i], b = s[ixj];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int pow2ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

__global__ void __launch_bounds__(kSelBlock) select_update_kernel(SelArgs A, MethodParams P, int l) {
  __shared__ uint64_t s_key[PLAN_MAX_N];
  __shared__ double s_w[kMaxCes];
  __shared__ double s_mu[8];
  __shared__ double s_sum;
  const int slot = A.slots[blockIdx.x];
  const ReqDesc &D = A.desc[slot];
  DistState &Sd = A.dist[slot];
  ResultRec &R = A.result[slot];
  if (R.status != 0) return;
  const int N = D.N, n = D.n_ces, q = D.n_es;
  const size_t base = (size_t)slot * A.max_N;
  const float *r = A.resid + base, *cu = A.cost + base;
  const float *p = A.p + base * 8;
  const bool last = (l == P.L - 1);

  // ConstraintEliteSet: the n smallest (r_j, j).
  const int P1 = pow2ceil(N);
  for (int i = threadIdx.x; i < P1; i += kSelBlock)
    s_key[i] = i < N ? ((uint64_t)order_key(r[i]) << 32) | (uint32_t)i : ~0ull;
  __syncthreads();
  bitonic_sort(s_key, P1);
  // EliteSet: the q smallest (c_u + r, j) over the ConstraintEliteSet.
  const int P2 = pow2ceil(n);
  uint64_t k2[4];
  int cnt = 0;
  for (int i = threadIdx.x; i < P2; i += kSelBlock, ++cnt) {
    if (i < n) {
      uint32_t idx = (uint32_t)(s_key[i] & 0xFFFFFFFFu);
      if (A.tr_ces) A.tr_ces[((size_t)slot * P.L + l) * A.max_ces + i] = (int32_t)idx;
      float c = cu[idx] + r[idx];
      k2[cnt] = ((uint64_t)order_key(c) << 32) | idx;
    } else {
      k2[cnt] = ~0ull;
    }
  }
  __syncthreads();
  cnt = 0;
  for (int i = threadIdx.x; i < P2; i += kSelBlock, ++cnt) s_key[i] = k2[cnt];
  __syncthreads();
  bitonic_sort(s_key, P2);

  // Weights s_j = exp(-(c_j - c_min) / gamma) over the EliteSet (FP64).
  const uint32_t i0 = (uint32_t)(s_key[0] & 0xFFFFFFFFu);
  const double cmin = (double)(cu[i0] + r[i0]);
  for (int i = threadIdx.x; i < q; i += kSelBlock) {
    uint32_t idx = (uint32_t)(s_key[i] & 0xFFFFFFFFu);
    double c = (double)(cu[idx] + r[idx]);
    s_w[i] = exp(-(c - cmin) / P.gamma);
    if (A.tr_es) A.tr_es[((size_t)slot * P.L + l) * A.max_es + i] = (int32_t)idx;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int a = threadIdx.x;
    double m = 0.0, ssum = 0.0;
    for (int i = 0; i < q; ++i) {
      uint32_t idx = (uint32_t)(s_key[i] & 0xFFFFFFFFu);
      m += s_w[i] * (double)p[(size_t)idx * 8 + a];
      ssum += s_w[i];
    }
    s_mu[a] = (1.0 - P.eta) * Sd.mu[a] + P.eta * m / ssum;
    if (a == 0) s_sum = ssum;
  }
  __syncthreads();
  double snew = 0.0;
  if (threadIdx.x < 64) {
    const int a = threadIdx.x >> 3, b = threadIdx.x & 7;
    double c = 0.0;
    for (int i = 0; i < q; ++i) {
      uint32_t idx = (uint32_t)(s_key[i] & 0xFFFFFFFFu);
      c += s_w[i] * ((double)p[(size_t)idx * 8 + a] - s_mu[a]) * ((double)p[(size_t)idx * 8 + b] - s_mu[b]);
    }
    snew = (1.0 - P.eta) * Sd.sigma[a * 8 + b] + P.eta * c / s_sum;
  }
  __syncthreads();
  if (threadIdx.x < 64) Sd.sigma[threadIdx.x] = snew;
  if (threadIdx.x < 8) Sd.mu[threadIdx.x] = s_mu[threadIdx.x];
  __syncthreads();
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    double sym[64];
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) sym[a * 8 + b] = 0.5 * (Sd.sigma[a * 8 + b] + Sd.sigma[b * 8 + a]);
    for (int i = 0; i < 64; ++i) Sd.sigma[i] = sym[i];
    s_ok = chol8(sym, P.cov_jitter, Sd.chol) ? 1 : 0;
    if (A.tr_mu) {
      for (int a = 0; a < 8; ++a) A.tr_mu[((size_t)slot * P.L + l) * 8 + a] = Sd.mu[a];
      for (int i = 0; i < 64; ++i) A.tr_sigma[((size_t)slot * P.L + l) * 64 + i] = sym[i];
    }
    R.iterations = l + 1;
    if (last) {
      // Return: lowest c_u + r in the final EliteSet.
      const uint32_t b = i0;
      R.best = (int32_t)b;
      for (int a = 0; a < 8; ++a) R.p[a] = (double)p[(size_t)b * 8 + a];
      const float *zb = A.zs + (base + b) * kZ;
      const double n10 = 10.0, tf = P.t_f;
      const double x0 = D.ego[0], y0 = D.ego[1], vx0 = D.ego[2], vy0 = D.ego[3];
      const double ax0 = D.ego[4], ay0 = D.ego[5];
      R.xi[0] = x0;
      R.xi[1] = x0 + vx0 * tf / n10;
      R.xi[2] = x0 + 2.0 * vx0 * tf / n10 + ax0 * tf * tf / (n10 * (n10 - 1.0));
      for (int c = 0; c < 8; ++c) R.xi[3 + c] = (double)zb[c] + x0 + vx0 * tf * (double)(3 + c) / n10;
      R.xi[11] = y0;
      R.xi[12] = y0 + vy0 * tf / n10;
      R.xi[13] = y0 + 2.0 * vy0 * tf / n10 + ay0 * tf * tf / (n10 * (n10 - 1.0));
      for (int c = 0; c < 6; ++c) R.xi[14 + c] = (double)zb[8 + c];
      R.xi[20] = R.xi[21] = (double)zb[14];
      R.cost_upper = (double)cu[b];
      R.residual = (double)r[b];
      R.flags = (r[b] > 0.f) ? PLAN_F_INFEASIBLE : 0u;
      if (D.init_mode == kInitSession || D.init_mode == kInitGiven) R.flags |= PLAN_F_WARM;
      if (D.session_wb >= 0) {
        double *st = A.sess + (size_t)D.session_wb * 72;
        for (int a = 0; a < 8; ++a) st[a] = Sd.mu[a];
        for (int i = 0; i < 64; ++i) st[8 + i] = sym[i];
      }
    }
    if (!s_ok) R.status = PLAN_E_INVALID;
  }
  // Trace of this iteration's samples, residuals and costs.
  if (A.tr_p) {
    const size_t tb = ((size_t)slot * P.L + l) * A.max_N;
    for (int i = threadIdx.x; i < N; i += kSelBlock) {
      for (int a = 0; a < 8; ++a) A.tr_p[(tb + i) * 8 + a] = p[(size_t)i * 8 + a];
      A.tr_r[tb + i] = r[i];
      A.tr_c[tb + i] = cu[i];
    }
  }
  __syncthreads();
  if (last || !s_ok) return;
  // Draw the samples of iteration l + 1 from N(mu, Sigma).
  float *pw = A.p + base * 8;
  for (int j = threadIdx.x; j < N; j += kSelBlock)
    draw_sample(P, D, Sd, j, D.first_iter + l + 1, false, pw + (size_t)j * 8);
}

}  // namespace plan

// Launch wrappers (C++ linkage, used by the engine).
namespace plan {
hipError_t launch_lower(const LowerArgs &a, const MethodParams &p, int nblocks, size_t lds,
                        hipStream_t st) {
  hipLaunchKernelGGL(lower_kernel, dim3(nblocks), dim3(kBlock), lds, st, a, p);
  return hipGetLastError();
}
hipError_t launch_init(const SelArgs &a, const MethodParams &p, int nreq, hipStream_t st) {
  hipLaunchKernelGGL(init_kernel, dim3(nreq), dim3(kSelBlock), 0, st, a, p);
  return hipGetLastError();
}
hipError_t launch_select(const SelArgs &a, const MethodParams &p, int nreq, int l, hipStream_t st) {
  hipLaunchKernelGGL(select_update_kernel, dim3(nreq), dim3(kSelBlock), 0, st, a, p, l);
  return hipGetLastError();
}
}  // namespace plan
