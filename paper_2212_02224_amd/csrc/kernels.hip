// kernels.hip -- CDNA4 (gfx950) kernels of the batched bi-level planner.
//
//   lower_kernel          for every sample of every resident request: the draw
//                         p_j ~ N(mu, Sigma) of Alg. 1 (Philox4x32-10 +
//                         Box-Muller), the Step-1 QP through its precomputed
//                         affine map (Sec. III-C, eq. over_3), K iterations of
//                         Alg. 2, then r_j and c_u,j.
//   select_update_kernel  ConstraintEliteSet / EliteSet (Alg. 1) by radix
//                         selection or rank counting, the update of eqs. mean_update,
//                         cov_update, s_formula (FP64) and the Cholesky factor
//                         used by the next draw.
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
// Layout: a workgroup of 4 waves serves samples of one request; each sample
// takes ceil(T/(64 IPL)) waves, IPL horizon instants per lane. The neighbours' positions
// at every instant are staged in LDS once per workgroup. The 15 sums over
// time of N^T g are formed by a transpose-reduction across the wave (17
// shuffles), the small A^-1 product by broadcasting through scalar
// registers.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_internal.h"
#include "rng.h"
#include "traj64.h"

namespace plan {

// ---------------------------------------------------------------------------
// Fast scalar helpers (hardware rcp / rsq / sqrt, ~1 ulp).
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ float bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ uint32_t bcastu(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

// Cross-lane moves of gfx950: v_permlane32_swap exchanges the upper 32 lanes
// of a with the lower 32 lanes of b; v_permlane16_swap exchanges rows 1 and 3
// of a with rows 0 and 2 of b (a row is 16 lanes). DPP row_mirror reads lane
// 15 - i of the row, row_half_mirror lane 7 - i of the half row, quad_perm
// permutes within groups of 4.
__device__ __forceinline__ void swap32(float &a, float &b) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float &a, float &b) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141;
constexpr int kDppRowRor8 = 0x128;  // row_ror:8, lane i reads lane i ^ 8 of its row
constexpr int kDppQuadSwap2 = 0x4e;  // quad_perm [2,3,0,1]
constexpr int kDppQuadSwap1 = 0xb1;  // quad_perm [1,0,3,2]

__device__ __forceinline__ float wave_sum(float v) {
  float a = v, b = v;
  swap32(a, b);  // a + b = own + (lane ^ 32)
  v = a + b;
  a = v;
  b = v;
  swap16(a, b);  // + (lane ^ 16)
  v = a + b;
  v += dpp<kDppRowMirror>(v);
  v += dpp<kDppRowHalfMirror>(v);
  v += dpp<kDppQuadSwap2>(v);
  v += dpp<kDppQuadSwap1>(v);
  return v;
}

// Sum over the 64 lanes of 16 per-lane values; every lane l returns value
// l >> 2. Each step halves the values a lane holds by pairing it with a lane
// that differs in one more index bit (lane bits 5, 4, 3, 2), then the last
// two steps finish the sum inside groups of 4 lanes.
__device__ __forceinline__ float reduce16(const float (&v)[16], int lane) {
  float a[8], b[4], c[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float x = v[i], y = v[i + 8];
    swap32(x, y);  // lanes < 32: (v[i], partner v[i]); lanes >= 32: (partner v[i+8], v[i+8])
    a[i] = x + y;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float x = a[i], y = a[i + 4];
    swap16(x, y);
    b[i] = x + y;
  }
  const bool h3 = lane & 8, h2 = lane & 4;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    float keep = h3 ? b[i + 2] : b[i];
    float send = h3 ? b[i] : b[i + 2];
    c[i] = keep + dpp<kDppRowMirror>(send);  // partner 15 - i: other bit 3, same row
  }
  float keep = h2 ? c[1] : c[0];
  float send = h2 ? c[0] : c[1];
  float d = keep + dpp<kDppRowHalfMirror>(send);  // partner 7 - i: other bit 2, same bit 3
  d += dpp<kDppQuadSwap2>(d);
  d += dpp<kDppQuadSwap1>(d);
  return d;
}

// ---------------------------------------------------------------------------
// Random numbers: rng.h (Philox4x32-10 and Box-Muller).

// Lower Cholesky factor of A + jitter I (8x8, FP64). Returns false if not
// positive definite.
__device__ bool chol8(const double *A, double jitter, double *Lo) {
  for (int i = 0; i < 64; ++i) Lo[i] = 0.0;
  for (int jc = 0; jc < 8; ++jc) {
    double d = A[jc * 8 + jc] + jitter;
    for (int k = 0; k < jc; ++k) d -= Lo[jc * 8 + k] * Lo[jc * 8 + k];
    if (!(d > 0.0)) return false;
    const double l = sqrt(d), il = 1.0 / l;
    Lo[jc * 8 + jc] = l;
    for (int i = jc + 1; i < 8; ++i) {
      double s = A[i * 8 + jc];
      for (int k = 0; k < jc; ++k) s -= Lo[i * 8 + k] * Lo[jc * 8 + k];
      Lo[i * 8 + jc] = s * il;
    }
  }
  return true;
}

// Exact moments of the structured initial sampler (the fixed grid
// discretises the same distribution and uses them too).
__device__ void structured_moments(const MethodParams &P, double *mu, double *sg) {
  double mc = (P.lane_c[0] + P.lane_c[1] + P.lane_c[2]) / 3.0;
  double vc = 0.0;
  for (int i = 0; i < 3; ++i) vc += (P.lane_c[i] - mc) * (P.lane_c[i] - mc);
  vc /= 3.0;
  double vm = 0.5 * (P.vd_lo + P.vd_hi);
  double vv = (P.vd_hi - P.vd_lo) * (P.vd_hi - P.vd_lo) / 12.0;
  for (int i = 0; i < 64; ++i) sg[i] = 0.0;
  if (P.behaviour == PLAN_BEHAV_GOALS) {
    for (int a = 0; a < 8; ++a) mu[a] = 0.0;
    mu[0] = P.t_f * vm;
    sg[0] = P.t_f * P.t_f * vv;
    mu[1] = mc;
    sg[9] = vc + P.lane_sigma * P.lane_sigma;
    return;
  }
  for (int a = 0; a < 4; ++a) {
    mu[a] = mc;
    mu[4 + a] = vm;
    for (int b = 0; b < 4; ++b) sg[a * 8 + b] = vc + (a == b ? P.lane_sigma * P.lane_sigma : 0.0);
    sg[(4 + a) * 8 + 4 + a] = vv;
  }
}

// Behavioural inputs of sample j (of N) from its normals z, the words wb1 of
// Philox block 1 and the lane word sel: the structured initial sampler, the
// fixed grid, or N(mu, chol chol^T); with goal positions only p[0] (x_f - x0)
// and p[1] (y_f) are drawn and the other slots are 0.
__device__ __forceinline__ void finish_draw(const MethodParams &P, bool structured, int j, int N, uint32_t sel,
                                            const float (&z)[8], const uint32_t (&wb1)[4], const double *mu,
                                            const double *chol, float (&p)[8]) {
  const bool goals = P.behaviour == PLAN_BEHAV_GOALS;
#pragma unroll
  for (int a = 0; a < 8; ++a) p[a] = 0.f;
  if (structured && P.sampler == PLAN_SAMPLER_GRID) {
    const int nb = (N + 2) / 3;
    const double lane = P.lane_c[j % 3];
    const double v = P.vd_lo + (P.vd_hi - P.vd_lo) * ((double)(j / 3) + 0.5) / (double)nb;
    if (goals) {
      p[0] = (float)(P.t_f * v);
      p[1] = (float)lane;
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        p[m] = (float)lane;
        p[4 + m] = (float)v;
      }
    }
  } else if (structured) {
    const int ln = (int)(((uint64_t)sel * 3u) >> 32);
    const double lc = P.lane_c[ln];
    if (goals) {
      const double u = (double)((wb1[0] >> 8) + 1u) * (1.0 / 16777216.0);
      p[0] = (float)(P.t_f * (P.vd_lo + (P.vd_hi - P.vd_lo) * u));
      p[1] = (float)(lc + P.lane_sigma * (double)z[0]);
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        p[m] = (float)(lc + P.lane_sigma * (double)z[m]);
        const double u = (double)((wb1[m] >> 8) + 1u) * (1.0 / 16777216.0);
        p[4 + m] = (float)(P.vd_lo + (P.vd_hi - P.vd_lo) * u);
      }
    }
  } else {
    const int nd = goals ? 2 : 8;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a >= nd) continue;
      double s = mu[a];
#pragma unroll
      for (int b = 0; b <= a; ++b) s += chol[a * 8 + b] * (double)z[b];
      p[a] = (float)s;
    }
  }
}

// Sample j of upper iteration l, drawn by one wave: lanes 0-2 each run one
// Philox block, lanes 0-3 one Box-Muller pair; the eight values are returned
// uniform across the wave. mu/chol point to LDS (Gaussian draws only).
__device__ void wave_draw(const MethodParams &P, uint64_t seed, int j, int N, int l, bool structured,
                          const double *mu, const double *chol, int lane, float (&p)[8]) {
  uint32_t w[4];
  rng_block(seed, j, l, lane < 3 ? lane : 2, w);
  // Box-Muller pair m (lane m < 4) uses words 2(m & 1), 2(m & 1) + 1 of block m >> 1.
  const int src = (lane & 3) >> 1;
  uint32_t w0 = __shfl(w[0], src, 64), w1 = __shfl(w[1], src, 64);
  uint32_t w2 = __shfl(w[2], src, 64), w3 = __shfl(w[3], src, 64);
  const bool odd = lane & 1;
  float n0, n1;
  normals2(odd ? w2 : w0, odd ? w3 : w1, n0, n1);
  float z[8];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    z[2 * m] = bcast(n0, m);
    z[2 * m + 1] = bcast(n1, m);
  }
  uint32_t wb1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) wb1[m] = bcastu(w[m], 1);
  finish_draw(P, structured, j, N, bcastu(w[0], 2), z, wb1, mu, chol, p);
}

// ---------------------------------------------------------------------------
// Lower level.

struct Lane {
  // basis rows of this lane's instant (free columns)
  float bx[8], bdx[8], bddx[8];
  float by7, bdy7, bddy7;
  // fixed part of the trajectory (relative x frame, without vx0)
  float xf, xdf, xddf, yf, ydf, yddf;
};

struct Scal {
  float vx0, rho, ia, ib, ell_a, ell_b;
  float v_min, v_max, a_max, kmax, inv_kmax, c_max, kappa_abs, y_lb, y_ub, v_eps;
  int n_road;                    // knots of the road profile (0: constant road)
  float road_x0, road_idx, dt;   // first knot from x0, 1 / knot spacing, t_f / (T - 1)
};

// Road at one instant (Table ineq_list: the centripetal row's kappa(x(t)) and
// the lane limits y_lb(x(t)), y_ub(x(t))).
struct RoadAt {
  float kappa_abs, y_lb, y_ub;
};

// The request's road profile (knots in LDS as (kappa, y_lb, y_ub, 0)) at the
// trajectory's position x_rel + vx0 t_k from x0 (x_rel in the frame relative
// to x0 + vx0 t), linear between knots and constant beyond; the constant road
// without a profile. ROAD = false: launches whose requests have no profile
// (the lookup compiles away).
template <bool ROAD>
__device__ __forceinline__ RoadAt road_at(const Scal &S, const float4 *__restrict__ road, float x_rel, int t) {
  RoadAt r;
  if (!ROAD || S.n_road == 0) {
    r.kappa_abs = S.kappa_abs;
    r.y_lb = S.y_lb;
    r.y_ub = S.y_ub;
    return r;
  }
  const float xe = fmaf(S.vx0, (float)t * S.dt, x_rel);
  const float u = fminf(fmaxf((xe - S.road_x0) * S.road_idx, 0.f), (float)(S.n_road - 1));
  const int i = min((int)u, max(S.n_road - 2, 0));
  const float f = S.n_road > 1 ? u - (float)i : 0.f;
  const float4 a = road[i], b = road[S.n_road > 1 ? i + 1 : i];
  r.kappa_abs = fabsf(fmaf(f, b.x - a.x, a.x));
  r.y_lb = fmaf(f, b.y - a.y, a.y);
  r.y_ub = fmaf(f, b.z - a.z, a.z);
  return r;
}

// reduce16's sums, bit for bit, through LDS. Before its two quad steps,
// reduce16 leaves lane l (p = l & 15) the sum of value l >> 2 over lanes
// q + {0, 32, 16, 48} for q = p, p ^ 15, p ^ 7, p ^ 8, as the balanced tree
// ((G(p) + G(p^15)) + (G(p^7) + G(p^8))), G(q) = (v_q + v_q+32) + (v_q+16 +
// v_q+48). Here value k of lane s goes to s_w[64 k + 4 (s & 15) + (s >> 4)]
// (this wave's 16 x 64 floats), so the four values of G(q) are one 16-byte
// read; lane l adds the same 16 values in the same tree and finishes with
// the same quad steps: 17 vector instructions against 35. The writes of one
// value and the 16-byte reads each touch 64 distinct banks. The wave's own
// LDS operations run in order, so the reads see the writes, and a later
// call's writes follow this call's reads.
constexpr int kRedFloats = 16 * 64;  // per wave
__device__ __forceinline__ float reduce16_lds(const float (&v)[16], int lane, float *s_w) {
  float *col = s_w + 4 * (lane & 15) + (lane >> 4);
#pragma unroll
  for (int k = 0; k < 16; ++k) col[64 * k] = v[k];
  __builtin_amdgcn_wave_barrier();
  const int p = lane & 15;
  const float4 *row = reinterpret_cast<const float4 *>(s_w + 64 * (lane >> 2));
  auto grp = [&](int q) -> float {
    const float4 x = row[q];
    return (x.x + x.z) + (x.y + x.w);
  };
  float d = (grp(p) + grp(p ^ 15)) + (grp(p ^ 7) + grp(p ^ 8));
  __builtin_amdgcn_wave_barrier();
  d += dpp<kDppQuadSwap2>(d);
  d += dpp<kDppQuadSwap1>(d);
  return d;
}

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

// Neighbour corrections at one instant, in ellipse-scaled units:
// sum_i (max(1, 1/r_i) - 1) (dx_i / a, dy_i / b), r_i the normalised
// distance (closed form of step split_alpha_o with the clip of clip_d_o);
// at the centre (r = 0) alpha = 0 and d = 1 give (1, 0). The table holds two
// neighbours per float4 entry, pre-divided by (a, b); loads run one entry
// ahead of the arithmetic, and the distance tests of an entry are formed
// before the (rarely taken) near branches.
__device__ __forceinline__ void near_update(float q, float dx, float dy, float &ax, float &ay) {
  if (q < 1.f) {
    const float f = (q > 0.f ? frsq(q) : 1.f) - 1.f;
    ax = fmaf(f, dx, ax + (q > 0.f ? 0.f : 1.f));
    ay = fmaf(f, dy, ay);
  }
}

// One entry (two neighbours) at one instant. GATE: the distance tests run
// only when some lane of the wave is within one ellipse unit of either
// neighbour along x. |dx| >= 1 gives dx^2 >= 1 in FP32 and so q >= 1 (no
// update), hence the gate changes no result. On the headline's scenes about
// 90% of (wave, neighbour) pairs fail it, so the common case costs two
// subtractions and two compares; it pays where a lane carries two instants
// (measured -10% at M = 20) and in the FP32 matrix-core form (-7%), not with
// one instant per lane (within +-2%) or in the FP16 split (much slower), where
// the launches leave it out.
// `live`: the lanes whose instant is inside the horizon (the others take no
// part in the gate).
template <bool GATE>
__device__ __forceinline__ void pair_update(float xs, float ys, const float4 &o, uint64_t live, float &ax,
                                            float &ay) {
  const float dx0 = xs - o.x, dx1 = xs - o.z;
  if (!GATE || (__builtin_amdgcn_ballot_w64(fminf(fabsf(dx0), fabsf(dx1)) < 1.f) & live) != 0) {
    const float dy0 = ys - o.y, dy1 = ys - o.w;
    const float q0 = fmaf(dx0, dx0, dy0 * dy0), q1 = fmaf(dx1, dx1, dy1 * dy1);
    near_update(q0, dx0, dy0, ax, ay);
    near_update(q1, dx1, dy1, ax, ay);
  }
}

// Neighbour sums of one lane's instant t (the matrix-core kernels): the
// entries of pairs c and c + 1 in alternating registers. GATE skips a pair
// as pair_update does; every matrix-core launch takes it (at the headline
// shape: FP32 form 91.2 -> 85.1 ms, FP16 split 77.7 -> 73.3 ms).
template <bool GATE>
__device__ __forceinline__ void neighbour_pass(const float4 *__restrict__ obs, int npair, int T, int t,
                                               float xs, float ys, uint64_t live, float &ax, float &ay) {
  ax = 0.f;
  ay = 0.f;
  if (npair == 0) return;
  const float4 *p = obs + t;
  float4 a = p[0], b;
  int c = 0;
  for (; c + 1 < npair; c += 2) {
    b = p[(c + 1) * T];
    pair_update<GATE>(xs, ys, a, live, ax, ay);
    a = p[(c + 2 < npair ? c + 2 : c + 1) * T];
    pair_update<GATE>(xs, ys, b, live, ax, ay);
  }
  if (c < npair) pair_update<GATE>(xs, ys, a, live, ax, ay);
}

// Differences between the targets of one (alpha, d) step and the current
// trajectory at one instant: x axis (obstacles, velocity, acceleration) and
// y axis (obstacles plus the lane bounds, velocity, acceleration).
struct Corr {
  float dox, dvx, dax, wy, dvy, day;
};

// Steps split_alpha_o .. update_slack of Alg. 2 at one instant, from the
// trajectory state s there and the neighbour sums (ax, ay) of
// neighbour_pass. da_prev carries d_a of the previous step. All differences
// are zero where tv is false.
__device__ __forceinline__ Corr targets_from(const State6 &s, const Scal &S, const RoadAt &rd, float ax, float ay,
                                             bool tv, float &da_prev) {
  float dox = ax * S.ell_a, doy = ay * S.ell_b;
  // velocity / acceleration polar variables and their clips
  const float v2 = fmaf(s.xd, s.xd, s.yd * s.yd);
  const float a2 = fmaf(s.xdd, s.xdd, s.ydd * s.ydd);
  const bool vz = !(v2 > 0.f), az = !(a2 > 0.f);
  const float rv = vz ? 0.f : frsq(v2);
  const float ra = az ? 0.f : frsq(a2);
  const float vn = v2 * rv, an = a2 * ra;
  // |sin(alpha_a - alpha_v)|: cross product of the unit vectors (atan2(0, 0)
  // = 0 maps a zero vector to (1, 0))
  const float ex = vz ? 1.f : s.xd, rv1 = vz ? 1.f : rv;
  const float fx = az ? 1.f : s.xdd, ra1 = az ? 1.f : ra;
  const float sig = fabsf(fmaf(s.ydd, ex, -fx * s.yd)) * (rv1 * ra1);
  const float vlo = fmaxf(S.v_min, fsqrt(da_prev * sig * S.inv_kmax));
  float vhi = S.v_max;
  if (rd.kappa_abs > 0.f) {
    const float cv = ex * rv1;
    const float den = rd.kappa_abs * cv * cv;
    if (den > 0.f) vhi = fminf(vhi, fsqrt(S.c_max * frcp(den)));
  }
  const float dv = fminf(fmaxf(vn, vlo), vhi);
  const float ahi = sig > 0.f ? fminf(S.a_max, dv * dv * S.kmax * frcp(sig)) : S.a_max;
  const float dan = fminf(an, ahi);
  const float kv = (dv - vn) * rv, ka = (dan - an) * ra;
  Corr c;
  c.dvx = vz ? dv : kv * s.xd;
  c.dvy = kv * s.yd;
  c.dax = az ? dan : ka * s.xdd;
  c.day = ka * s.ydd;
  if (tv) da_prev = dan;
  // lane bounds: e - s - G xi = clip(y, y_lb, y_ub) - y
  c.wy = doy + (fminf(fmaxf(s.y, rd.y_lb), rd.y_ub) - s.y);
  c.dox = dox;
  if (!tv) c.dox = c.wy = c.dvx = c.dvy = c.dax = c.day = 0.f;
  return c;
}

template <bool ROAD, bool GATE>
__device__ __forceinline__ Corr targets_at(const State6 &s, const Scal &S, const float4 *__restrict__ obs,
                                           const float4 *__restrict__ road, int npair, int T, int t, bool tv,
                                           float &da_prev) {
  float ax, ay;
  neighbour_pass<GATE>(obs, npair, T, t, s.x * S.ia, s.y * S.ib, __builtin_amdgcn_ballot_w64(tv), ax, ay);
  return targets_from(s, S, road_at<ROAD>(S, road, s.x, t), ax, ay, tv, da_prev);
}

// One target pass over this lane's IPL instants (slots): the trajectory at
// each, the neighbour sums of all slots in one loop over the neighbour pairs
// (the slots' dependency chains interleave), then the targets of each slot.
// t0: slot 0's instant, unclamped.
template <int IPL, bool ROAD>
__device__ __forceinline__ void target_pass(const Lane (&L)[IPL], const Scal &S, const float (&zs)[15],
                                            const float4 *__restrict__ obs, const float4 *__restrict__ road,
                                            int npair, int T, int t0, const int (&tt)[IPL], const bool (&tv)[IPL],
                                            float (&da_prev)[IPL], Corr (&cr)[IPL]) {
  State6 st[IPL];
  float xs[IPL], ys[IPL], ax[IPL], ay[IPL];
#pragma unroll
  for (int u = 0; u < IPL; ++u) {
    st[u] = eval_traj(L[u], zs, S.vx0);
    xs[u] = st[u].x * S.ia;
    ys[u] = st[u].y * S.ib;
    ax[u] = 0.f;
    ay[u] = 0.f;
  }
  if (IPL == 1 && npair > 0) {
    // one entry ahead (the update is branch-free here, and a small launch
    // is bound by its latency)
    float4 cur = obs[tt[0]];
    for (int c = 0; c < npair; ++c) {
      const float4 nxt = obs[(c + 1 < npair ? c + 1 : c) * T + tt[0]];
      pair_update<false>(xs[0], ys[0], cur, ~0ull, ax[0], ay[0]);
      cur = nxt;
    }
  } else if (npair > 0) {
    // Entries of pairs c and c + 1 in alternating registers (no copies
    // between steps). Slot u reads instant t0 + 64 u unclamped, an immediate
    // offset from slot 0's address: past the horizon that is another pair's
    // row or the far padding, and such lanes are not live.
    const float4 *base = obs + t0;
    uint64_t live[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) live[u] = __builtin_amdgcn_ballot_w64(tv[u]);
    float4 a[IPL], b[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) a[u] = base[u * kWave];
    int c = 0;
    for (; c + 1 < npair; c += 2) {
      const float4 *pb = base + (c + 1) * T;
#pragma unroll
      for (int u = 0; u < IPL; ++u) b[u] = pb[u * kWave];
#pragma unroll
      for (int u = 0; u < IPL; ++u) pair_update<IPL == 2>(xs[u], ys[u], a[u], live[u], ax[u], ay[u]);
      const float4 *pa = base + (c + 2 < npair ? c + 2 : c + 1) * T;
#pragma unroll
      for (int u = 0; u < IPL; ++u) a[u] = pa[u * kWave];
#pragma unroll
      for (int u = 0; u < IPL; ++u) pair_update<IPL == 2>(xs[u], ys[u], b[u], live[u], ax[u], ay[u]);
    }
    if (c < npair) {
#pragma unroll
      for (int u = 0; u < IPL; ++u) pair_update<IPL == 2>(xs[u], ys[u], a[u], live[u], ax[u], ay[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < IPL; ++u)
    cr[u] = targets_from(st[u], S, road_at<ROAD>(S, road, st[u].x, tt[u]), ax[u], ay[u], tv[u], da_prev[u]);
}

// This lane's share of N^T g at one instant.
__device__ __forceinline__ void g_of(const Lane &L, const Corr &c, float (&g)[16]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) g[k] = fmaf(L.bx[k], c.dox, fmaf(L.bdx[k], c.dvx, L.bddx[k] * c.dax));
#pragma unroll
  for (int k = 0; k < 6; ++k) g[8 + k] = fmaf(L.bx[k], c.wy, fmaf(L.bdx[k], c.dvy, L.bddx[k] * c.day));
  g[14] = fmaf(L.by7, c.wy, fmaf(L.bdy7, c.dvy, L.bddy7 * c.day));
  g[15] = 0.f;
}

// Residual r (sum of max(0, g) over Table ineq_list) and upper cost c_u at
// one instant of the trajectory state s.
template <bool ROAD>
__device__ __forceinline__ void residual_at(const State6 &s, const Scal &S, const float4 *__restrict__ obs,
                                            const float4 *__restrict__ road, int npair, int T, int t, bool tv,
                                            float &res, float &cost) {
  const RoadAt rd = road_at<ROAD>(S, road, s.x, t);
  const float xs = s.x * S.ia, ys = s.y * S.ib;
  float r = 0.f;
  for (int c = 0; c < npair; ++c) {
    const float4 o = obs[c * T + t];
    float dx = xs - o.x, dy = ys - o.y;
    r += fmaxf(0.f, 1.f - fmaf(dx, dx, dy * dy));
    dx = xs - o.z;
    dy = ys - o.w;
    r += fmaxf(0.f, 1.f - fmaf(dx, dx, dy * dy));
  }
  const float vn = fsqrt(fmaf(s.xd, s.xd, s.yd * s.yd));
  const float an = fsqrt(fmaf(s.xdd, s.xdd, s.ydd * s.ydd));
  r += fmaxf(0.f, vn - S.v_max) + fmaxf(0.f, S.v_min - vn) + fmaxf(0.f, an - S.a_max);
  const float vd = fmaxf(vn, S.v_eps);
  const float curv = fabsf(s.ydd * s.xd - s.xdd * s.yd) * frcp(vd * vd * vd);
  r += fmaxf(0.f, curv - S.kmax);
  r += fmaxf(0.f, fabsf(s.xd * s.xd * rd.kappa_abs) - S.c_max);
  r += fmaxf(0.f, s.y - rd.y_ub) + fmaxf(0.f, rd.y_lb - s.y);
  const float e = vn - S.v_max;
  res = tv ? r : 0.f;
  cost = tv ? e * e : 0.f;
}

// Logical workgroup index of dispatched workgroup b out of n. Workgroups go
// round-robin to the 8 XCDs (b % 8), each with its own L2; XCD x takes one
// contiguous range of logical workgroups, so neighbouring samples' residual
// and cost words (4 bytes each, a few samples per workgroup) meet in one L2
// and reach HBM as whole sectors. A bijection for any n.
__device__ __forceinline__ int xcd_logical(int b, int n) {
  const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + i;
}

// Workgroup -> slot: binary search of the logical workgroup index in the
// prefix counts of the launch's active slots (uniform scalar loads). Returns
// the slot and the workgroup's rank within it.
__device__ __forceinline__ int2 block_slot(const LowerArgs &A) {
  int lo = 0, hi = A.n_act - 1;
  const int b = xcd_logical(blockIdx.x, gridDim.x);
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.blk_prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return make_int2(A.act_slots[lo], b - A.blk_prefix[lo]);
}

// Neighbour positions relative to the reference line x0 + vx0 t, divided by
// the ellipse axes, two neighbours per entry [pair][T] (an odd last one is
// paired with a point far away). Constant velocities as in the collision
// row of Table ineq_list. `pad` entries after the last pair hold far points
// (the vector-ALU kernel reads up to kObsPad entries past a pair's row).
__device__ void stage_neighbours(const ReqDesc &D, const MethodParams &P, float4 *s_obs, int pad = 0) {
  const int T = D.T, M = D.M, npair = (M + 1) >> 1;
  if (npair > 0)
    for (int i = threadIdx.x; i < pad; i += blockDim.x) s_obs[npair * T + i] = make_float4(1e18f, 1e18f, 1e18f, 1e18f);
  const double x0 = D.ego[0], vx0 = D.ego[2];
  const double ia = 1.0 / P.ell_a, ib = 1.0 / P.ell_b;
  for (int idx = threadIdx.x; idx < npair * T; idx += blockDim.x) {
    const int c = idx / T, k = idx - c * T;
    const double tk = P.t_f * (double)k / (double)(T - 1);
    float v[4];
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * c + h;
      if (i < M) {
        v[2 * h] = (float)(((D.obs[i][0] - x0) + (D.obs[i][2] - vx0) * tk) * ia);
        v[2 * h + 1] = (float)((D.obs[i][1] + D.obs[i][3] * tk) * ib);
      } else {
        v[2 * h] = 1e18f;
        v[2 * h + 1] = 1e18f;
      }
    }
    s_obs[idx] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Iteration 0 of a request that starts from the initial sampler when that is
// the decoder sampler: its samples are in the rows, written by the decoder.
__device__ __forceinline__ bool decoded_start(const ReqDesc &D, const MethodParams &P, int l) {
  return l == 0 && D.init_mode == kInitStructured && P.sampler == PLAN_SAMPLER_DECODER;
}

// Road profile knots into LDS as (kappa, y_lb, y_ub, 0).
__device__ void stage_road(const ReqDesc &D, float4 *s_road) {
  for (int i = threadIdx.x; i < D.n_road; i += blockDim.x)
    s_road[i] = make_float4((float)D.road[i][0], (float)D.road[i][1], (float)D.road[i][2], 0.f);
}

// Sampling distribution of upper iteration l into LDS (Gaussian draws only):
// the request's or the session's at iteration 0 (factored here), else the
// one the previous update left with its factor. At iteration 0 the first
// workgroup of the request (first) also copies the prior it read into the
// slot's own state, where the update of that iteration reads it: the session
// store is shared, and another request of the same session may write it
// while this request's update runs.
__device__ void load_distribution(const LowerArgs &A, const ReqDesc &D, const MethodParams &P, int slot, int l,
                                  bool first, double *s_mu, double *s_chol) {
  if (l == 0) {
    const double *m0 = D.mu0, *s0 = D.sigma0;
    if (D.init_mode == kInitSession) {
      m0 = A.sess + (size_t)D.session * 72;
      s0 = m0 + 8;
    }
    if (threadIdx.x == 0) {
      for (int a = 0; a < 8; ++a) s_mu[a] = m0[a];
      if (!chol8(s0, P.cov_jitter, s_chol))
        for (int i = 0; i < 64; ++i) s_chol[i] = 0.0;  // reported by the update
    }
    if (first && threadIdx.x < 72) {
      DistState &Sd = A.dist[slot];
      if (threadIdx.x < 8) Sd.mu[threadIdx.x] = m0[threadIdx.x];
      else Sd.sigma[threadIdx.x - 8] = s0[threadIdx.x - 8];
    }
  } else if (threadIdx.x < 72) {
    const DistState &Sd = A.dist[slot];
    if (threadIdx.x < 8) s_mu[threadIdx.x] = Sd.mu[threadIdx.x];
    else s_chol[threadIdx.x - 8] = Sd.chol[threadIdx.x - 8];
  }
}

__device__ __forceinline__ Scal make_scal(const ReqDesc &D, const MethodParams &P) {
  Scal S;
  S.vx0 = (float)D.ego[2];
  S.rho = (float)P.rho;
  S.ia = (float)(1.0 / P.ell_a);
  S.ib = (float)(1.0 / P.ell_b);
  S.ell_a = (float)P.ell_a;
  S.ell_b = (float)P.ell_b;
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
  S.n_road = D.n_road;
  S.road_x0 = (float)(D.road_x0 - D.ego[0]);
  S.road_idx = (float)(1.0 / D.road_dx);
  S.dt = (float)(P.t_f / (double)(D.T - 1));
  return S;
}

// Part of the trajectory at instant tt fixed by the initial conditions
// (eq. boundary_cond_initial: c0, c1, c2 of each axis), x relative to the
// reference line and without vx0.
__device__ __forceinline__ State6 fixed_part(const float *Bt, int Tp, int tt, const ReqDesc &D,
                                             const MethodParams &P) {
  const double y0 = D.ego[1], vy0 = D.ego[3], ax0 = D.ego[4], ay0 = D.ego[5];
  const double n = 10.0, tf = P.t_f;
  // relative x frame: c0 = c1 = 0, c2 = ax0 t_f^2 / (n (n - 1))
  const double cx2 = ax0 * tf * tf / (n * (n - 1.0));
  const double cy0 = y0, cy1 = y0 + vy0 * tf / n;
  const double cy2 = y0 + 2.0 * vy0 * tf / n + ay0 * tf * tf / (n * (n - 1.0));
  const float W0 = Bt[(kColFix + 0) * Tp + tt], W1 = Bt[(kColFix + 1) * Tp + tt], W2 = Bt[(kColFix + 2) * Tp + tt];
  const float Wd0 = Bt[(kColFix + 3) * Tp + tt], Wd1 = Bt[(kColFix + 4) * Tp + tt],
              Wd2 = Bt[(kColFix + 5) * Tp + tt];
  const float Wdd0 = Bt[(kColFix + 6) * Tp + tt], Wdd1 = Bt[(kColFix + 7) * Tp + tt],
              Wdd2 = Bt[(kColFix + 8) * Tp + tt];
  const float fx2 = (float)cx2, fy0 = (float)cy0, fy1 = (float)cy1, fy2 = (float)cy2;
  State6 f;
  f.x = W2 * fx2;
  f.xd = Wd2 * fx2;
  f.xdd = Wdd2 * fx2;
  f.y = fmaf(W0, fy0, fmaf(W1, fy1, W2 * fy2));
  f.yd = fmaf(Wd0, fy0, fmaf(Wd1, fy1, Wd2 * fy2));
  f.ydd = fmaf(Wdd0, fy0, fmaf(Wdd1, fy1, Wdd2 * fy2));
  return f;
}

// Step 1 (eq. over_3 through its affine map): free coefficient v of
// z_bar = S p' + R b', b' = (ax0, y0, vy0, ay0), p' = [y_d, v_d - vx0]
// (set-points) or [x_f - x0 - vx0 t_f, y_f, 0 ...] (goal positions: c10 of x
// in the frame relative to x0 + vx0 t, and c9 = c10 of y).
// Inputs of step1_coef that do not depend on the sample: row v of the two
// step-1 tables and the ego terms (loaded before the sample is drawn).
struct Step1In {
  float s1[8], r1[4], bb[4];
  double vx0;
};
__device__ __forceinline__ Step1In step1_inputs(const float *S1, const ReqDesc &D, int v) {
  Step1In t;
  const float *R1 = S1 + 16 * 8;
#pragma unroll
  for (int m = 0; m < 8; ++m) t.s1[m] = S1[v * 8 + m];
#pragma unroll
  for (int m = 0; m < 4; ++m) t.r1[m] = R1[v * 4 + m];
  t.bb[0] = (float)D.ego[4];
  t.bb[1] = (float)D.ego[1];
  t.bb[2] = (float)D.ego[3];
  t.bb[3] = (float)D.ego[5];
  t.vx0 = D.ego[2];
  return t;
}
__device__ __forceinline__ float step1_coef(const Step1In &t, const MethodParams &P, const float (&pin)[8]) {
  const double vx0 = t.vx0;
  float pp[8];
  if (P.behaviour == PLAN_BEHAV_GOALS) {
#pragma unroll
    for (int m = 0; m < 8; ++m) pp[m] = 0.f;
    pp[0] = (float)((double)pin[0] - vx0 * P.t_f);
    pp[1] = pin[1];
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      pp[m] = pin[m];
      pp[4 + m] = (float)((double)pin[4 + m] - vx0);
    }
  }
  float zb = 0.f;
#pragma unroll
  for (int m = 0; m < 8; ++m) zb = fmaf(t.s1[m], pp[m], zb);
#pragma unroll
  for (int m = 0; m < 4; ++m) zb = fmaf(t.r1[m], t.bb[m], zb);
  return zb;
}

// FP64 coefficients of xi (absolute x) from the free coefficients: lane
// owners write coefficient v of z (and of z_bar); writer_fixed adds c0..c2.
__device__ __forceinline__ void write_xi(const ReqDesc &D, const MethodParams &P, double *xs, double *xb, int v,
                                         float z, float zb, bool writer_fixed) {
  const double x0 = D.ego[0], y0 = D.ego[1], vx0 = D.ego[2], vy0 = D.ego[3];
  const double ax0 = D.ego[4], ay0 = D.ego[5];
  const double n = 10.0, tf = P.t_f;
  if (v < 8) {
    const double ref = x0 + vx0 * tf * (double)(3 + v) / n;
    xs[3 + v] = (double)z + ref;
    xb[3 + v] = (double)zb + ref;
  } else if (v < 14) {
    xs[11 + 3 + (v - 8)] = (double)z;
    xb[11 + 3 + (v - 8)] = (double)zb;
  } else if (v == 14) {
    xs[11 + 9] = xs[11 + 10] = (double)z;
    xb[11 + 9] = xb[11 + 10] = (double)zb;
  }
  if (writer_fixed) {
    const double c0 = x0, c1 = x0 + vx0 * tf / n;
    const double c2 = x0 + 2.0 * vx0 * tf / n + ax0 * tf * tf / (n * (n - 1.0));
    const double e0 = y0, e1 = y0 + vy0 * tf / n;
    const double e2 = y0 + 2.0 * vy0 * tf / n + ay0 * tf * tf / (n * (n - 1.0));
    xs[0] = xb[0] = c0;
    xs[1] = xb[1] = c1;
    xs[2] = xb[2] = c2;
    xs[11] = xb[11] = e0;
    xs[12] = xb[12] = e1;
    xs[13] = xb[13] = e2;
  }
}

// IPL instants per lane: instant (wi IPL + u) 64 + lane in slot u of wave wi
// of a sample; ceil(T / (64 IPL)) waves per sample, 4 / that samples per
// workgroup (wave sl NW + wi is wave wi of sample sl).
struct LowerShape {
  int NW, spb, wave, lane, sl, wi;
};
template <int IPL>
__device__ __forceinline__ LowerShape lower_shape(int T) {
  LowerShape h;
  h.NW = (T + kWave * IPL - 1) / (kWave * IPL);
  h.spb = 4 / h.NW;
  h.wave = threadIdx.x / kWave;
  h.lane = threadIdx.x % kWave;
  h.sl = h.wave / h.NW;
  h.wi = h.wave - h.sl * h.NW;
  return h;
}

// The part of a lower-level workgroup's state that depends on its request
// alone (not on the upper iteration or on which samples it serves): the
// method's scalars, the basis rows of the lane's instants with the fixed part
// of the trajectory, and the lane's row of A^-1 and D.
template <int IPL>
struct LowerSetup {
  Lane L[IPL];
  Scal S;
  float arow[4];  // A^-1[v][4 (lane & 3) + i], v = lane >> 2
  float Dv;
};

// Set-up of a request: its neighbour table (and road profile) into LDS and
// the register part. The LDS tables are ready after the next barrier.
template <int IPL, bool ROAD>
__device__ __forceinline__ void lower_setup(const LowerArgs &A, const MethodParams &P, const ReqDesc &D,
                                            float4 *s_obs, float4 *s_road, LowerSetup<IPL> &U) {
  const LowerShape h = lower_shape<IPL>(D.T);
  const int T = D.T;
  stage_neighbours(D, P, s_obs, kObsPad);
  if constexpr (ROAD) stage_road(D, s_road);
  U.S = make_scal(D, P);
  // Basis rows of this lane's instants and the fixed part of the trajectory.
  const float *Bt = A.basis + D.basis_off;
  const int Tp = D.basis_tpad;
#pragma unroll
  for (int u = 0; u < IPL; ++u) {
    const int t = (h.wi * IPL + u) * kWave + h.lane;
    const int tt = t < T ? t : T - 1;
    Lane &L = U.L[u];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      L.bx[c] = Bt[(kColW + c) * Tp + tt];
      L.bdx[c] = Bt[(kColWd + c) * Tp + tt];
      L.bddx[c] = Bt[(kColWdd + c) * Tp + tt];
    }
    L.by7 = Bt[(kColY7 + 0) * Tp + tt];
    L.bdy7 = Bt[(kColY7 + 1) * Tp + tt];
    L.bddy7 = Bt[(kColY7 + 2) * Tp + tt];
    const State6 f = fixed_part(Bt, Tp, tt, D, P);
    L.xf = f.x;
    L.xdf = f.xd;
    L.xddf = f.xdd;
    L.yf = f.y;
    L.ydf = f.yd;
    L.yddf = f.ydd;
  }
  const int v = h.lane >> 2;
  const float *Pj = A.proj + (size_t)D.tm_idx * kProjFloats;
#pragma unroll
  for (int i = 0; i < 4; ++i) U.arow[i] = Pj[v * 16 + 4 * (h.lane & 3) + i];
  U.Dv = Pj[256 + v];
}

// The samples of workgroup `rank` of the request in `slot` at upper
// iteration l, with the request's set-up in U and LDS: the sample p_j,
// step 1, K projection iterations, residual and upper cost, rows written.
// Every thread of the workgroup calls it (it holds barriers).
// s_gred: 4 x kRedFloats floats for the two-instants-per-lane sums; s_zb: 4 x
// 16 floats for its coefficient broadcasts.
template <int IPL, bool ROAD>
__device__ __forceinline__ void lower_item(const LowerArgs &A, const MethodParams &P, const ReqDesc &D, int slot,
                                           int rank, int l, const LowerSetup<IPL> &U, const float4 *s_obs,
                                           const float4 *s_road, float (*s_red)[4 * IPL][16], double *s_mu,
                                           double *s_chol, float *s_gred, float *s_zb) {
  const LowerShape h = lower_shape<IPL>(D.T);
  const int T = D.T, M = D.M, N = D.N;
  const int npair = (M + 1) >> 1;
  const int NW = h.NW, spb = h.spb, wave = h.wave, lane = h.lane, sl = h.sl, wi = h.wi;
  const int j = rank * spb + sl;
  const bool active = (sl < spb) && (j < N);
  int tt[IPL];
  bool tv[IPL];
#pragma unroll
  for (int u = 0; u < IPL; ++u) {
    const int t = (wi * IPL + u) * kWave + lane;
    tv[u] = active && t < T;
    tt[u] = t < T ? t : T - 1;
  }
  const size_t slot_off = (size_t)D.row_off;
  const Scal &S = U.S;
  const Lane(&L)[IPL] = U.L;

  // samples in the rows already: the caller's, or the decoder sampler's
  const bool forced = D.init_mode == kInitForced || decoded_start(D, P, l);
  const bool structured = !forced && l == 0 && D.init_mode == kInitStructured;
  if (!forced && !structured) load_distribution(A, D, P, slot, l, rank == 0, s_mu, s_chol);
  const int v = lane >> 2;
  const float Dv = U.Dv;
  const uint64_t seed = D.seed;
  const int draw_iter = D.first_iter + l;
  __syncthreads();  // neighbour table and distribution ready

  // Sample p_j (Alg. 1: draw from N(mu, Sigma); iteration 0 may use the
  // structured initial sampler), or the caller's samples.
  float pin[8];
  if (forced) {
#pragma unroll
    for (int m = 0; m < 8; ++m) pin[m] = active ? A.p[(slot_off + j) * 8 + m] : 0.f;
  } else {
    wave_draw(P, seed, j, N, draw_iter, structured, s_mu, s_chol, lane, pin);
  }
  // the step-1 rows are read before the sample is stored, so that store
  // cannot hold their loads back
  const float zb = step1_coef(step1_inputs(A.step1 + (size_t)D.t_idx * kStep1Floats, D, v), P, pin);
  if (!forced && active && wi == 0 && lane == 0) {
    float4 *dst = reinterpret_cast<float4 *>(A.p + (slot_off + j) * 8);
    dst[0] = make_float4(pin[0], pin[1], pin[2], pin[3]);
    dst[1] = make_float4(pin[4], pin[5], pin[6], pin[7]);
  }
  float z = zb, mu = 0.f;
  float zs[15];
  // Every lane's copy of the 15 coefficients (lane 4 c holds coefficient c):
  // v_readlane to scalar registers, or with two instants per lane through
  // this wave's 16 words of LDS (one write, four 16-byte broadcast reads, no
  // vector instructions; the wave's LDS operations run in order).
  auto broadcast_z = [&]() {
    if constexpr (IPL == 2) {
      float *w = s_zb + 16 * wave;
      if ((lane & 3) == 0) w[lane >> 2] = z;
      __builtin_amdgcn_wave_barrier();
      const float4 *w4 = reinterpret_cast<const float4 *>(w);
      const float4 q0 = w4[0], q1 = w4[1], q2 = w4[2], q3 = w4[3];
      zs[0] = q0.x; zs[1] = q0.y; zs[2] = q0.z; zs[3] = q0.w;
      zs[4] = q1.x; zs[5] = q1.y; zs[6] = q1.z; zs[7] = q1.w;
      zs[8] = q2.x; zs[9] = q2.y; zs[10] = q2.z; zs[11] = q2.w;
      zs[12] = q3.x; zs[13] = q3.y; zs[14] = q3.z;
      __builtin_amdgcn_wave_barrier();
    } else {
#pragma unroll
      for (int c = 0; c < 15; ++c) zs[c] = bcast(z, 4 * c);
    }
  };
  broadcast_z();

  // Initial d_a: clip(|a(xi_bar)|, 0, a_max).
  float da_prev[IPL];
#pragma unroll
  for (int u = 0; u < IPL; ++u) {
    State6 s = eval_traj(L[u], zs, S.vx0);
    da_prev[u] = fminf(fsqrt(fmaf(s.xdd, s.xdd, s.ydd * s.ydd)), S.a_max);
  }

  const float4 *obs = s_obs;
  int buf = 0;
  // Sums over the sample's instants, one 64-instant block at a time: the
  // blocks (slot u of wave wi is block wi IPL + u) are reduced on their own
  // and added in block order, so the result is the same for IPL 1 and 2.
  const int B = NW * IPL, Beff = (T + kWave - 1) / kWave;
  // r: this lane's block sums of value `col`; lanes with `write` publish them.
  auto combine = [&](const float (&r)[IPL], bool write, int col) -> float {
    if (Beff == 1) return r[0];  // one block: slot 0 of wave 0
    float acc = 0.f;
    if (NW == 1) {
#pragma unroll
      for (int u = 0; u < IPL; ++u)
        if (u < Beff) acc += r[u];
      return acc;
    }
    if (write) {
#pragma unroll
      for (int u = 0; u < IPL; ++u) s_red[buf][wave * IPL + u][col] = r[u];
    }
    __syncthreads();
    if (sl < spb)  // a wave beyond the last sample of the group only syncs
      for (int b = 0; b < Beff; ++b) acc += s_red[buf][sl * B + b][col];
    return acc;
  };
  Corr cr[IPL];
  auto pass = [&]() -> float {
    target_pass<IPL, ROAD>(L, S, zs, obs, s_road, npair, T, wi * IPL * kWave + lane, tt, tv, da_prev, cr);
    float r[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
      float g[16];
      g_of(L[u], cr[u], g);
      if constexpr (IPL == 2) r[u] = reduce16_lds(g, lane, s_gred + wave * kRedFloats);
      else r[u] = reduce16(g, lane);
    }
    const float acc = combine(r, (lane & 3) == 0, v);
    if (NW > 1) buf ^= 1;
    return acc;
  };

  float Gv = pass();

  const int K = P.K;
  const int rs_addr = 64 * (lane & 3);  // byte address of lane 16 (lane & 3), the row's first rhs of this quarter
  for (int k = 1; k <= K; ++k) {
    // xi-update (eq. split_xy) in the free coordinates: lane 4 v + j adds
    // the terms k = 4 j .. 4 j + 3 of row v of A^-1 (rhs_k from lane 4 k, a
    // cross-lane read on the LDS crossbar), and the four quarter sums are
    // added over the lane quad, (q0 + q1) + (q2 + q3) in every lane
    const float rhs = fmaf(Dv, zb - z, fmaf(S.rho, Gv, mu));
    float dz = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      dz = fmaf(U.arow[i], __int_as_float(__builtin_amdgcn_ds_bpermute(rs_addr + 16 * i, __float_as_int(rhs))), dz);
    dz += dpp<kDppQuadSwap1>(dz);
    dz += dpp<kDppQuadSwap2>(dz);
    z += dz;
    broadcast_z();
    if (k < K) {
      Gv = pass();
      mu = fmaf(0.5f * S.rho, Gv, mu);  // eq. update_lagrange
    }
  }

  // Residual and upper cost of xi* = xi^K, per block as above.
  float rb[IPL], cb[IPL];
#pragma unroll
  for (int u = 0; u < IPL; ++u) {
    residual_at<ROAD>(eval_traj(L[u], zs, S.vx0), S, obs, s_road, npair, T, tt[u], tv[u], rb[u], cb[u]);
    rb[u] = wave_sum(rb[u]);
    cb[u] = wave_sum(cb[u]);
  }
  const float rr = combine(rb, lane == 0, 0);
  const float cc = combine(cb, lane == 0, 1);

  if (active) {
    const size_t row = slot_off + j;
    // all 16 entries (the pad one is 0), so each row is one whole 64-byte
    // line; every wave of the sample holds the same z, the first stores it
    if (wi == 0 && (lane & 3) == 0) A.zs[row * kZ + v] = z;
    if (wi == 0 && lane == 0) {
      A.resid[row] = rr;
      A.cost[row] = cc;
    }
    if (A.xi_star_out != nullptr && wi == 0 && ((lane & 3) == 0 || lane == 61))
      write_xi(D, P, A.xi_star_out + (size_t)j * 22, A.xi_bar_out + (size_t)j * 22, (lane & 3) == 0 ? v : 99, z,
               zb, lane == 61);
  }
}

// One upper iteration of the launch's requests: workgroup b serves the
// samples of rank b - prefix[slot] of its request. Three waves per SIMD with
// two instants per lane (the road variant would otherwise take a few more
// registers than that allows).
template <int IPL, bool ROAD>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(IPL == 2 ? 3 : 4)))
lower_kernel(LowerArgs A, MethodParams P) {
  extern __shared__ float4 s_obs[];
  __shared__ float s_red[2][4 * IPL][16];
  __shared__ double s_mu[8], s_chol[64];
  __shared__ float4 s_road[ROAD ? PLAN_MAX_ROAD : 1];
  __shared__ __align__(16) float s_gred[IPL == 2 ? 4 * kRedFloats : 4];
  __shared__ __align__(16) float s_zb[IPL == 2 ? 4 * 16 : 4];

  const int2 bi = block_slot(A);
  const ReqDesc &D = A.desc[bi.x];
  const int l = A.l_uniform >= 0 ? A.l_uniform : D.cur_iter;
  LowerSetup<IPL> U;
  lower_setup<IPL, ROAD>(A, P, D, s_obs, s_road, U);
  lower_item<IPL, ROAD>(A, P, D, bi.x, bi.y, l, U, s_obs, s_road, s_red, s_mu, s_chol, s_gred, s_zb);
}

// ---------------------------------------------------------------------------
// Lower level on the matrix cores (FP16 high/low split, FP32 accumulation).
//
// With TPW = 2 or 4 a workgroup serves 16 samples of one request with
// ceil(T / (4 TPW)) waves; wave w owns the instant tiles TPW w .. TPW w +
// TPW - 1 (4 instants each). Lane l of every
// wave belongs to sample n = l % 16 and to lane group g = l / 16, which holds
//   * free coefficients 4g .. 4g + 3 of its sample (state z, z_bar, lambda),
//   * at each tile, position / velocity / acceleration of both axes at
//     instant 4 tile + g (the accumulator layout of the evaluation product).
// Per tile and iteration, with every operand split as v = hi + lo in FP16:
//   evaluation  [x, xd, xdd](4 instants) = fixed + B_hi z + B_lo z
//               (v_mfma_f32_16x16x16_f16, z = [z_hi; z_lo]; 2 per axis)
//   N^T g       += C_hi d_hi + C_hi d_lo + C_lo d_hi
//               (v_mfma_f32_16x16x32_f16: both axes' differences of an
//               instant in one operand; 3 per tile)
// and once per iteration the xi-update dz = A^-1 rhs (3 products). The basis
// table is staged in LDS per workgroup. N^T g is accumulated per pair of
// tiles (2p, 2p + 1) from zero; the pair sums meet in LDS, each of the 256
// values is summed over the pairs in pair order by one thread, and every wave
// applies the same update. Large launches use TPW = 4 (two workgroups fit a
// CU and cover each other's barriers), middle ones TPW = 2 (two tiles per
// wave, 16 samples), and launches whose workgroups all fit the chip at once
// TPW = 1: a workgroup of 8 samples with one tile pair per wave (ceil(T / 8)
// waves, twice the workgroups and half the serial work of 16-sample ones;
// a 13-wave workgroup takes a CU to itself). There columns n
// and n + 8 of every product carry sample n & 7, the lanes of columns 8..15
// keep the pair's second tile, and that tile's N^T g products start from the
// first tile's sum rotated across the row: every sum is formed as with
// TPW = 4, so results are the same bit for bit. Everything between the
// products is the FP32 code of the VALU kernel.

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mma(h4 a, h4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f4 mma32(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// v = hi + lo: hi is v cut to 11 significant bits (exact in FP16 in its
// normal range), lo the remainder rounded to FP16.
__device__ __forceinline__ void split4(f4 v, h4 &hi, h4 &lo) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const float h = __uint_as_float(__float_as_uint(v[u]) & 0xFFFFE000u);
    hi[u] = (_Float16)h;
    lo[u] = (_Float16)(v[u] - h);
  }
}

// (d0, d1, d2, 0, e0, e1, e2, 0) split into high and low halves.
__device__ __forceinline__ void split_corr(const Corr &c, h8 &hi, h8 &lo) {
  h4 h0, l0, h1, l1;
  split4(f4{c.dox, c.dvx, c.dax, 0.f}, h0, l0);
  split4(f4{c.wy, c.dvy, c.day, 0.f}, h1, l1);
  hi = h8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
  lo = h8{l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
}

// FP32 matrix-core product 16 x 4 by 4 x 16: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; D row 4 (l / 16) + u, column l % 16 is element u of
// lane l.
__device__ __forceinline__ f4 mma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 4 x 4 transpose across the lane groups of a sample: lane group g holds
// a[g][0..3] (lanes n, n + 16, n + 32, n + 48 of sample n); returns
// b[g][u] = a[u][g]. Exchanging the off-diagonal 2 x 2 blocks between the
// half-waves, then the off-diagonal elements of each block between the
// 16-lane rows of each half.
__device__ __forceinline__ f4 transpose_groups(f4 a) {
  float a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
  swap32(a0, a2);
  swap32(a1, a3);
  swap16(a0, a1);
  swap16(a2, a3);
  return f4{a0, a1, a2, a3};
}

__device__ __forceinline__ void swap32u(uint32_t &a, uint32_t &b) {
  auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}

// Evaluation operands from the state: lanes 0..31 hold the x coefficients,
// 32..63 the y coefficients; one exchange of half-waves gives
// bx = [x_hi; x_lo] and by = [y_hi; y_lo] (lane group g holds rows 4g..4g+3).
__device__ __forceinline__ void coef_operands(f4 z, h4 &bx, h4 &by) {
  h4 hi, lo;
  split4(z, hi, lo);
  uint2 a = __builtin_bit_cast(uint2, hi), b = __builtin_bit_cast(uint2, lo);
  swap32u(a.x, b.x);
  swap32u(a.y, b.y);
  bx = __builtin_bit_cast(h4, a);
  by = __builtin_bit_cast(h4, b);
}

// Draw of Alg. 1 for the 16 columns of a wave (column n: sample j; in the
// 8-sample layout two columns draw the same sample): lane group g runs
// Philox block min(g, 2) and Box-Muller pair g of the column's sample; the
// same values as wave_draw.
__device__ void group_draw(const MethodParams &P, uint64_t seed, int j, int N, int l, bool structured,
                           const double *mu, const double *chol, int lane, float (&p)[8]) {
  const int n = lane & 15, g = lane >> 4;
  uint32_t w[4];
  rng_block(seed, j, l, g < 3 ? g : 2, w);
  const int src = n + 16 * (g >> 1);
  const uint32_t w0 = __shfl(w[0], src, 64), w1 = __shfl(w[1], src, 64);
  const uint32_t w2 = __shfl(w[2], src, 64), w3 = __shfl(w[3], src, 64);
  const bool odd = g & 1;
  float n0, n1;
  normals2(odd ? w2 : w0, odd ? w3 : w1, n0, n1);
  float z[8];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    z[2 * m] = __shfl(n0, n + 16 * m, 64);
    z[2 * m + 1] = __shfl(n1, n + 16 * m, 64);
  }
  uint32_t wb1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) wb1[m] = __shfl(w[m], n + 16, 64);
  const uint32_t sel = __shfl(w[0], n + 32, 64);
  finish_draw(P, structured, j, N, sel, z, wb1, mu, chol, p);
}

// Dynamic LDS of the matrix-core kernel: basis table [4 NT][kEvInstHalfs]
// (F32: [4 NT][kEv32InstFloats]), neighbours [pair of neighbours][T]
// (float4), fixed trajectory part [4 NT][2] (float4), N^T g per tile pair
// [ceil(NT / 2)][64] (float4), total [64].
//
// F32 selects the FP32 form of the same dataflow: every product on the
// matrix cores in FP32 (v_mfma_f32_16x16x4f32, one instant of a tile or one
// group of 4 coefficients per instruction), no operand splitting:
//   evaluation  4 products per tile (2 per axis), the coefficient operand
//               regrouped once per pass by a 4 x 4 transpose across the
//               lane groups of each sample;
//   N^T g       6 products per tile (one per axis and derivative order, the
//               instants of the tile along K, each lane's own differences as
//               its B element);
//   xi-update   4 products per iteration (A^-1 in FP32, rhs transposed).
// Four tiles per wave without the road profile: held to 128 registers per
// lane (one is spilled), which keeps two 7-wave workgroups per CU; with 129
// the FP16 split fits one and runs 50% longer.
template <int TPW, bool ROAD, bool F32>
__global__ void __launch_bounds__(kWave *(TPW == 1 ? kMfmaMaxPairs : kMfmaMaxT / (4 * TPW)))
    __attribute__((amdgpu_waves_per_eu(TPW == 4 && !ROAD ? 4 : 1))) lower_mfma_kernel(LowerArgs A, MethodParams P) {
  extern __shared__ float4 s_dyn[];
  __shared__ double s_mu[8], s_chol[64];
  __shared__ float s_rc[kMfmaMaxPairs][kMfmaSamples][2];
  __shared__ float4 s_road[ROAD ? PLAN_MAX_ROAD : 1];

  const int2 bi = block_slot(A);
  const int slot = bi.x;
  const ReqDesc &D = A.desc[slot];
  const int l = A.l_uniform >= 0 ? A.l_uniform : D.cur_iter;
  const int T = D.T, M = D.M, N = D.N;
  const int npair = (M + 1) >> 1;
  const int NT = (T + 3) >> 2;
  const int NPr = (NT + 1) >> 1;       // tile pairs
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int n = lane & 15, g = lane >> 4;
  // TPW = 1: a workgroup of 8 samples, one tile pair per wave. Columns n and
  // n + 8 of every product carry the same sample (its state held twice); the
  // lanes of columns 8..15 take the pair's second tile (hh = 1).
  constexpr bool kHalf = TPW == 1;
  const int hh = kHalf ? n >> 3 : 0;
  const int j = bi.y * (kHalf ? kMfmaSamples / 2 : kMfmaSamples) + (kHalf ? (n & 7) : n);
  const bool active = j < N;
  const size_t slot_off = (size_t)D.row_off;

  // 4 NT instants x 240 bytes (F32: 192 bytes), in float4
  const int tab_f4 = F32 ? NT * kEv32InstFloats : NT * kEvInstHalfs / 2;
  _Float16 *s_tab = reinterpret_cast<_Float16 *>(s_dyn);
  float4 *s_obs = s_dyn + tab_f4;
  float4 *s_fix = s_obs + npair * T;
  float4 *s_part = s_fix + 8 * NT;
  float4 *s_G = s_part + NPr * kWave;

  {
    const float4 *src = reinterpret_cast<const float4 *>(A.mops + D.mops_off);
    for (int i = threadIdx.x; i < tab_f4; i += blockDim.x) s_dyn[i] = src[i];
  }
  stage_neighbours(D, P, s_obs);
  if constexpr (ROAD) stage_road(D, s_road);
  const bool forced = D.init_mode == kInitForced || decoded_start(D, P, l);
  const bool structured = !forced && l == 0 && D.init_mode == kInitStructured;
  if (!forced && !structured) load_distribution(A, D, P, slot, l, bi.y == 0, s_mu, s_chol);
  const Scal S = make_scal(D, P);
  {
    // fixed part per instant: (x, xd + vx0, xdd, 0), (y, yd, ydd, 0); zero
    // beyond the horizon
    const float *Bt = A.basis + D.basis_off;
    const int Tp = D.basis_tpad;
    for (int t = threadIdx.x; t < 4 * NT; t += blockDim.x) {
      float4 fx = make_float4(0.f, 0.f, 0.f, 0.f), fy = fx;
      if (t < T) {
        const State6 f = fixed_part(Bt, Tp, t, D, P);
        fx = make_float4(f.x, S.vx0 + f.xd, f.xdd, 0.f);
        fy = make_float4(f.y, f.yd, f.ydd, 0.f);
      }
      s_fix[2 * t] = fx;
      s_fix[2 * t + 1] = fy;
    }
  }

  // Per-lane offsets (in halves) into the basis table, relative to the first
  // instant of a tile.
  //   evaluation (row n = 4 a + q, column group g): 4 coefficients from
  //   4 (g % 2) of order min(q, 2) (row q = 3 is not used) at instant a;
  //   the low-half operand multiplies both halves of z (the lo x lo term
  //   only adds precision).
  const int ev_off = (n >> 2) * kEvInstHalfs + min(n & 3, 2) * 16 + 4 * (g & 1);
  //   accumulation (row n = coefficient, column group g = instant): orders
  //   0..2 of coefficient n of x (n < 8) or n - 8 of y (8 <= n < 15), the
  //   zero pad elsewhere.
  const int ac_x = g * kEvInstHalfs + (n < 8 ? n : kEvPad);
  const int ac_y = g * kEvInstHalfs + (n >= 8 && n < 15 ? kEvAxisHalfs + (n - 8) : kEvPad);
  const int q_step_x = n < 8 ? 16 : 0, q_step_y = n >= 8 && n < 15 ? 16 : 0;
  auto ev_op = [&](int tile, int axis, int half) -> h4 {
    return *reinterpret_cast<const h4 *>(s_tab + tile * 4 * kEvInstHalfs + ev_off + axis * kEvAxisHalfs +
                                         half * 8);
  };
  auto ac_op = [&](int tile, int half) -> h8 {
    const _Float16 *bx = s_tab + tile * 4 * kEvInstHalfs + ac_x + half * 8;
    const _Float16 *by = s_tab + tile * 4 * kEvInstHalfs + ac_y + half * 8;
    return h8{bx[0], bx[q_step_x], bx[2 * q_step_x], (_Float16)0.f,
              by[0], by[q_step_y], by[2 * q_step_y], (_Float16)0.f};
  };

  //   F32 form: the table holds (x c_g, x c_{4+g}, y c_g, y c_{4+g}) per
  //   (instant, order, g); evaluation row n = 4 a + q reads its group's
  //   float4, the accumulation row n (a coefficient) reads its basis value
  //   at instant g for each order from the x or the y entry, and the zero
  //   entry (y c_7, slot 15 of every order) for the other axis.
  const float *s_t32 = reinterpret_cast<const float *>(s_dyn);
  const int ev32 = (n >> 2) * kEv32InstFloats + min(n & 3, 2) * 16 + 4 * g;
  const int acx32 = g * kEv32InstFloats + (n < 8 ? (n & 3) * 4 + (n >> 2) : 15);
  const int acy32 = g * kEv32InstFloats + (n >= 8 ? ((n - 8) & 3) * 4 + 2 + ((n - 8) >> 2) : 15);

  h4 ai_hi, ai_lo;
  f4 ai32, Dv;
  {
    const float *Pj = A.proj + (size_t)D.tm_idx * kProjFloats;
    if constexpr (F32) {
      // A^-1 row n, columns 4 kb + g (kb = 0..3)
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) ai32[kb] = Pj[n * 16 + 4 * kb + g];
    } else {
      const h4 *Ai = reinterpret_cast<const h4 *>(A.mainv) + (size_t)D.tm_idx * 2 * kWave;
      ai_hi = Ai[lane];
      ai_lo = Ai[kWave + lane];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) Dv[u] = Pj[256 + 4 * g + u];
  }
  const uint64_t seed = D.seed;
  const int draw_iter = D.first_iter + l;
  __syncthreads();  // basis table, neighbours, fixed part and distribution ready

  float pin[8];
  if (forced) {
#pragma unroll
    for (int m = 0; m < 8; ++m) pin[m] = active ? A.p[(slot_off + j) * 8 + m] : 0.f;
  } else {
    group_draw(P, seed, j, N, draw_iter, structured, s_mu, s_chol, lane, pin);
  }
  // the step-1 rows are read before the sample is stored, so that store
  // cannot hold their loads back
  f4 zb;
  {
    const float *S1 = A.step1 + (size_t)D.t_idx * kStep1Floats;
#pragma unroll
    for (int u = 0; u < 4; ++u) zb[u] = step1_coef(step1_inputs(S1, D, 4 * g + u), P, pin);
  }
  if (!forced && active && wave == 0 && g == 0 && hh == 0) {
    float4 *dst = reinterpret_cast<float4 *>(A.p + (slot_off + j) * 8);
    dst[0] = make_float4(pin[0], pin[1], pin[2], pin[3]);
    dst[1] = make_float4(pin[4], pin[5], pin[6], pin[7]);
  }
  f4 z = zb, mu = {0.f, 0.f, 0.f, 0.f};

  // Coefficient operands of a pass: FP16 halves (bx, by), or for F32 the
  // transposed state bz (bz[u] = coefficient 4 u + g of the lane's sample).
  struct CoefOps {
    h4 bx, by;
    f4 bz;
  };
  auto coef_ops = [&](f4 zz) -> CoefOps {
    CoefOps o;
    if constexpr (F32) o.bz = transpose_groups(zz);
    else coef_operands(zz, o.bx, o.by);
    return o;
  };

  // Trajectory state at this lane's instant of a tile.
  auto evaluate = [&](int tile, const CoefOps &co) -> State6 {
    const float4 cx = s_fix[2 * (4 * tile + g)], cy = s_fix[2 * (4 * tile + g) + 1];
    f4 ex = {cx.x, cx.y, cx.z, cx.w}, ey = {cy.x, cy.y, cy.z, cy.w};
    if constexpr (F32) {
      const float4 a = *reinterpret_cast<const float4 *>(s_t32 + tile * 4 * kEv32InstFloats + ev32);
      ex = mma_f32(a.x, co.bz[0], ex);
      ex = mma_f32(a.y, co.bz[1], ex);
      ey = mma_f32(a.z, co.bz[2], ey);
      ey = mma_f32(a.w, co.bz[3], ey);
    } else {
      ex = mma(ev_op(tile, 0, 0), co.bx, ex);
      ex = mma(ev_op(tile, 0, 1), co.bx, ex);
      ey = mma(ev_op(tile, 1, 0), co.by, ey);
      ey = mma(ev_op(tile, 1, 1), co.by, ey);
    }
    State6 st;
    st.x = ex[0];
    st.xd = ex[1];
    st.xdd = ex[2];
    st.y = ey[0];
    st.yd = ey[1];
    st.ydd = ey[2];
    return st;
  };

  float da[TPW];
  // One target pass over this wave's tiles at the current z (first: the
  // initial d_a from the same evaluation); returns N^T g of the workgroup.
  auto accumulate = [&](int tile, const Corr &c, f4 acc) -> f4 {
    if constexpr (F32) {
      const float *bx = s_t32 + tile * 4 * kEv32InstFloats + acx32;
      const float *by = s_t32 + tile * 4 * kEv32InstFloats + acy32;
      acc = mma_f32(bx[0], c.dox, acc);
      acc = mma_f32(bx[16], c.dvx, acc);
      acc = mma_f32(bx[32], c.dax, acc);
      acc = mma_f32(by[0], c.wy, acc);
      acc = mma_f32(by[16], c.dvy, acc);
      return mma_f32(by[32], c.day, acc);
    } else {
      h8 dh, dl;
      split_corr(c, dh, dl);
      const h8 ch = ac_op(tile, 0), cl = ac_op(tile, 1);
      acc = mma32(ch, dh, acc);
      acc = mma32(ch, dl, acc);
      return mma32(cl, dh, acc);
    }
  };
  // N^T g of a tile pair: tile b's products accumulate onto tile a's sum.
  auto pass = [&](bool first) -> f4 {
    const CoefOps co = coef_ops(z);
    if constexpr (kHalf) {
      const int pair = wave, ta = 2 * pair;
      if (ta < NT) {
        // both tiles' products over all 16 columns; each lane keeps its
        // column half's tile (the fixed part it reads is its own instant's)
        const bool has_b = ta + 1 < NT;
        const int t = 4 * (ta + hh) + g;
        const State6 s0 = evaluate(ta, co), s1 = has_b ? evaluate(ta + 1, co) : s0;
        const State6 st = hh ? s1 : s0;
        if (first) da[0] = fminf(fsqrt(fmaf(st.xdd, st.xdd, st.ydd * st.ydd)), S.a_max);
        const Corr c = targets_at<ROAD, true>(st, S, s_obs, s_road, npair, T, t < T ? t : T - 1, active && t < T,
                                              da[0]);
        // tile a's sum of each sample sits in column n < 8; rotated to column
        // n + 8 it starts tile b's products there, and the pair's sum comes
        // back to column n (the same chain as one wave over both tiles). The
        // rotations run on every lane before any per-lane choice: a lane
        // switched off would read as zero.
        const f4 a0 = accumulate(ta, c, f4{0.f, 0.f, 0.f, 0.f});
        f4 rot, acc;
#pragma unroll
        for (int u = 0; u < 4; ++u) rot[u] = dpp<kDppRowRor8>(a0[u]);
        if (has_b) {
          const f4 a1 = accumulate(ta + 1, c, rot);
#pragma unroll
          for (int u = 0; u < 4; ++u) rot[u] = dpp<kDppRowRor8>(a1[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = hh ? a1[u] : rot[u];
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = hh ? rot[u] : a0[u];
        }
        s_part[pair * kWave + lane] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
    } else {
#pragma unroll
      for (int pr = 0; pr < TPW / 2; ++pr) {
        const int pair = wave * (TPW / 2) + pr;
        if (2 * pair < NT) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int i = 2 * pr + h, tile = 2 * pair + h;
            if (tile < NT) {
              const int t = 4 * tile + g;
              const State6 st = evaluate(tile, co);
              if (first) da[i] = fminf(fsqrt(fmaf(st.xdd, st.xdd, st.ydd * st.ydd)), S.a_max);
              acc = accumulate(tile, targets_at<ROAD, true>(st, S, s_obs, s_road, npair, T, t < T ? t : T - 1,
                                                       active && t < T, da[i]),
                               acc);
            }
          }
          s_part[pair * kWave + lane] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
      }
    }
    __syncthreads();
    {
      const float *pp = reinterpret_cast<const float *>(s_part);
      float *gg = reinterpret_cast<float *>(s_G);
      for (int e = threadIdx.x; e < 4 * kWave; e += blockDim.x) {
        // all loads first (they are independent), then the sum in pair order
        float v[kMfmaMaxPairs];
#pragma unroll
        for (int w = 0; w < kMfmaMaxPairs; ++w) v[w] = w < NPr ? pp[w * 4 * kWave + e] : 0.f;
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < kMfmaMaxPairs; ++w)
          if (w < NPr) sum += v[w];
        gg[e] = sum;
      }
    }
    __syncthreads();
    const float4 q = s_G[lane];
    return f4{q.x, q.y, q.z, q.w};
  };

  f4 G = pass(true);
  const int K = P.K;
  for (int k = 1; k <= K; ++k) {
    // xi-update (eq. split_xy): dz = A^-1 rhs on the matrix cores
    f4 rhs;
#pragma unroll
    for (int u = 0; u < 4; ++u) rhs[u] = fmaf(Dv[u], zb[u] - z[u], fmaf(S.rho, G[u], mu[u]));
    f4 dz = {0.f, 0.f, 0.f, 0.f};
    if constexpr (F32) {
      const f4 rt = transpose_groups(rhs);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) dz = mma_f32(ai32[kb], rt[kb], dz);
      z += dz;
    } else {
      rhs *= kRhsScale;
      h4 rh, rl;
      split4(rhs, rh, rl);
      dz = mma(ai_hi, rh, dz);
      dz = mma(ai_hi, rl, dz);
      dz = mma(ai_lo, rh, dz);
      z += dz * (float)(1.0 / (kAinvScale * kRhsScale));
    }
    if (k < K) {
      G = pass(false);
      mu += (0.5f * S.rho) * G;  // eq. update_lagrange
    }
  }

  // Residual and upper cost of xi* = xi^K: per tile pair, summed over the
  // 4 lane groups of a sample, then over the pairs in pair order.
  {
    const CoefOps co = coef_ops(z);
#pragma unroll
    for (int pr = 0; pr < (kHalf ? 1 : TPW / 2); ++pr) {
      const int pair = kHalf ? wave : wave * (TPW / 2) + pr;
      if (2 * pair < NT) {
        float rr = 0.f, cc = 0.f;
        if constexpr (kHalf) {
          const int ta = 2 * pair, t = 4 * (ta + hh) + g;
          const bool has_b = ta + 1 < NT;
          const State6 s0 = evaluate(ta, co), s1 = has_b ? evaluate(ta + 1, co) : s0;
          float r1, c1;
          residual_at<ROAD>(hh ? s1 : s0, S, s_obs, s_road, npair, T, t < T ? t : T - 1, active && t < T, r1,
                            c1);
          rr = r1 + dpp<kDppRowRor8>(r1);  // tile a's term plus tile b's (column n ^ 8)
          cc = c1 + dpp<kDppRowRor8>(c1);
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int tile = 2 * pair + h;
            if (tile < NT) {
              const int t = 4 * tile + g;
              float r1, c1;
              residual_at<ROAD>(evaluate(tile, co), S, s_obs, s_road, npair, T, t < T ? t : T - 1,
                                active && t < T, r1, c1);
              rr += r1;
              cc += c1;
            }
          }
        }
        float a = rr, b = rr;
        swap32(a, b);
        rr = a + b;
        a = rr;
        b = rr;
        swap16(a, b);
        rr = a + b;
        a = cc;
        b = cc;
        swap32(a, b);
        cc = a + b;
        a = cc;
        b = cc;
        swap16(a, b);
        cc = a + b;
        if (g == 0) {
          s_rc[pair][n][0] = rr;
          s_rc[pair][n][1] = cc;
        }
      }
    }
  }
  __syncthreads();
  if (wave != 0 || !active || hh != 0) return;
  float rr = 0.f, cc = 0.f;
  for (int w = 0; w < NPr; ++w) {
    rr += s_rc[w][n][0];
    cc += s_rc[w][n][1];
  }
  const size_t row = slot_off + j;
  reinterpret_cast<float4 *>(A.zs + row * kZ)[g] = make_float4(z[0], z[1], z[2], z[3]);
  if (g == 0) {
    A.resid[row] = rr;
    A.cost[row] = cc;
  }
  if (A.xi_star_out != nullptr) {
    double *xs = A.xi_star_out + (size_t)j * 22, *xb = A.xi_bar_out + (size_t)j * 22;
#pragma unroll
    for (int u = 0; u < 4; ++u) write_xi(D, P, xs, xb, 4 * g + u, z[u], zb[u], g == 3 && u == 3);
  }
}

// Value v of lane `lane` (a constant) on every lane, FP64 as two 32-bit reads.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / sqrt(x) for x > 0 in FP64: the hardware estimate refined by two Newton
// steps y <- y + (y / 2)(1 - x y^2), each at least squaring the relative
// error, so the result is within a few units of the last place.
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// Lower Cholesky factor of A + jitter I (8x8, FP64) by lanes 0..7 of a
// wave, lane i owning row i: column j is finished by lane j (diagonal) and
// lanes i > j (below it) in parallel, with row j of L read from lane j. Every
// lane of the wave must call it; returns false on all lanes if A + jitter I
// is not positive definite.
__device__ bool chol8_wave(const double *A, double jitter, double *Lo, int lane) {
  const int i = lane & 7;
  double row[8], Lr[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    row[k] = A[i * 8 + k] + (k == i ? jitter : 0.0);
    Lr[k] = 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double s = row[j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= Lr[k] * readlane_d(Lr[k], j);
    // lane j: s is the pivot; lanes i > j: s is the numerator of L[i][j]
    const double piv = readlane_d(s, j);
    ok = ok && piv > 0.0;
    const double y = ok ? rsqrt_d(piv) : 1.0;
    if (i == j) Lr[j] = piv * y;
    else if (i > j) Lr[j] = s * y;
  }
  if (lane < 8)
#pragma unroll
    for (int k = 0; k < 8; ++k) Lo[i * 8 + k] = ok ? Lr[k] : 0.0;
  return ok;
}

// ---------------------------------------------------------------------------
// Selection and update: one 4-wave workgroup per request.

__device__ __forceinline__ uint32_t order_key(float f) {
  uint32_t b = __float_as_uint(f);
  if (f != f) return 0xFFFFFFFFu;  // NaN sorts last
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Exclusive prefix sum over the block of one value per thread; returns the
// thread's offset and writes the total to *total. Uses s_tmp[16] and two
// barriers.
__device__ uint32_t block_exscan(uint32_t x, uint32_t *s_tmp, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < kSelBlock / 64; ++w) {
    uint32_t t = s_tmp[w];
    if (w < wave) base += t;
    tot += t;
  }
  *total = tot;
  __syncthreads();
  return base + incl - x;
}

// Exclusive prefix sum over the block with a single barrier: the wave totals
// go to s_w[0..3], which must not be in use by a call still in flight (give
// consecutive calls distinct slots). Returns the thread's offset.
__device__ __forceinline__ uint32_t block_exscan1(uint32_t x, uint32_t *s_w, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_w[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < kSelBlock / kWave; ++w) {
    const uint32_t t = s_w[w];
    if (w < wave) base += t;
    tot += t;
  }
  *total = tot;
  return base + incl - x;
}

// Select the `want` smallest of the distinct composite keys
// s_k[0..cnt) = (key << 32) | position by counting, for each key, the keys
// below it (its rank); thread t ranks position t. The positions of the
// selected keys go to s_out[0..want) in increasing order and the position of
// rank 0 to *s_first (written before the first barrier). s_k holds an even
// number of entries (a last ~0 pads an odd cnt); cnt <= kSelBlock. Uses
// s_tmp[0..4) and two barriers. Returns the thread's index in s_out, or -1 if
// its key is not selected.
__device__ int rank_select(const unsigned long long *s_k, int cnt, int want, uint32_t *s_out, uint32_t *s_first,
                           uint32_t *s_tmp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = (cnt + 1) >> 1;
  const ulonglong2 *s_k2 = reinterpret_cast<const ulonglong2 *>(s_k);
  bool sel = false;
  if (tid < cnt) {
    const unsigned long long ki = s_k[tid];
    uint32_t rank = 0;
#pragma unroll 8
    for (int j = 0; j < half; ++j) {
      const ulonglong2 v = s_k2[j];
      rank += (v.x < ki) + (v.y < ki);
    }
    sel = rank < (uint32_t)want;
    if (rank == 0) *s_first = (uint32_t)tid;
  }
  const uint64_t bal = __ballot(sel);
  if (lane == 0) s_tmp[wave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += s_tmp[w];
  const int pos = sel ? (int)(before + __popcll(bal & ((1ull << lane) - 1ull))) : -1;
  if (sel) s_out[pos] = (uint32_t)tid;
  __syncthreads();
  return pos;
}

// Select the `want` smallest (key, position) pairs of s_key[0..cnt) (ties to
// the lower position) and write their positions, in increasing order, to
// s_out[0..want). If at least `want` keys equal the smallest key, they are
// the first `want` of those. Otherwise a radix select on the 32-bit keys,
// 8 bits per pass, narrows a prefix until the keys matching it are exactly
// the ones still wanted or all bits are fixed; one scan then ranks the
// members equal to the prefix by position. cnt <= PLAN_MAX_N. If s_wmin is
// given it holds the minima of s_key over the four waves' shares (written
// before a barrier), and the first pass over the keys is skipped.
__device__ void block_select(const uint32_t *s_key, int cnt, int want, uint32_t *s_out, uint32_t *s_hist,
                             uint32_t *s_tmp, const uint32_t *s_wmin) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Positions are split into contiguous chunks, one per thread, so the scans
  // below run in position order.
  const int chunk = (cnt + kSelBlock - 1) / kSelBlock;
  const int p0 = min(cnt, tid * chunk), p1 = min(cnt, p0 + chunk);
  // smallest key and its multiplicity
  uint32_t kmin = 0xFFFFFFFFu;
  if (s_wmin == nullptr) {
    for (int i = p0; i < p1; ++i) kmin = min(kmin, s_key[i]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, 64));
    if (lane == 0) s_tmp[wave] = kmin;
    __syncthreads();
    s_wmin = s_tmp;
  }
  kmin = s_wmin[0];
  for (int w = 1; w < kSelBlock / kWave; ++w) kmin = min(kmin, s_wmin[w]);
  uint32_t nmin = 0;
  for (int i = p0; i < p1; ++i) nmin += s_key[i] == kmin;
  uint32_t tot_min;
  uint32_t min_before = block_exscan1(nmin, s_tmp + 4, &tot_min);
  if (tot_min >= (uint32_t)want) {
    // the first `want` positions holding the smallest key
    for (int i = p0; i < p1 && min_before < (uint32_t)want; ++i)
      if (s_key[i] == kmin) s_out[min_before++] = (uint32_t)i;
    __syncthreads();
    return;
  }

  uint32_t prefix = 0, mask = 0;
  int remaining = want;
  {
    prefix = 0;
    mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
      for (int i = tid; i < 256; i += kSelBlock) s_hist[i] = 0;
      __syncthreads();
      for (int i0 = 0; i0 < cnt; i0 += kSelBlock) {
        const int i = i0 + tid;
        const uint32_t k = i < cnt ? s_key[i] : 0u;
        const bool match = i < cnt && (k & mask) == prefix;
        const uint32_t digit = (k >> shift) & 255u;
        // one atomic for the lanes sharing the first matching lane's digit
        // (skewed keys would otherwise serialise on one bin)
        const uint64_t act = __ballot(match);
        if (act) {
          const int leader = __builtin_ctzll(act);
          const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)digit, leader);
          const uint64_t same = __ballot(match && digit == dl);
          if (lane == leader) atomicAdd(&s_hist[dl], (uint32_t)__popcll(same));
          if (match && digit != dl) atomicAdd(&s_hist[digit], 1u);
        }
      }
      __syncthreads();
      if (tid < 64) {
        uint32_t h[4], sum = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          h[u] = s_hist[4 * tid + u];
          sum += h[u];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          uint32_t y = __shfl_up(incl, d, 64);
          if (tid >= d) incl += y;
        }
        uint32_t before = incl - sum;
        for (int u = 0; u < 4; ++u) {
          if (before < (uint32_t)remaining && (uint32_t)remaining <= before + h[u]) {
            s_tmp[16] = 4 * tid + u;
            s_tmp[17] = before;
            s_tmp[18] = h[u];
          }
          before += h[u];
        }
      }
      __syncthreads();
      const uint32_t b = s_tmp[16];
      remaining -= (int)s_tmp[17];
      prefix |= b << shift;
      mask |= 0xFFu << shift;
      const bool exact = s_tmp[18] == (uint32_t)remaining;
      __syncthreads();
      if (exact) break;  // every key matching the prefix is selected
    }
  }
  uint32_t eq = 0;
  for (int i = p0; i < p1; ++i) eq += (s_key[i] & mask) == prefix;
  uint32_t tot;
  uint32_t eq_before = block_exscan(eq, s_tmp, &tot);
  uint32_t sel = 0;
  for (int i = p0; i < p1; ++i) {
    const uint32_t k = s_key[i] & mask;
    if (k < prefix) ++sel;
    else if (k == prefix) sel += (eq_before++ < (uint32_t)remaining);
  }
  eq_before -= eq;
  uint32_t pos = block_exscan(sel, s_tmp, &tot);
  for (int i = p0; i < p1; ++i) {
    const uint32_t k = s_key[i] & mask;
    bool take = k < prefix;
    if (k == prefix) take = eq_before++ < (uint32_t)remaining;
    if (take) s_out[pos++] = (uint32_t)i;
  }
  __syncthreads();
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sample mean and covariance (normalised by N) of the rows p[0..N) (x 8),
// FP64, two passes: the prior of the first update when the samples come
// from the decoder sampler. Thread t sums rows t, t + 256, ...; each wave
// sums its lanes in a fixed butterfly order and the four wave sums meet in
// LDS (part), so the result does not depend on timing.
__device__ void sample_moments(const float *p, int N, double *s_mu, double *s_sig, double (*part)[64 + 8]) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  double m[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) m[a] = 0.0;
  for (int i = tid; i < N; i += kSelBlock) {
    const float4 u = reinterpret_cast<const float4 *>(p + (size_t)i * 8)[0];
    const float4 v = reinterpret_cast<const float4 *>(p + (size_t)i * 8)[1];
    const float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
    for (int a = 0; a < 8; ++a) m[a] += (double)x[a];
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) m[a] = wave_sum_d(m[a]);
  if (lane == 0)
    for (int a = 0; a < 8; ++a) part[w][a] = m[a];
  __syncthreads();
  if (tid < 8) s_mu[tid] = (((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid]) / (double)N;
  __syncthreads();
  double mu[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) mu[a] = s_mu[a];
  double c[36];  // upper triangle, row by row
#pragma unroll
  for (int k = 0; k < 36; ++k) c[k] = 0.0;
  for (int i = tid; i < N; i += kSelBlock) {
    const float4 u = reinterpret_cast<const float4 *>(p + (size_t)i * 8)[0];
    const float4 v = reinterpret_cast<const float4 *>(p + (size_t)i * 8)[1];
    const float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    double d[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) d[a] = (double)x[a] - mu[a];
    int k = 0;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = a; b < 8; ++b) c[k++] += d[a] * d[b];
  }
#pragma unroll
  for (int k = 0; k < 36; ++k) c[k] = wave_sum_d(c[k]);
  __syncthreads();  // part is read above
  if (lane == 0)
    for (int k = 0; k < 36; ++k) part[w][k] = c[k];
  __syncthreads();
  if (tid < 64) {
    int a = tid >> 3, b = tid & 7;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int k = a * 8 - a * (a - 1) / 2 + (b - a);
    s_sig[tid] = (((part[0][k] + part[1][k]) + part[2][k]) + part[3][k]) / (double)N;
  }
  __syncthreads();
}

// LDS of the selection / update of one request: the select kernel's static
// arrays, or (fused iterations) a part of the lower kernel's dynamic LDS
// with s_key and s_c sized for the request's N.
struct SelLds {
  uint32_t *s_key;                 // [N] residual keys
  float *s_c;                      // [N] c_u + r
  uint32_t *s_ces;                 // [kMaxCes]
  unsigned long long *s_key2;      // [kSelBlock + 2] (key << 32) | CES position, 16-byte aligned
  unsigned long long *s_bestw;     // [kSelBlock / kWave]
  uint32_t *s_es;                  // [kMaxCes]
  uint32_t *s_hist;                // [256]
  uint32_t *s_tmp;                 // [32]
  uint32_t *s_wmin;                // [kSelBlock / kWave]
  double *s_w;                     // [kMaxEs]
  float (*s_p)[8];                 // [kMaxEs][8], 16-byte aligned
  double *s_mu, *s_sig;            // [8], [64]
  double (*s_part)[64 + 8];        // [4][72]
  double *s_wsum;                  // [4]
  uint32_t *s_first;               // [1]
  double (*s_rc64)[2];             // [3][2]
};

// Bytes of a SelLds for n_keys keys (16-byte aligned parts, in the order
// sel_lds_carve lays them out).
__host__ __device__ constexpr size_t sel_lds_bytes(int n_keys) {
  return 16 * (((size_t)n_keys * 4 + 15) / 16) * 2 + 16 * ((kMaxCes * 4 + 15) / 16) * 2 +
         16 * (((kSelBlock + 2) * 8 + 15) / 16) + 16 * ((kSelBlock / kWave * 8 + 15) / 16) + 16 * (256 * 4 / 16) +
         16 * (32 * 4 / 16) + 16 * ((kSelBlock / kWave * 4 + 15) / 16) + 16 * (kMaxEs * 8 / 16) +
         16 * (kMaxEs * 32 / 16) + 16 * (8 * 8 / 16) + 16 * (64 * 8 / 16) + 16 * (4 * 72 * 8 / 16) + 16 * 2 + 16 +
         16 * (3 * 2 * 8 / 16);
}

__device__ inline SelLds sel_lds_carve(char *base, int n_keys) {
  SelLds L;
  size_t o = 0;
  auto take = [&](size_t bytes) -> char * {
    char *q = base + o;
    o += 16 * ((bytes + 15) / 16);
    return q;
  };
  L.s_key = reinterpret_cast<uint32_t *>(take((size_t)n_keys * 4));
  L.s_c = reinterpret_cast<float *>(take((size_t)n_keys * 4));
  L.s_ces = reinterpret_cast<uint32_t *>(take(kMaxCes * 4));
  L.s_es = reinterpret_cast<uint32_t *>(take(kMaxCes * 4));
  L.s_key2 = reinterpret_cast<unsigned long long *>(take((kSelBlock + 2) * 8));
  L.s_bestw = reinterpret_cast<unsigned long long *>(take(kSelBlock / kWave * 8));
  L.s_hist = reinterpret_cast<uint32_t *>(take(256 * 4));
  L.s_tmp = reinterpret_cast<uint32_t *>(take(32 * 4));
  L.s_wmin = reinterpret_cast<uint32_t *>(take(kSelBlock / kWave * 4));
  L.s_w = reinterpret_cast<double *>(take(kMaxEs * 8));
  L.s_p = reinterpret_cast<float(*)[8]>(take(kMaxEs * 32));
  L.s_mu = reinterpret_cast<double *>(take(8 * 8));
  L.s_sig = reinterpret_cast<double *>(take(64 * 8));
  L.s_part = reinterpret_cast<double(*)[72]>(take(4 * 72 * 8));
  L.s_wsum = reinterpret_cast<double *>(take(4 * 8));
  L.s_first = reinterpret_cast<uint32_t *>(take(4));
  L.s_rc64 = reinterpret_cast<double(*)[2]>(take(3 * 2 * 8));
  return L;
}

// ConstraintEliteSet, EliteSet and the update of mu, Sigma (and on the last
// iteration the result) for the request in `slot` at upper iteration l
// (l_uniform, or the descriptor's cur_iter), by one workgroup of kSelBlock
// threads.
__device__ __forceinline__ void select_update_body(const SelArgs &A, const MethodParams &P, int slot,
                                                   const SelLds &Ls) {
  uint32_t *const s_key = Ls.s_key;
  float *const s_c = Ls.s_c;
  uint32_t *const s_ces = Ls.s_ces;
  unsigned long long *const s_key2 = Ls.s_key2;
  unsigned long long *const s_bestw = Ls.s_bestw;
  uint32_t *const s_es = Ls.s_es;
  uint32_t *const s_hist = Ls.s_hist;
  uint32_t *const s_tmp = Ls.s_tmp;
  uint32_t *const s_wmin = Ls.s_wmin;
  double *const s_w = Ls.s_w;
  float(*const s_p)[8] = Ls.s_p;
  double *const s_mu = Ls.s_mu, *const s_sig = Ls.s_sig;
  double(*const s_part)[64 + 8] = Ls.s_part;
  double *const s_wsum = Ls.s_wsum;
  uint32_t &s_first = *Ls.s_first;

  ReqDesc &D = A.desc[slot];
  DistState &Sd = A.dist[slot];
  ResultRec &R = A.result[slot];
  const int tid = threadIdx.x;
  const int l = A.l_uniform >= 0 ? A.l_uniform : D.cur_iter;
  const int N = D.N, n = D.n_ces, q = D.n_es;
  const size_t base = (size_t)D.row_off;
  const float *r = A.resid + base, *cu = A.cost + base;
  const float *p = A.p + base * 8;
  const bool last = (l == P.L - 1);

  // Residual keys and costs c_u + r of all samples into LDS, and the
  // smallest key of each wave's share.
  uint32_t kmin = 0xFFFFFFFFu;
#pragma unroll 4
  for (int i = tid; i < N; i += kSelBlock) {
    const float rr = r[i], cc = cu[i];
    const uint32_t k = order_key(rr);
    s_key[i] = k;
    s_c[i] = cc + rr;
    kmin = min(kmin, k);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, 64));
  if ((tid & 63) == 0) s_wmin[tid >> 6] = kmin;
  // Distribution before this update: the prior at iteration 0.
  if (l == 0 && decoded_start(D, P, l)) {
    sample_moments(p, N, s_mu, s_sig, s_part);
    if (tid == 0) {
      bool fin = true;
      for (int i = 0; i < 8; ++i) fin &= isfinite(s_mu[i]);
      for (int i = 0; i < 64; ++i) fin &= isfinite(s_sig[i]);
      R.status = fin ? 0 : PLAN_E_INVALID;  // e.g. a decoder activation beyond the FP16 range
      R.iterations = 0;
    }
  } else if (l == 0) {
    if (tid == 0) {
      int ok = 1;
      if (D.init_mode == kInitStructured) {
        structured_moments(P, s_mu, s_sig);
      } else {
        // the prior the lower level drew from, copied into the slot's state
        // by its first workgroup (a session's store may change meanwhile)
        for (int a = 0; a < 8; ++a) s_mu[a] = Sd.mu[a];
        for (int i = 0; i < 64; ++i) s_sig[i] = Sd.sigma[i];
        double Lt[64];
        ok = chol8(s_sig, P.cov_jitter, Lt) ? 1 : 0;
      }
      R.status = ok ? 0 : PLAN_E_INVALID;
      R.iterations = 0;
    }
  } else {
    for (int i = tid; i < 72; i += kSelBlock) {
      if (i < 8) s_mu[i] = Sd.mu[i];
      else s_sig[i - 8] = Sd.sigma[i - 8];
    }
  }
  __syncthreads();
  if (R.status != 0) return;

  // ConstraintEliteSet: the n smallest (r_j, j).
  block_select(s_key, N, n, s_ces, s_hist, s_tmp, s_wmin);
  // EliteSet: the q smallest (c_u + r, j) over the ConstraintEliteSet, whose
  // members are listed in increasing sample index, so the CES position
  // breaks ties as the sample index does. Up to one member per thread they
  // are ranked by counting (the member of rank 0 is the lowest cost of the
  // EliteSet, ties: lower index); larger sets go through the radix select
  // on the cost keys (s_key is free again) and a minimum over the set.
  // The EliteSet's rows go to s_p and their weights
  // s_j = exp(-(c_j - c_min) / gamma), FP64, to s_w, in EliteSet order.
  uint32_t jbest;
  if (n <= kSelBlock) {
    // Thread t owns CES member t: its row is loaded while the ranks are
    // counted, and written where the member lands in the EliteSet.
    float4 row0 = make_float4(0.f, 0.f, 0.f, 0.f), row1 = row0;
    uint32_t jown = 0;
    if (tid < n) {
      jown = s_ces[tid];
      s_key2[tid] = ((unsigned long long)order_key(s_c[jown]) << 32) | (unsigned long long)tid;
      if (A.tr_ces) A.tr_ces[((size_t)slot * P.L + l) * A.max_ces + tid] = (int32_t)jown;
      const float4 *pr = reinterpret_cast<const float4 *>(p + (size_t)jown * 8);
      row0 = pr[0];
      row1 = pr[1];
    }
    if (tid == 0 && (n & 1)) s_key2[n] = ~0ull;
    __syncthreads();
    const int pos = rank_select(s_key2, n, q, s_es, &s_first, s_tmp);
    jbest = s_ces[s_first];
    if (pos >= 0) {
      reinterpret_cast<float4 *>(s_p[pos])[0] = row0;
      reinterpret_cast<float4 *>(s_p[pos])[1] = row1;
      s_w[pos] = exp(-((double)s_c[jown] - (double)s_c[jbest]) / P.gamma);
      if (A.tr_es) A.tr_es[((size_t)slot * P.L + l) * A.max_es + pos] = (int32_t)jown;
    }
  } else {
    for (int i = tid; i < n; i += kSelBlock) {
      const uint32_t j = s_ces[i];
      s_key[i] = order_key(s_c[j]);
      if (A.tr_ces) A.tr_ces[((size_t)slot * P.L + l) * A.max_ces + i] = (int32_t)j;
    }
    __syncthreads();
    block_select(s_key, n, q, s_es, s_hist, s_tmp, nullptr);
    unsigned long long best = ~0ull;
    for (int i = tid; i < q; i += kSelBlock) {
      const uint32_t pos = s_es[i];
      best = min(best, ((unsigned long long)s_key[pos] << 32) | pos);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const unsigned long long o = __shfl_xor(best, d, 64);
      best = min(best, o);
    }
    if ((tid & 63) == 0) s_bestw[tid >> 6] = best;
    __syncthreads();
    for (int w = 0; w < kSelBlock / kWave; ++w) best = min(best, s_bestw[w]);
    jbest = s_ces[(uint32_t)(best & 0xFFFFFFFFull)];
    // all loads first, then the LDS writes (q <= kMaxEs)
    constexpr int kRowIt = kMaxEs * 8 / kSelBlock;
    float pv[kRowIt];
#pragma unroll
    for (int u = 0; u < kRowIt; ++u) {
      const int e = tid + u * kSelBlock;
      pv[u] = e < q * 8 ? p[(size_t)s_ces[s_es[e >> 3]] * 8 + (e & 7)] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kRowIt; ++u) {
      const int e = tid + u * kSelBlock;
      if (e < q * 8) s_p[e >> 3][e & 7] = pv[u];
    }
    const double cmin = (double)s_c[jbest];
    for (int i = tid; i < q; i += kSelBlock) {
      const uint32_t j = s_ces[s_es[i]];
      s_w[i] = exp(-((double)s_c[j] - cmin) / P.gamma);
      if (A.tr_es) A.tr_es[((size_t)slot * P.L + l) * A.max_es + i] = (int32_t)j;
    }
  }
  __syncthreads();
  // eq. mean_update and eq. cov_update in one pass over the EliteSet,
  // about the current mean mu: with d_i = p_i - mu, S = sum s_i,
  // u = sum s_i d_i / S and C = sum s_i d_i d_i^T, the new mean is
  // mu + eta u and the weighted scatter about it is C + S (eta^2 - 2 eta) u u^T.
  // Wave w sums elites w, w + 4, ...; lane e the entry (e / 8, e % 8), each
  // term s_i (d_a d_b) with the differences multiplied first, so C_ab and C_ba
  // are bitwise equal. The four partial sums are added in wave order.
  {
    const int e = tid & 63, part = tid >> 6, a = e >> 3, b = e & 7;
    const double mua = s_mu[a], mub = s_mu[b];
    double c = 0.0, sa = 0.0, ss = 0.0;
#pragma unroll 4
    for (int i = part; i < q; i += 4) {
      const double w = s_w[i];
      const double da = (double)s_p[i][a] - mua, db = (double)s_p[i][b] - mub;
      c += w * (da * db);
      sa += w * da;
      ss += w;
    }
    s_part[part][e] = c;
    if (b == 0) s_part[part][64 + a] = sa;
    if (e == 0) s_wsum[part] = ss;
  }
  __syncthreads();
  if (tid < 64) {
    const int a = tid >> 3, b = tid & 7;
    const double S = ((s_wsum[0] + s_wsum[1]) + s_wsum[2]) + s_wsum[3];
    const double C = ((s_part[0][tid] + s_part[1][tid]) + s_part[2][tid]) + s_part[3][tid];
    const double ua = (((s_part[0][64 + a] + s_part[1][64 + a]) + s_part[2][64 + a]) + s_part[3][64 + a]) / S;
    const double ub = (((s_part[0][64 + b] + s_part[1][64 + b]) + s_part[2][64 + b]) + s_part[3][64 + b]) / S;
    const double cs = P.eta * (C / S + P.eta * (P.eta - 2.0) * (ua * ub));
    const double nab = (1.0 - P.eta) * s_sig[a * 8 + b] + cs, nba = (1.0 - P.eta) * s_sig[b * 8 + a] + cs;
    const double sym = 0.5 * (nab + nba);
    s_part[0][tid] = sym;  // each thread reads only its own entry of row 0 above
    Sd.sigma[tid] = sym;
    if (A.tr_sigma) A.tr_sigma[((size_t)slot * P.L + l) * 64 + tid] = sym;
    const double mun = s_mu[b] + P.eta * ub;  // component b (threads 0..7: a = 0)
    if (tid < 8) {
      Sd.mu[tid] = mun;
      if (A.tr_mu) A.tr_mu[((size_t)slot * P.L + l) * 8 + tid] = mun;
    }
    if (D.session_wb >= 0 && last) {
      double *st = A.sess + (size_t)D.session_wb * 72;
      st[8 + tid] = sym;
      if (tid < 8) st[tid] = mun;
    }
  }
  __syncthreads();
  if (tid < 64) {
    const bool ok = chol8_wave(&s_part[0][0], P.cov_jitter, Sd.chol, tid);
    if (tid == 0) {
      R.iterations = l + 1;
      if (!ok) R.status = PLAN_E_INVALID;
      if (A.l_uniform < 0) D.cur_iter = l + 1;
    }
  }
  if (last) {
    // Return: lowest c_u + r in the final EliteSet (ties: lower index),
    // written by waves 1-3 while wave 0 factors the covariance. The returned
    // trajectory's residual over Table ineq_list and its upper cost are
    // evaluated again in FP64 (instant k on thread 64 + k, k + 192, ...),
    // summed per wave in lane order and then over the waves in wave order;
    // they set the result's residual, cost and infeasible flag, and the
    // trajectory's positions at every instant are stored.
    double(*const s_rc64)[2] = Ls.s_rc64;
    if (tid >= 64) {
      const int t = tid - 64;
      const uint32_t b = jbest;
      const double n10 = 10.0, tf = P.t_f;
      const double x0 = D.ego[0], y0 = D.ego[1], vx0 = D.ego[2], vy0 = D.ego[3];
      const double ax0 = D.ego[4], ay0 = D.ego[5];
      const float *zb = A.zs + (base + b) * kZ;
      double xi[22];
      xi[0] = x0;
      xi[1] = x0 + vx0 * tf / n10;
      xi[2] = x0 + 2.0 * vx0 * tf / n10 + ax0 * tf * tf / (n10 * (n10 - 1.0));
      xi[11] = y0;
      xi[12] = y0 + vy0 * tf / n10;
      xi[13] = y0 + 2.0 * vy0 * tf / n10 + ay0 * tf * tf / (n10 * (n10 - 1.0));
#pragma unroll
      for (int c = 0; c < 8; ++c) xi[3 + c] = (double)zb[c] + x0 + vx0 * tf * (double)(3 + c) / n10;
#pragma unroll
      for (int c = 0; c < 6; ++c) xi[14 + c] = (double)zb[8 + c];
      xi[20] = xi[21] = (double)zb[14];
      if (t < 22) R.xi[t] = xi[t];
      if (t < 8) R.p[t] = (double)p[(size_t)b * 8 + t];
      double rr = 0.0, cc = 0.0;
      for (int k = t; k < D.T; k += kSelBlock - kWave) {
        double rk, ck, xk, yk;
        residual_cost64(D, P, xi, k, rk, ck, xk, yk);
        rr += rk;
        cc += ck;
        if (A.traj) {
          A.traj[((size_t)slot * A.traj_stride + k) * 2] = xk;
          A.traj[((size_t)slot * A.traj_stride + k) * 2 + 1] = yk;
        }
      }
      rr = wave_sum_d(rr);
      cc = wave_sum_d(cc);
      if ((tid & 63) == 0) {
        s_rc64[(tid >> 6) - 1][0] = rr;
        s_rc64[(tid >> 6) - 1][1] = cc;
      }
    }
    __syncthreads();
    if (tid == 64) {
      const double r64 = (s_rc64[0][0] + s_rc64[1][0]) + s_rc64[2][0];
      R.best = (int32_t)jbest;
      R.cost_upper = (s_rc64[0][1] + s_rc64[1][1]) + s_rc64[2][1];
      R.residual = r64;
      uint32_t fl = (r64 > 0.0) ? PLAN_F_INFEASIBLE : 0u;
      if (D.init_mode == kInitSession || D.init_mode == kInitGiven) fl |= PLAN_F_WARM;
      R.flags = fl;
    }
  }
  // Trace of this iteration's samples, residuals and costs.
  if (A.tr_p) {
    const size_t tb = ((size_t)slot * P.L + l) * A.max_N;
    for (int i = tid; i < N; i += kSelBlock) {
      for (int a = 0; a < 8; ++a) A.tr_p[(tb + i) * 8 + a] = p[(size_t)i * 8 + a];
      A.tr_r[tb + i] = r[i];
      A.tr_c[tb + i] = cu[i];
    }
  }
}

__global__ void __launch_bounds__(kSelBlock) select_update_kernel(SelArgs A, MethodParams P) {
  __shared__ uint32_t s_key[PLAN_MAX_N];
  __shared__ float s_c[PLAN_MAX_N];
  __shared__ uint32_t s_ces[kMaxCes];
  __shared__ __align__(16) unsigned long long s_key2[kSelBlock + 2];
  __shared__ unsigned long long s_bestw[kSelBlock / kWave];
  __shared__ uint32_t s_es[kMaxCes];
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_tmp[32];
  __shared__ uint32_t s_wmin[kSelBlock / kWave];
  __shared__ double s_w[kMaxEs];
  __shared__ __align__(16) float s_p[kMaxEs][8];
  __shared__ double s_mu[8], s_sig[64];
  __shared__ double s_part[4][64 + 8];
  __shared__ double s_wsum[4];
  __shared__ uint32_t s_first;
  __shared__ double s_rc64[3][2];
  const SelLds Ls{s_key, s_c, s_ces, s_key2, s_bestw, s_es, s_hist, s_tmp, s_wmin, s_w, s_p, s_mu, s_sig,
                  s_part, s_wsum, &s_first, s_rc64};
  select_update_body(A, P, A.slots[blockIdx.x], Ls);
}

// ---------------------------------------------------------------------------
// Every upper iteration of a launch group in one launch (Alg. 1's loop on
// the device).
//
// The launch has one workgroup per work item: item g = l W + w (W
// workgroups per iteration, w in the launch's workgroup order) is the
// samples of rank w - prefix[i] of active request i at upper iteration l. A
// workgroup takes its item from a counter when it starts, so items are taken
// in increasing order, and only by workgroups that are running. The
// workgroup that completes the last item of request i at iteration l runs
// that request's selection and update (the body of select_update_kernel) and
// then publishes l + 1; an item of iteration l + 1 does its request set-up
// and then waits for that before it draws. Every item an item waits for has
// a smaller index and was taken by a running workgroup, so the launch
// finishes however many workgroups are resident.
//
// Waits are bounded: after wait_ticks of the wall clock (or once another
// workgroup has given up) a workgroup sets the give-up word and skips its
// item; later workgroups skip theirs, and the requests whose updates did not
// all run get status PLAN_E_TIMEOUT. The last workgroup to finish sets the
// control words back to zero for the next launch.
//
// Control words (zero at launch):
//   [0] next work item   [1] give-up word   [2] workgroups finished
//   [4 + i]              workgroups of request i done (over all iterations)
//   [4 + n_act + i]      updates of request i that have run
struct FusedArgs {
  uint32_t *ctl;
  uint64_t wait_ticks;  // wall-clock ticks a wait may last
};

// Thread 0 of a workgroup: wait until *ready >= l, with the bounds above.
// True: the update has run and its writes are visible to the workgroup
// after the next barrier.
__device__ bool wait_update(const uint32_t *ready, uint32_t l, uint32_t *gave_up, uint64_t wait_ticks) {
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (;;) {
    if (__hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= l) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    }
    if (__hip_atomic_load(gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if ((uint64_t)wall_clock64() - t0 > wait_ticks) {
      __hip_atomic_store(gave_up, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

template <int IPL, bool ROAD>
__global__ void __launch_bounds__(kBlock) lower_fused_kernel(LowerArgs A, SelArgs SA, MethodParams P, FusedArgs F) {
  extern __shared__ float4 s_dyn[];  // neighbour table, then the selection's arrays
  __shared__ float s_red[2][4 * IPL][16];
  __shared__ double s_mu[8], s_chol[64];
  __shared__ float4 s_road[ROAD ? PLAN_MAX_ROAD : 1];
  __shared__ __align__(16) float s_gred[IPL == 2 ? 4 * kRedFloats : 4];
  __shared__ __align__(16) float s_zb[IPL == 2 ? 4 * 16 : 4];
  __shared__ int s_msg[3];

  const int n_act = A.n_act;
  const int W = A.blk_prefix[n_act];
  uint32_t *const claim = F.ctl, *const gave_up = F.ctl + 1, *const finished = F.ctl + 2;
  uint32_t *const done = F.ctl + 4, *const ready = F.ctl + 4 + n_act;
  if (threadIdx.x == 0) {
    int g = -1;
    if (__hip_atomic_load(gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      g = (int)__hip_atomic_fetch_add(claim, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_msg[0] = g;
  }
  __syncthreads();
  // values broadcast through LDS are uniform: readfirstlane keeps them, and
  // every address derived from them, in scalar registers
  const int g = __builtin_amdgcn_readfirstlane(s_msg[0]);
  if (g >= 0 && g < W * P.L) {
    const int l = g / W, w = g - l * W;
    int lo = 0, hi = n_act - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.blk_prefix[mid] <= w) lo = mid;
      else hi = mid - 1;
    }
    const int pos = lo, slot = A.act_slots[pos];
    const ReqDesc &D = A.desc[slot];
    LowerSetup<IPL> U;
    lower_setup<IPL, ROAD>(A, P, D, s_dyn, s_road, U);
    bool go = true;
    if (l > 0) {
      if (threadIdx.x == 0) s_msg[1] = wait_update(ready + pos, (uint32_t)l, gave_up, F.wait_ticks);
      __syncthreads();
      go = __builtin_amdgcn_readfirstlane(s_msg[1]) != 0;
    }
    if (go) {
      lower_item<IPL, ROAD>(A, P, D, slot, w - A.blk_prefix[pos], l, U, s_dyn, s_road, s_red, s_mu, s_chol,
                            s_gred, s_zb);
      // every wave's rows written and its reads done, at device scope,
      // before the workgroup counts itself
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint32_t nb = (uint32_t)(A.blk_prefix[pos + 1] - A.blk_prefix[pos]);
        const uint32_t old = __hip_atomic_fetch_add(done + pos, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_msg[2] = old + 1 == nb * (uint32_t)(l + 1);
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_msg[2])) {
        // the last item of this request at iteration l: its update
        SelArgs sa = SA;
        sa.l_uniform = l;
        select_update_body(sa, P, slot, sel_lds_carve(reinterpret_cast<char *>(s_dyn), PLAN_MAX_N));
        // the update's writes and reads complete before the next iteration
        // may overwrite the rows
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
          __hip_atomic_store(ready + pos, (uint32_t)(l + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    s_msg[0] = __hip_atomic_fetch_add(finished, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (!__builtin_amdgcn_readfirstlane(s_msg[0])) return;
  // the last workgroup to finish
  if (__hip_atomic_load(gave_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
    for (int i = threadIdx.x; i < n_act; i += kBlock)
      if (__hip_atomic_load(ready + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)P.L)
        SA.result[A.act_slots[i]].status = PLAN_E_TIMEOUT;
  __syncthreads();  // every thread has read the words before they are cleared
  for (int i = threadIdx.x; i < 4 + 2 * n_act; i += kBlock) F.ctl[i] = 0u;
}

// Dynamic LDS of a fused launch: the neighbour table or the selection's
// arrays, whichever is larger. The selection's arrays are sized for
// PLAN_MAX_N keys whatever the requests' N: at fixed offsets their addresses
// are constants.
size_t fused_lds_bytes(size_t obs_lds) {
  return obs_lds > sel_lds_bytes(PLAN_MAX_N) ? obs_lds : sel_lds_bytes(PLAN_MAX_N);
}

// Fused launch of one launch group: nblocks workgroups per iteration, one
// launch workgroup per (iteration, workgroup).
hipError_t launch_lower_fused(const LowerArgs &a, const SelArgs &sa, const MethodParams &p, uint32_t *ctl,
                              int nblocks, int ipl, bool road, size_t obs_lds, uint64_t wait_ticks, hipStream_t st,
                              hipEvent_t ev0, hipEvent_t ev1) {
  if (ipl != 1 && ipl != 2) return hipErrorInvalidValue;
  if (nblocks <= 0 || p.L <= 0 || (int64_t)nblocks * p.L > 0x7fffffff) return hipErrorInvalidValue;
  auto kern = ipl == 1 ? (road ? lower_fused_kernel<1, true> : lower_fused_kernel<1, false>)
                       : (road ? lower_fused_kernel<2, true> : lower_fused_kernel<2, false>);
  const size_t lds = fused_lds_bytes(obs_lds);
  FusedArgs F;
  F.ctl = ctl;
  F.wait_ticks = wait_ticks;
  const int grid = nblocks * p.L;
  if (ev0)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), (uint32_t)lds, st, ev0, ev1, 0, a, sa, p, F);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, st, a, sa, p, F);
  return hipGetLastError();
}

hipError_t launch_lower(const LowerArgs &a, const MethodParams &p, int nblocks, int ipl, bool road, size_t lds,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ipl != 1 && ipl != 2) return hipErrorInvalidValue;
  auto kern = ipl == 1 ? (road ? lower_kernel<1, true> : lower_kernel<1, false>)
                       : (road ? lower_kernel<2, true> : lower_kernel<2, false>);
  if (ev0)
    hipExtLaunchKernelGGL(kern, dim3(nblocks), dim3(kBlock), (uint32_t)lds, st, ev0, ev1, 0, a, p);
  else
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kBlock), lds, st, a, p);
  return hipGetLastError();
}
hipError_t launch_lower_mfma(const LowerArgs &a, const MethodParams &p, int nblocks, int tpw, bool road, bool f32,
                             int T, size_t lds, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if ((tpw != 1 && tpw != 2 && tpw != 4) || T < 1 || T > kMfmaMaxT) return hipErrorInvalidValue;
  const int waves = tpw == 1 ? ((T + 3) / 4 + 1) / 2 : (T + 4 * tpw - 1) / (4 * tpw);
  using K = void (*)(LowerArgs, MethodParams);
  const K k1 = f32 ? (road ? lower_mfma_kernel<1, true, true> : lower_mfma_kernel<1, false, true>)
                   : (road ? lower_mfma_kernel<1, true, false> : lower_mfma_kernel<1, false, false>);
  const K k2 = f32 ? (road ? lower_mfma_kernel<2, true, true> : lower_mfma_kernel<2, false, true>)
                   : (road ? lower_mfma_kernel<2, true, false> : lower_mfma_kernel<2, false, false>);
  const K k4 = f32 ? (road ? lower_mfma_kernel<4, true, true> : lower_mfma_kernel<4, false, true>)
                   : (road ? lower_mfma_kernel<4, true, false> : lower_mfma_kernel<4, false, false>);
  const K kern = tpw == 1 ? k1 : tpw == 2 ? k2 : k4;
  if (ev0 != nullptr)
    hipExtLaunchKernelGGL(kern, dim3(nblocks), dim3(kWave * waves), (uint32_t)lds, st, ev0, ev1, 0, a, p);
  else
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kWave * waves), lds, st, a, p);
  return hipGetLastError();
}

hipError_t launch_select(const SelArgs &a, const MethodParams &p, int nreq, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL(select_update_kernel, dim3(nreq), dim3(kSelBlock), 0, st, ev0, ev1, 0, a, p);
  else
    hipLaunchKernelGGL(select_update_kernel, dim3(nreq), dim3(kSelBlock), 0, st, a, p);
  return hipGetLastError();
}
}  // namespace plan
