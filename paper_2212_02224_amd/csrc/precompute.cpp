// precompute.cpp -- sample-independent matrices of the lower level, built
// once per horizon length T (and obstacle count M) in FP64 on the host and
// stored as FP32 tables for the kernels (Sec. III-C: the KKT inverse is
// computed once, irrespective of the batch size).
//
//   basis   Bernstein polynomials of order 10 on tau = t / t_f and their first
//           two time derivatives at t_k = k t_f / (T - 1) (eq. param).
//   step1   affine map of the Step-1 QP of Alg. 1 restricted to the free
//           coefficients: z_bar = S p' + R b', with p' = [y_d, v_d - vx0]
//           (set-points) or [x_f - x0 - vx0 t_f, y_f] (goal positions) and
//           b' = (ax0, y0, vy0, ay0); x is taken relative to x0 + vx0 t.
//   proj    inverse of A = N^T N + rho N^T (F^T F + G^T G) N (the xi-update
//           of Alg. 2, eq. split_xy, in the free coordinates), block diagonal
//           in x (8 x 8) and y (7 x 7), and D = diag(N^T N). With goal
//           positions the slots of c10 (x) and c9 = c10 (y) hold the goal:
//           they are fixed, so their rows and columns of the inverse and
//           their D are zero and the inverse is that of the reduced A.
//   mfma    the same basis and inverse as FP16 high/low pairs, laid out as
//           the per-lane operands of v_mfma_f32_16x16x16_f16 (reduced-
//           precision lower level).
#include "precompute.h"

#include <cmath>
#include <cstring>
#include <stdexcept>

namespace plan {

namespace {

constexpr int kDeg = 10;
constexpr int kNC = 11;

// Bernstein values of degree m at tau: b[0..m] (de Casteljau recurrence).
void bernstein(int m, double tau, double *b) {
  for (int i = 0; i <= m; ++i) b[i] = 0.0;
  b[0] = 1.0;
  for (int d = 1; d <= m; ++d) {
    for (int i = d; i >= 1; --i) b[i] = (1.0 - tau) * b[i] + tau * b[i - 1];
    b[0] = (1.0 - tau) * b[0];
  }
}

// Rows of W, Wd, Wdd at one instant via the derivative recurrence
// dB_i,n = n (B_i-1,n-1 - B_i,n-1).
void basis_row(double tau, double t_f, double *W, double *Wd, double *Wdd) {
  double b10[kNC], b9[kNC], b8[kNC];
  bernstein(kDeg, tau, b10);
  bernstein(kDeg - 1, tau, b9);
  bernstein(kDeg - 2, tau, b8);
  for (int i = 0; i <= kDeg; ++i) {
    W[i] = b10[i];
    double d1 = (i >= 1 ? b9[i - 1] : 0.0) - (i <= kDeg - 1 ? b9[i] : 0.0);
    Wd[i] = kDeg * d1 / t_f;
    double d2 = (i >= 2 ? b8[i - 2] : 0.0) - 2.0 * (i >= 1 && i - 1 <= kDeg - 2 ? b8[i - 1] : 0.0) +
                (i <= kDeg - 2 ? b8[i] : 0.0);
    Wdd[i] = kDeg * (kDeg - 1) * d2 / (t_f * t_f);
  }
}

// In-place inverse of a symmetric positive definite n x n matrix (Cholesky).
void spd_inverse(double *A, int n) {
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) throw std::runtime_error("matrix not positive definite");
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = s / L[j * n + j];
    }
  }
  // inverse columns: solve L L^T x = e_c
  std::vector<double> inv(n * n);
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
      y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * inv[k * n + c];
      inv[i * n + c] = s / L[i * n + i];
    }
  }
  std::memcpy(A, inv.data(), sizeof(double) * n * n);
}

// Free-coordinate selections: x free = c3..c10 (8); y free = c3..c8 and the
// shared value of c9 = c10 (ydot(t_f) = 0).
void null_x(double *Nx /* 11 x 8 */) {
  std::memset(Nx, 0, sizeof(double) * kNC * 8);
  for (int c = 0; c < 8; ++c) Nx[(3 + c) * 8 + c] = 1.0;
}
void null_y(double *Ny /* 11 x 7 */) {
  std::memset(Ny, 0, sizeof(double) * kNC * 7);
  for (int c = 0; c < 6; ++c) Ny[(3 + c) * 7 + c] = 1.0;
  Ny[9 * 7 + 6] = 1.0;
  Ny[10 * 7 + 6] = 1.0;
}

// v^T N for a row v of length 11.
template <int NF>
void project_row(const double *row, const double *Nm, double *out) {
  for (int c = 0; c < NF; ++c) {
    double s = 0.0;
    for (int i = 0; i < kNC; ++i) s += row[i] * Nm[i * NF + c];
    out[c] = s;
  }
}

}  // namespace

void build_basis(int T, double t_f, BasisTable &bt) {
  bt.T = T;
  bt.Tpad = (T + 63) / 64 * 64;
  bt.W.assign(T * kNC, 0.0);
  bt.Wd.assign(T * kNC, 0.0);
  bt.Wdd.assign(T * kNC, 0.0);
  for (int k = 0; k < T; ++k) {
    double tau = T > 1 ? (double)k / (double)(T - 1) : 0.0;
    basis_row(tau, t_f, &bt.W[k * kNC], &bt.Wd[k * kNC], &bt.Wdd[k * kNC]);
  }
  bt.table.assign((size_t)kBasisCols * bt.Tpad, 0.f);
  auto col = [&](int c) { return &bt.table[(size_t)c * bt.Tpad]; };
  for (int k = 0; k < T; ++k) {
    const double *W = &bt.W[k * kNC], *Wd = &bt.Wd[k * kNC], *Wdd = &bt.Wdd[k * kNC];
    for (int c = 0; c < 8; ++c) {
      col(kColW + c)[k] = (float)W[3 + c];
      col(kColWd + c)[k] = (float)Wd[3 + c];
      col(kColWdd + c)[k] = (float)Wdd[3 + c];
    }
    col(kColY7 + 0)[k] = (float)(W[9] + W[10]);
    col(kColY7 + 1)[k] = (float)(Wd[9] + Wd[10]);
    col(kColY7 + 2)[k] = (float)(Wdd[9] + Wdd[10]);
    for (int c = 0; c < 3; ++c) {
      col(kColFix + c)[k] = (float)W[c];
      col(kColFix + 3 + c)[k] = (float)Wd[c];
      col(kColFix + 6 + c)[k] = (float)Wdd[c];
    }
    col(kColT)[k] = (float)(t_f * (double)k / (double)(T - 1));
  }
}

// Step-1 QP with goal positions: minimise sum_k w_s (xddot_k^2 + yddot_k^2)
// over the coefficients left free by the initial conditions and the final
// boundary (x, y, ydot)(t_f) = (x_f, y_f, 0) (eq. final_boundary): x c3..c9
// (slots 0..6; slot 7 = c10 = x_f, relative), y c3..c8 (slots 8..13; slot
// 14 = c9 = c10 = y_f).
void build_step1_goals(const BasisTable &bt, const CostWeights &cw, double t_f, Step1Table &st) {
  const int T = bt.T;
  const double n = kDeg;
  st.S.assign(16 * 8, 0.0);
  st.R.assign(16 * 4, 0.0);
  // ---- x axis (relative frame): c0 = c1 = 0, c2 = ax0 t_f^2 / 90, c10 = p'0
  {
    double H[49] = {0}, gx2[7] = {0}, gx10[7] = {0};
    const double cfix2 = t_f * t_f / (n * (n - 1.0));
    for (int k = 0; k < T; ++k) {
      const double *Wdd = &bt.Wdd[k * kNC];
      double n1[7];
      for (int a = 0; a < 7; ++a) n1[a] = Wdd[3 + a];
      for (int a = 0; a < 7; ++a) {
        for (int b = 0; b < 7; ++b) H[a * 7 + b] += 2.0 * cw.w_s * n1[a] * n1[b];
        gx2[a] += 2.0 * cw.w_s * n1[a] * Wdd[2] * cfix2;
        gx10[a] += 2.0 * cw.w_s * n1[a] * Wdd[10];
      }
    }
    spd_inverse(H, 7);
    for (int a = 0; a < 7; ++a) {
      double s0 = 0.0, s2 = 0.0;
      for (int b = 0; b < 7; ++b) {
        s0 -= H[a * 7 + b] * gx10[b];
        s2 -= H[a * 7 + b] * gx2[b];
      }
      st.S[a * 8 + 0] = s0;
      st.R[a * 4 + 0] = s2;
    }
    st.S[7 * 8 + 0] = 1.0;
  }
  // ---- y axis: c0..c2 = E (y0, vy0, ay0), c9 = c10 = p'1
  {
    double E[kNC * 3] = {0};
    E[0 * 3 + 0] = 1.0;
    E[1 * 3 + 0] = 1.0;
    E[1 * 3 + 1] = t_f / n;
    E[2 * 3 + 0] = 1.0;
    E[2 * 3 + 1] = 2.0 * t_f / n;
    E[2 * 3 + 2] = t_f * t_f / (n * (n - 1.0));
    double H[36] = {0}, ge[6 * 3] = {0}, gf[6] = {0};
    for (int k = 0; k < T; ++k) {
      const double *Wdd = &bt.Wdd[k * kNC];
      double n1[6], e1[3] = {0, 0, 0};
      for (int a = 0; a < 6; ++a) n1[a] = Wdd[3 + a];
      for (int m = 0; m < 3; ++m)
        for (int i = 0; i < 3; ++i) e1[m] += Wdd[i] * E[i * 3 + m];
      for (int a = 0; a < 6; ++a) {
        for (int b = 0; b < 6; ++b) H[a * 6 + b] += 2.0 * cw.w_s * n1[a] * n1[b];
        for (int m = 0; m < 3; ++m) ge[a * 3 + m] += 2.0 * cw.w_s * n1[a] * e1[m];
        gf[a] += 2.0 * cw.w_s * n1[a] * (Wdd[9] + Wdd[10]);
      }
    }
    spd_inverse(H, 6);
    for (int a = 0; a < 6; ++a) {
      double s1 = 0.0, r[3] = {0, 0, 0};
      for (int b = 0; b < 6; ++b) {
        s1 -= H[a * 6 + b] * gf[b];
        for (int m = 0; m < 3; ++m) r[m] -= H[a * 6 + b] * ge[b * 3 + m];
      }
      st.S[(8 + a) * 8 + 1] = s1;
      for (int m = 0; m < 3; ++m) st.R[(8 + a) * 4 + 1 + m] = r[m];
    }
    st.S[14 * 8 + 1] = 1.0;
  }
  st.table.resize(kStep1Floats);
  for (int i = 0; i < 16 * 8; ++i) st.table[i] = (float)st.S[i];
  for (int i = 0; i < 16 * 4; ++i) st.table[16 * 8 + i] = (float)st.R[i];
}

// Step-1 QP (Alg. 1, Sec. II-C cost) reduced to the free coefficients:
// minimise sum_k w (a_k^T c - beta_k)^2 over c = N z + c_fix.
void build_step1(const BasisTable &bt, const CostWeights &cw, double t_f, bool goals, Step1Table &st) {
  if (goals) {
    build_step1_goals(bt, cw, t_f, st);
    return;
  }
  const int T = bt.T;
  double Nx[kNC * 8], Ny[kNC * 7];
  null_x(Nx);
  null_y(Ny);
  const double n = kDeg;
  // ---- x axis, relative to x0 + vx0 t: beta = k_p (v_d - vx0), c_fix = e2 ax0 t_f^2/90
  double Hx[64] = {0}, Sx[8 * 4] = {0}, rx[8] = {0};
  {
    double cfix2 = t_f * t_f / (n * (n - 1.0));  // per unit ax0
    for (int k = 0; k < T; ++k) {
      const double *Wd = &bt.Wd[k * kNC], *Wdd = &bt.Wdd[k * kNC];
      int seg = (4 * k) / T;
      double a1[kNC], a2[kNC];
      for (int i = 0; i < kNC; ++i) {
        a1[i] = Wdd[i];                 // c_s: xddot
        a2[i] = Wdd[i] + cw.k_p * Wd[i]; // c_v: xddot + k_p xdot
      }
      double n1[8], n2[8];
      project_row<8>(a1, Nx, n1);
      project_row<8>(a2, Nx, n2);
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) Hx[a * 8 + b] += 2.0 * (cw.w_s * n1[a] * n1[b] + cw.w_v * n2[a] * n2[b]);
      for (int a = 0; a < 8; ++a) {
        Sx[a * 4 + seg] += 2.0 * cw.w_v * cw.k_p * n2[a];
        rx[a] -= 2.0 * (cw.w_s * n1[a] * a1[2] + cw.w_v * n2[a] * a2[2]) * cfix2;
      }
    }
    spd_inverse(Hx, 8);
  }
  // ---- y axis: beta = k_p y_d, c_fix = E (y0, vy0, ay0)
  double Hy[49] = {0}, Sy[7 * 4] = {0}, Ry[7 * 3] = {0};
  {
    double E[kNC * 3] = {0};
    E[0 * 3 + 0] = 1.0;
    E[1 * 3 + 0] = 1.0;
    E[1 * 3 + 1] = t_f / n;
    E[2 * 3 + 0] = 1.0;
    E[2 * 3 + 1] = 2.0 * t_f / n;
    E[2 * 3 + 2] = t_f * t_f / (n * (n - 1.0));
    for (int k = 0; k < T; ++k) {
      const double *W = &bt.W[k * kNC], *Wd = &bt.Wd[k * kNC], *Wdd = &bt.Wdd[k * kNC];
      int seg = (4 * k) / T;
      double a1[kNC], a2[kNC];
      for (int i = 0; i < kNC; ++i) {
        a1[i] = Wdd[i];                                   // c_s: yddot
        a2[i] = Wdd[i] + cw.k_p * W[i] + cw.k_v * Wd[i];  // c_l
      }
      double n1[7], n2[7];
      project_row<7>(a1, Ny, n1);
      project_row<7>(a2, Ny, n2);
      double e1[3] = {0}, e2[3] = {0};
      for (int m = 0; m < 3; ++m)
        for (int i = 0; i < kNC; ++i) {
          e1[m] += a1[i] * E[i * 3 + m];
          e2[m] += a2[i] * E[i * 3 + m];
        }
      for (int a = 0; a < 7; ++a)
        for (int b = 0; b < 7; ++b) Hy[a * 7 + b] += 2.0 * (cw.w_s * n1[a] * n1[b] + cw.w_l * n2[a] * n2[b]);
      for (int a = 0; a < 7; ++a) {
        Sy[a * 4 + seg] += 2.0 * cw.w_l * cw.k_p * n2[a];
        for (int m = 0; m < 3; ++m) Ry[a * 3 + m] -= 2.0 * (cw.w_s * n1[a] * e1[m] + cw.w_l * n2[a] * e2[m]);
      }
    }
    spd_inverse(Hy, 7);
  }
  // S (16 x 8) on p' = [y_d(4), v_d - vx0 (4)], R (16 x 4) on b' = (ax0, y0, vy0, ay0)
  st.S.assign(16 * 8, 0.0);
  st.R.assign(16 * 4, 0.0);
  for (int a = 0; a < 8; ++a) {
    for (int m = 0; m < 4; ++m) {
      double s = 0.0;
      for (int b = 0; b < 8; ++b) s += Hx[a * 8 + b] * Sx[b * 4 + m];
      st.S[a * 8 + 4 + m] = s;
    }
    double s = 0.0;
    for (int b = 0; b < 8; ++b) s += Hx[a * 8 + b] * rx[b];
    st.R[a * 4 + 0] = s;
  }
  for (int a = 0; a < 7; ++a) {
    for (int m = 0; m < 4; ++m) {
      double s = 0.0;
      for (int b = 0; b < 7; ++b) s += Hy[a * 7 + b] * Sy[b * 4 + m];
      st.S[(8 + a) * 8 + m] = s;
    }
    for (int m = 0; m < 3; ++m) {
      double s = 0.0;
      for (int b = 0; b < 7; ++b) s += Hy[a * 7 + b] * Ry[b * 3 + m];
      st.R[(8 + a) * 4 + 1 + m] = s;
    }
  }
  st.table.resize(kStep1Floats);
  for (int i = 0; i < 16 * 8; ++i) st.table[i] = (float)st.S[i];
  for (int i = 0; i < 16 * 4; ++i) st.table[16 * 8 + i] = (float)st.R[i];
}

void build_proj(const BasisTable &bt, int M, double rho, bool goals, ProjTable &pt) {
  const int T = bt.T;
  double WtW[kNC * kNC] = {0}, DtD[kNC * kNC] = {0}, AtA[kNC * kNC] = {0};
  for (int k = 0; k < T; ++k)
    for (int i = 0; i < kNC; ++i)
      for (int j = 0; j < kNC; ++j) {
        WtW[i * kNC + j] += bt.W[k * kNC + i] * bt.W[k * kNC + j];
        DtD[i * kNC + j] += bt.Wd[k * kNC + i] * bt.Wd[k * kNC + j];
        AtA[i * kNC + j] += bt.Wdd[k * kNC + i] * bt.Wdd[k * kNC + j];
      }
  // H_x = M W^T W + Wd^T Wd + Wdd^T Wdd; H_y adds G^T G = 2 W^T W.
  double Hx[kNC * kNC], Hy[kNC * kNC];
  for (int i = 0; i < kNC * kNC; ++i) {
    Hx[i] = M * WtW[i] + DtD[i] + AtA[i];
    Hy[i] = (M + 2) * WtW[i] + DtD[i] + AtA[i];
  }
  double Nx[kNC * 8], Ny[kNC * 7];
  null_x(Nx);
  null_y(Ny);
  auto reduce = [&](const double *H, const double *Nm, int nf, double *Aout, double *Dout) {
    for (int a = 0; a < nf; ++a)
      for (int b = 0; b < nf; ++b) {
        double h = 0.0, nn = 0.0;
        for (int i = 0; i < kNC; ++i)
          for (int j = 0; j < kNC; ++j) h += Nm[i * nf + a] * H[i * kNC + j] * Nm[j * nf + b];
        for (int i = 0; i < kNC; ++i) nn += Nm[i * nf + a] * Nm[i * nf + b];
        Aout[a * nf + b] = nn + rho * h;
        if (a == b) Dout[a] = nn;
      }
  };
  // goal positions fix the last slot of each axis: the free set is the
  // first 7 (x) and 6 (y) columns of the selections
  const int fx = goals ? 7 : 8, fy = goals ? 6 : 7;
  double Nxr[kNC * 8], Nyr[kNC * 7];
  for (int i = 0; i < kNC; ++i) {
    for (int c = 0; c < fx; ++c) Nxr[i * fx + c] = Nx[i * 8 + c];
    for (int c = 0; c < fy; ++c) Nyr[i * fy + c] = Ny[i * 7 + c];
  }
  double Ax[64], Ay[49], Dx[8], Dy[7];
  reduce(Hx, Nxr, fx, Ax, Dx);
  reduce(Hy, Nyr, fy, Ay, Dy);
  spd_inverse(Ax, fx);
  spd_inverse(Ay, fy);
  pt.Ainv.assign(16 * 16, 0.0);
  pt.D.assign(16, 0.0);
  for (int a = 0; a < fx; ++a) {
    for (int b = 0; b < fx; ++b) pt.Ainv[a * 16 + b] = Ax[a * fx + b];
    pt.D[a] = Dx[a];
  }
  for (int a = 0; a < fy; ++a) {
    for (int b = 0; b < fy; ++b) pt.Ainv[(8 + a) * 16 + 8 + b] = Ay[a * fy + b];
    pt.D[8 + a] = Dy[a];
  }
  pt.table.resize(kProjFloats);
  for (int i = 0; i < 256; ++i) pt.table[i] = (float)pt.Ainv[i];
  for (int i = 0; i < 16; ++i) pt.table[256 + i] = (float)pt.D[i];
}

namespace {

// FP16 bits of v rounded to nearest, and of the rounded remainder.
uint16_t half_bits(double v) {
  const _Float16 h = (_Float16)v;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
void split_half(double v, uint16_t &hi, uint16_t &lo) {
  const _Float16 h = (_Float16)v;
  std::memcpy(&hi, &h, 2);
  lo = half_bits(v - (double)h);
}

// Basis value of free coefficient c of an axis (x: c3..c10; y: c3..c8, then
// c9 + c10; anything else 0) for derivative order q at instant t.
double free_basis(const BasisTable &bt, bool y_axis, int q, int t, int c) {
  if (q > 2 || t >= bt.T || c < 0) return 0.0;  // beyond the horizon: zero
  const std::vector<double> &B = q == 0 ? bt.W : (q == 1 ? bt.Wd : bt.Wdd);
  const double *row = &B[(size_t)t * kNC];
  if (!y_axis) return c < 8 ? row[3 + c] : 0.0;
  if (c < 6) return row[3 + c];
  if (c == 6) return row[9] + row[10];
  return 0.0;
}

}  // namespace

void build_mfma_basis(const BasisTable &bt, std::vector<uint16_t> &ops) {
  const int NI = 4 * ((bt.T + 3) / 4);
  ops.assign((size_t)NI * kEvInstHalfs, 0);
  for (int t = 0; t < NI; ++t)
    for (int ax = 0; ax < 2; ++ax)
      for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 8; ++c) {
          uint16_t *e = &ops[(size_t)t * kEvInstHalfs + ax * kEvAxisHalfs + q * 16];
          split_half(t < bt.T ? free_basis(bt, ax == 1, q, t, c) : 0.0, e[c], e[8 + c]);
        }
}

void build_mfma32_basis(const BasisTable &bt, std::vector<uint16_t> &ops) {
  const int NI = 4 * ((bt.T + 3) / 4);
  std::vector<float> tab((size_t)NI * kEv32InstFloats, 0.f);
  for (int t = 0; t < NI && t < bt.T; ++t)
    for (int q = 0; q < 3; ++q)
      for (int g = 0; g < 4; ++g) {
        float *e = &tab[(size_t)t * kEv32InstFloats + q * 16 + g * 4];
        e[0] = (float)free_basis(bt, false, q, t, g);
        e[1] = (float)free_basis(bt, false, q, t, 4 + g);
        e[2] = (float)free_basis(bt, true, q, t, g);
        e[3] = (float)free_basis(bt, true, q, t, 4 + g);
      }
  ops.assign(tab.size() * 2, 0);
  std::memcpy(ops.data(), tab.data(), tab.size() * sizeof(float));
}

void build_mfma_inverse(const ProjTable &pt, std::vector<uint16_t> &ops) {
  ops.assign(2 * 64 * 4, 0);
  for (int lane = 0; lane < 64; ++lane)
    for (int u = 0; u < 4; ++u) {
      const int i = lane % 16, k = 4 * (lane / 16) + u;
      split_half(kAinvScale * pt.Ainv[i * 16 + k], ops[(0 * 64 + lane) * 4 + u], ops[(1 * 64 + lane) * 4 + u]);
    }
}


size_t dec_frag_half(int r, int k, int K) {
  return ((((size_t)(r >> 4) * (K >> 5) + (k >> 5)) * 64 + (r & 15) + 16 * ((k >> 3) & 3)) << 3) + (k & 7);
}

const char *build_decoder(const plan_decoder &dec, DecoderTables &t) {
  static const int n_in[6] = {kDecIn, kDecHidden, kDecHidden, kDecHidden, kDecHidden, kDecHidden5};
  static const int n_out[6] = {kDecHidden, kDecHidden, kDecHidden, kDecHidden, kDecHidden5, PLAN_NP};
  auto finite = [](const double *v, size_t n) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(v[i])) return false;
    return true;
  };
  if (!std::isfinite(dec.bn_eps) || dec.bn_eps < 0) return "bn_eps must be finite and >= 0";
  for (int i = 0; i < 6; ++i) {
    if (!dec.W[i] || !dec.b[i]) return "decoder weights missing";
    if (!finite(dec.W[i], (size_t)n_out[i] * n_in[i]) || !finite(dec.b[i], n_out[i]))
      return "non-finite decoder weights";
    if (i == 5) break;
    if (!dec.bn_gamma[i] || !dec.bn_beta[i] || !dec.bn_mean[i] || !dec.bn_var[i]) return "BatchNorm arrays missing";
    if (!finite(dec.bn_gamma[i], n_out[i]) || !finite(dec.bn_beta[i], n_out[i]) ||
        !finite(dec.bn_mean[i], n_out[i]) || !finite(dec.bn_var[i], n_out[i]))
      return "non-finite BatchNorm arrays";
    for (int n = 0; n < n_out[i]; ++n)
      if (!(dec.bn_var[i][n] + dec.bn_eps > 0)) return "BatchNorm var + eps must be > 0";
  }
  // folded block i: W' (out x in) and shift, FP64
  auto fold = [&](int i, std::vector<double> &Wf, std::vector<double> &sh) {
    Wf.assign((size_t)n_out[i] * n_in[i], 0.0);
    sh.assign(n_out[i], 0.0);
    for (int n = 0; n < n_out[i]; ++n) {
      const double sc = dec.bn_gamma[i][n] / std::sqrt(dec.bn_var[i][n] + dec.bn_eps);
      for (int k = 0; k < n_in[i]; ++k) Wf[(size_t)n * n_in[i] + k] = sc * dec.W[i][(size_t)n * n_in[i] + k];
      sh[n] = sc * (dec.b[i][n] - dec.bn_mean[i][n]) + dec.bn_beta[i][n];
    }
  };
  std::vector<double> Wf, sh;
  for (int i = 0; i < kDecLayers; ++i) {
    fold(i, Wf, sh);
    double mx = 0.0;
    for (double v : Wf) mx = std::max(mx, std::fabs(v));
    if (mx > 1e30 || (mx > 0 && mx < 1e-30)) return "decoder weights out of range";
    const int e = mx > 0 ? -((int)std::floor(std::log2(mx)) + 1) : 0;
    const double s2 = std::ldexp(1.0, e);
    const int kin = i == 0 ? kDecInPad : n_in[i];
    t.w_hi[i].assign((size_t)n_out[i] * kin, 0);
    t.w_lo[i].assign((size_t)n_out[i] * kin, 0);
    for (int n = 0; n < n_out[i]; ++n)
      for (int k = 0; k < n_in[i]; ++k) {
        const size_t q = dec_frag_half(n, k, kin);
        split_half(Wf[(size_t)n * n_in[i] + k] * s2, t.w_hi[i][q], t.w_lo[i][q]);
      }
    t.shift[i].assign(sh.begin(), sh.end());
    t.inv_scale[i] = (float)std::ldexp(1.0, -e);
  }
  t.w6.assign((size_t)PLAN_NP * kDecHidden5, 0.f);
  t.b6.assign(PLAN_NP, 0.f);
  for (int a = 0; a < PLAN_NP; ++a) {
    for (int k = 0; k < kDecHidden5; ++k) t.w6[(size_t)a * kDecHidden5 + k] = (float)dec.W[5][(size_t)a * kDecHidden5 + k];
    t.b6[a] = (float)dec.b[5][a];
  }
  return nullptr;
}

}  // namespace plan
