// CPU emulation of the matrix-core lower level's tables and dataflow.
//
// Builds the FP16 high/low tables with the library's own host code, then runs
// the kernel's dataflow with a software model of the wave64 MFMA
// instructions (16x16x16 and 16x16x32 f16: lane l supplies K/4 elements of A
// row l % 16 and of B column l % 16; element u of lane l pairs with element
// u of every lane in the same 16-lane group; D row 4 (l / 16) + u, column
// l % 16 comes back in lane l) and compares
//   * the trajectory evaluation of 16 samples at every instant,
//   * the sums N^T g over the horizon,
//   * the xi-update A^-1 rhs
// with the same quantities in FP64. The per-lane table offsets are the
// kernel's. Prints the largest errors; exits non-zero if one exceeds its bound.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "precompute.h"

using namespace plan;

namespace {

float half_to_float(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (float)h;
}
uint16_t float_to_half(float v) {
  const _Float16 h = (_Float16)v;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

// Split of the kernel: hi = v cut to 11 significant bits, lo = rest rounded.
void split(float v, uint16_t &hi, uint16_t &lo) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  u &= 0xFFFFE000u;
  float h;
  std::memcpy(&h, &u, 4);
  hi = float_to_half(h);
  lo = float_to_half(v - h);
}

template <int KL>
struct Lanes {
  uint16_t v[64][KL];
};

// D = C + A B for one wave: element u of lane 16 g + i (A) pairs with element
// u of lane 16 g + j (B); products exact, sums in FP64 then rounded.
template <int KL>
void mma(const Lanes<KL> &A, const Lanes<KL> &B, float (&C)[64][4]) {
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      double s = C[j + 16 * (i / 4)][i % 4];
      for (int g = 0; g < 4; ++g)
        for (int u = 0; u < KL; ++u)
          s += (double)half_to_float(A.v[i + 16 * g][u]) * (double)half_to_float(B.v[j + 16 * g][u]);
      C[j + 16 * (i / 4)][i % 4] = (float)s;
    }
}

// The kernel's coef_operands: split the lane's 4 coefficients, then swap the
// upper half-wave of the high halves with the lower half-wave of the low.
void coef_operands(const float (&z)[64][4], Lanes<4> &bx, Lanes<4> &by) {
  Lanes<4> hi, lo;
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) split(z[l][u], hi.v[l][u], lo.v[l][u]);
  bx = hi;
  by = lo;
  for (int l = 0; l < 32; ++l)
    for (int u = 0; u < 4; ++u) {
      bx.v[l + 32][u] = lo.v[l][u];
      by.v[l][u] = hi.v[l + 32][u];
    }
}

double free_basis(const BasisTable &bt, bool y, int q, int t, int c) {
  const std::vector<double> &B = q == 0 ? bt.W : (q == 1 ? bt.Wd : bt.Wdd);
  const double *row = &B[(size_t)t * 11];
  if (!y) return c < 8 ? row[3 + c] : 0.0;
  if (c < 6) return row[3 + c];
  if (c == 6) return row[9] + row[10];
  return 0.0;
}

}  // namespace

int main(int argc, char **argv) {
  const int T = argc > 1 ? std::atoi(argv[1]) : 100;
  const int M = argc > 2 ? std::atoi(argv[2]) : 10;
  const double t_f = 5.0;
  BasisTable bt;
  build_basis(T, t_f, bt);
  ProjTable pt;
  build_proj(bt, M, 1.0, false, pt);
  std::vector<uint16_t> tab, inv;
  build_mfma_basis(bt, tab);
  build_mfma_inverse(pt, inv);
  const int NT = (T + 3) / 4;
  if (tab.size() != (size_t)4 * NT * kEvInstHalfs || inv.size() != 2 * 64 * 4) {
    std::printf("table sizes wrong\n");
    return 2;
  }
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  // 16 samples: coefficients of the size the planner sees (x relative to the
  // reference line up to ~80 m, y within the road), corrections up to a few m.
  double z[16][16];
  std::vector<double> d((size_t)16 * 4 * NT * 6, 0.0);  // [n][t][x q, y q]
  auto D = [&](int n, int t, int k) -> double & { return d[((size_t)n * 4 * NT + t) * 6 + k]; };
  for (int n = 0; n < 16; ++n) {
    for (int c = 0; c < 8; ++c) z[n][c] = 80.0 * U(rng);
    for (int c = 8; c < 15; ++c) z[n][c] = 7.0 * U(rng);
    z[n][15] = 0.0;
  }
  // state layout: lane (n, g) holds coefficients 4g..4g+3 of sample n
  float zl[64][4];
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) zl[l][u] = (float)z[l % 16][4 * (l / 16) + u];
  Lanes<4> bx, by;
  coef_operands(zl, bx, by);
  // operands as the kernel reads them (offsets in halves)
  auto ev_op = [&](int tile, int axis, int half) {
    Lanes<4> L;
    for (int l = 0; l < 64; ++l) {
      const int n = l % 16, g = l / 16;
      const int off = (n >> 2) * kEvInstHalfs + std::min(n & 3, 2) * 16 + 4 * (g & 1);
      for (int u = 0; u < 4; ++u)
        L.v[l][u] = tab[(size_t)tile * 4 * kEvInstHalfs + off + axis * kEvAxisHalfs + half * 8 + u];
    }
    return L;
  };
  auto ac_op = [&](int tile, int half) {
    Lanes<8> L;
    for (int l = 0; l < 64; ++l) {
      const int n = l % 16, g = l / 16;
      const int ac_x = g * kEvInstHalfs + (n < 8 ? n : kEvPad);
      const int ac_y = g * kEvInstHalfs + (n >= 8 && n < 15 ? kEvAxisHalfs + (n - 8) : kEvPad);
      const int sx = n < 8 ? 16 : 0, sy = n >= 8 && n < 15 ? 16 : 0;
      const size_t b = (size_t)tile * 4 * kEvInstHalfs + half * 8;
      const uint16_t v[8] = {tab[b + ac_x], tab[b + ac_x + sx], tab[b + ac_x + 2 * sx], 0,
                             tab[b + ac_y], tab[b + ac_y + sy], tab[b + ac_y + 2 * sy], 0};
      for (int u = 0; u < 8; ++u) L.v[l][u] = v[u];
    }
    return L;
  };
  double err_eval = 0.0, scale_eval = 0.0;
  float acc[64][4] = {};
  for (int tile = 0; tile < NT; ++tile) {
    float ex[64][4] = {}, ey[64][4] = {};
    mma(ev_op(tile, 0, 0), bx, ex);
    mma(ev_op(tile, 0, 1), bx, ex);
    mma(ev_op(tile, 1, 0), by, ey);
    mma(ev_op(tile, 1, 1), by, ey);
    for (int l = 0; l < 64; ++l) {
      const int n = l % 16, g = l / 16, t = 4 * tile + g;
      for (int q = 0; q < 3; ++q) {
        double rx = 0.0, ry = 0.0;
        if (t < T)
          for (int c = 0; c < 8; ++c) {
            rx += free_basis(bt, false, q, t, c) * z[n][c];
            ry += free_basis(bt, true, q, t, c) * z[n][8 + c];
          }
        err_eval = std::max(err_eval, std::max(std::fabs(ex[l][q] - rx), std::fabs(ey[l][q] - ry)));
        scale_eval = std::max(scale_eval, std::max(std::fabs(rx), std::fabs(ry)));
      }
    }
    // corrections at this tile's instants (zero beyond the horizon) as the
    // B operand: lane (n, g) holds (dx q0..2, 0, dy q0..2, 0) at 4 tile + g
    Lanes<8> dh, dlo;
    for (int l = 0; l < 64; ++l) {
      const int n = l % 16, g = l / 16, t = 4 * tile + g;
      for (int u = 0; u < 8; ++u) {
        const int q = u % 4;
        double v = 0.0;
        if (t < T && q < 3) {
          v = 3.0 * U(rng);
          D(n, t, (u < 4 ? 0 : 3) + q) = (float)v;
        }
        split((float)v, dh.v[l][u], dlo.v[l][u]);
      }
    }
    const Lanes<8> ch = ac_op(tile, 0), cl = ac_op(tile, 1);
    mma(ch, dh, acc);
    mma(ch, dlo, acc);
    mma(cl, dh, acc);
  }
  double err_acc = 0.0, scale_acc = 0.0;
  for (int l = 0; l < 64; ++l) {
    const int n = l % 16, g = l / 16;
    for (int u = 0; u < 4; ++u) {
      const int c = 4 * g + u;
      double r = 0.0;
      for (int t = 0; t < T; ++t)
        for (int q = 0; q < 3; ++q)
          r += c < 8 ? free_basis(bt, false, q, t, c) * D(n, t, q)
                     : (c < 15 ? free_basis(bt, true, q, t, c - 8) * D(n, t, 3 + q) : 0.0);
      err_acc = std::max(err_acc, std::fabs(acc[l][u] - r));
      scale_acc = std::max(scale_acc, std::fabs(r));
    }
  }
  // xi-update: dz = A^-1 rhs with the kernel's scalings
  double rhs[16][16];
  Lanes<4> rh, rl, aih, ail;
  std::memcpy(aih.v, &inv[0], sizeof(aih.v));
  std::memcpy(ail.v, &inv[64 * 4], sizeof(ail.v));
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) {
      const int n = l % 16, c = 4 * (l / 16) + u;
      rhs[n][c] = c < 15 ? 500.0 * U(rng) : 0.0;
      split((float)rhs[n][c] * kRhsScale, rh.v[l][u], rl.v[l][u]);
    }
  float dz[64][4] = {};
  mma(aih, rh, dz);
  mma(aih, rl, dz);
  mma(ail, rh, dz);
  double err_upd = 0.0, scale_upd = 0.0;
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) {
      const int n = l % 16, c = 4 * (l / 16) + u;
      double r = 0.0;
      for (int k = 0; k < 16; ++k) r += pt.Ainv[c * 16 + k] * rhs[n][k];
      const double got = (double)dz[l][u] / (kAinvScale * kRhsScale);
      err_upd = std::max(err_upd, std::fabs(got - r));
      scale_upd = std::max(scale_upd, std::fabs(r));
    }
  const double rel_eval = err_eval / scale_eval, rel_acc = err_acc / scale_acc, rel_upd = err_upd / scale_upd;
  std::printf("T=%d M=%d eval max|err| %.3e (rel %.2e)  N^T g %.3e (rel %.2e)  A^-1 rhs %.3e (rel %.2e)\n", T, M,
              err_eval, rel_eval, err_acc, rel_acc, err_upd, rel_upd);
  // about 22 significant bits per operand: relative errors a few 1e-7
  const bool ok = rel_eval < 4e-6 && rel_acc < 4e-6 && rel_upd < 4e-6;
  return ok ? 0 : 1;
}
