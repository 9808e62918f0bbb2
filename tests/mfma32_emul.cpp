// CPU emulation of the FP32 matrix-core lower level's tables and dataflow.
//
// Builds the FP32 basis table with the library's own host code, then runs
// the kernel's dataflow with software models of
//   * v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
//     B[l / 16][l % 16]; element u of lane l returns D[4 (l / 16) + u][l % 16];
//   * v_permlane32_swap (a, b): a's upper 32 lanes and b's lower 32 lanes
//     trade places; v_permlane16_swap (a, b): a's odd 16-lane rows and b's
//     even rows trade places,
// with the kernel's per-lane table offsets and its transpose of the
// coefficients across lane groups, and compares
//   * the trajectory evaluation of 16 samples at every instant,
//   * the sums N^T g over the horizon,
//   * the xi-update A^-1 rhs (A^-1 from the FP32 projection table)
// with the same quantities in FP64. Prints the largest errors; exits
// non-zero if one exceeds its bound.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "precompute.h"

using namespace plan;

namespace {

using Reg = float[64];  // one VGPR of a wave

// D = C + A B for one wave; products and sums in FP64, then rounded (the
// hardware's FP32 rounding differs in the last bit at most per step).
void mma(const Reg &A, const Reg &B, float (&C)[64][4]) {
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      double s = C[j + 16 * (i / 4)][i % 4];
      for (int k = 0; k < 4; ++k) s += (double)A[i + 16 * k] * (double)B[j + 16 * k];
      C[j + 16 * (i / 4)][i % 4] = (float)s;
    }
}

void swap32(Reg &a, Reg &b) {
  for (int l = 0; l < 32; ++l) std::swap(a[l + 32], b[l]);
}
void swap16(Reg &a, Reg &b) {
  for (int r = 0; r < 4; r += 2)
    for (int i = 0; i < 16; ++i) std::swap(a[16 * (r + 1) + i], b[16 * r + i]);
}

// The kernel's transpose_groups on a 4-register value.
void transpose_groups(const float (&in)[64][4], Reg (&out)[4]) {
  for (int u = 0; u < 4; ++u)
    for (int l = 0; l < 64; ++l) out[u][l] = in[l][u];
  swap32(out[0], out[2]);
  swap32(out[1], out[3]);
  swap16(out[0], out[1]);
  swap16(out[2], out[3]);
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
  std::vector<uint16_t> words;
  build_mfma32_basis(bt, words);
  const int NT = (T + 3) / 4;
  if (words.size() != (size_t)4 * NT * kEv32InstFloats * 2 || pt.table.size() != (size_t)kProjFloats) {
    std::printf("table sizes wrong\n");
    return 2;
  }
  std::vector<float> tab(words.size() / 2);
  std::memcpy(tab.data(), words.data(), tab.size() * 4);
  std::mt19937_64 rng(11);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double z[16][16];
  std::vector<double> d((size_t)16 * 4 * NT * 6, 0.0);  // [n][t][x q, y q]
  auto D = [&](int n, int t, int k) -> double & { return d[((size_t)n * 4 * NT + t) * 6 + k]; };
  for (int n = 0; n < 16; ++n) {
    for (int c = 0; c < 8; ++c) z[n][c] = (float)(80.0 * U(rng));
    for (int c = 8; c < 15; ++c) z[n][c] = (float)(7.0 * U(rng));
    z[n][15] = 0.0;
  }
  // state layout: lane (n, g) holds coefficients 4g..4g+3 of sample n
  float zl[64][4];
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) zl[l][u] = (float)z[l % 16][4 * (l / 16) + u];
  Reg bz[4];
  transpose_groups(zl, bz);
  // the transpose itself: lane (n, g), register u holds coefficient 4u + g
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u)
      if (bz[u][l] != (float)z[l % 16][4 * u + l / 16]) {
        std::printf("transpose wrong at lane %d register %d\n", l, u);
        return 1;
      }
  double err_eval = 0.0, scale_eval = 0.0;
  float acc[64][4] = {};
  for (int tile = 0; tile < NT; ++tile) {
    const float *base = tab.data() + (size_t)tile * 4 * kEv32InstFloats;
    Reg a[4];
    for (int l = 0; l < 64; ++l) {
      const int n = l % 16, g = l / 16;
      const int ev32 = (n >> 2) * kEv32InstFloats + std::min(n & 3, 2) * 16 + 4 * g;
      for (int e = 0; e < 4; ++e) a[e][l] = base[ev32 + e];
    }
    float ex[64][4] = {}, ey[64][4] = {};
    mma(a[0], bz[0], ex);
    mma(a[1], bz[1], ex);
    mma(a[2], bz[2], ey);
    mma(a[3], bz[3], ey);
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
    // corrections at this tile's instants (zero beyond the horizon): lane
    // (n, g) holds (dx q0..2, dy q0..2) at instant 4 tile + g
    Reg dv[6], ax[3], ay[3];
    for (int l = 0; l < 64; ++l) {
      const int n = l % 16, g = l / 16, t = 4 * tile + g;
      for (int k = 0; k < 6; ++k) {
        const float v = t < T ? (float)(3.0 * U(rng)) : 0.f;
        dv[k][l] = v;
        if (t < T) D(n, t, k) = v;
      }
      const int acx32 = g * kEv32InstFloats + (n < 8 ? (n & 3) * 4 + (n >> 2) : 15);
      const int acy32 = g * kEv32InstFloats + (n >= 8 ? ((n - 8) & 3) * 4 + 2 + ((n - 8) >> 2) : 15);
      for (int q = 0; q < 3; ++q) {
        ax[q][l] = base[acx32 + 16 * q];
        ay[q][l] = base[acy32 + 16 * q];
      }
    }
    for (int q = 0; q < 3; ++q) mma(ax[q], dv[q], acc);
    for (int q = 0; q < 3; ++q) mma(ay[q], dv[3 + q], acc);
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
  // xi-update: A^-1 row n, columns 4 kb + g from the FP32 projection table;
  // rhs transposed across the lane groups
  double rhs[16][16];
  float rl[64][4];
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) {
      const int n = l % 16, c = 4 * (l / 16) + u;
      rhs[n][c] = c < 15 ? (float)(500.0 * U(rng)) : 0.0;
      rl[l][u] = (float)rhs[n][c];
    }
  Reg rt[4], ai[4];
  transpose_groups(rl, rt);
  for (int l = 0; l < 64; ++l)
    for (int kb = 0; kb < 4; ++kb) ai[kb][l] = pt.table[(l % 16) * 16 + 4 * kb + l / 16];
  float dz[64][4] = {};
  for (int kb = 0; kb < 4; ++kb) mma(ai[kb], rt[kb], dz);
  double err_upd = 0.0, scale_upd = 0.0;
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u) {
      const int n = l % 16, c = 4 * (l / 16) + u;
      double r = 0.0;
      for (int k = 0; k < 16; ++k) r += pt.Ainv[c * 16 + k] * rhs[n][k];
      err_upd = std::max(err_upd, std::fabs(dz[l][u] - r));
      scale_upd = std::max(scale_upd, std::fabs(r));
    }
  const double rel_eval = err_eval / scale_eval, rel_acc = err_acc / scale_acc, rel_upd = err_upd / scale_upd;
  std::printf("T=%d M=%d eval max|err| %.3e (rel %.2e)  N^T g %.3e (rel %.2e)  A^-1 rhs %.3e (rel %.2e)\n", T, M,
              err_eval, rel_eval, err_acc, rel_acc, err_upd, rel_upd);
  // FP32 operands (tables rounded once) and FP32 sums: relative errors ~1e-7
  const bool ok = rel_eval < 2e-6 && rel_acc < 2e-6 && rel_upd < 2e-6;
  return ok ? 0 : 1;
}
