// precompute.h -- host FP64 construction of the per-T and per-(T, M) tables.
#pragma once

#include <cstdint>
#include <vector>

#include "plan_internal.h"

namespace plan {

struct CostWeights {
  double k_p, k_v, w_s, w_l, w_v;
};

struct BasisTable {
  int T = 0, Tpad = 0;
  std::vector<double> W, Wd, Wdd;  // T x 11 (FP64)
  std::vector<float> table;        // kBasisCols x Tpad (FP32, device layout)
};

struct Step1Table {
  std::vector<double> S, R;        // 16 x 8, 16 x 4 (FP64)
  std::vector<float> table;        // kStep1Floats
};

struct ProjTable {
  std::vector<double> Ainv, D;     // 16 x 16 block diagonal, 16
  std::vector<float> table;        // kProjFloats
};

void build_basis(int T, double t_f, BasisTable &bt);
// goals: behavioural inputs are goal positions (final boundary rows, cost
// c_s alone); the free slots 7 (c10 of x) and 14 (c9 = c10 of y) are then
// fixed by the goal and the inverse acts on the other 13.
void build_step1(const BasisTable &bt, const CostWeights &cw, double t_f, bool goals, Step1Table &st);
void build_proj(const BasisTable &bt, int M, double rho, bool goals, ProjTable &pt);

// FP16 bit patterns of the tables of the matrix-core lower level:
//   basis   [4 ceil(T/4)][kEvInstHalfs] (layout in plan_internal.h)
//   inverse [2][64 lanes][4]: high then low half of kAinvScale * A^-1 in the
//           A-operand lane order of v_mfma_f32_16x16x16_f16
void build_mfma_basis(const BasisTable &bt, std::vector<uint16_t> &ops);
void build_mfma_inverse(const ProjTable &pt, std::vector<uint16_t> &ops);

}  // namespace plan
