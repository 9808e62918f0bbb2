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
// The FP32 matrix-core form of the same table (kEv32InstFloats floats per
// instant, layout in plan_internal.h), returned as the FP16-sized words of
// its bytes so both forms share one device region.
void build_mfma32_basis(const BasisTable &bt, std::vector<uint16_t> &ops);
void build_mfma_inverse(const ProjTable &pt, std::vector<uint16_t> &ops);

// Device tables of the decoder sampler: each block's BatchNorm (inference
// form) and bias folded into its Linear layer in FP64,
//   W' = diag(gamma / sqrt(var + eps)) W,
//   shift = gamma (b - mean) / sqrt(var + eps) + beta,
// blocks 1-5 as FP16 high/low pairs of W' 2^e (e per layer, so that
// max |W' 2^e| lies in [1/2, 1)) with inv_scale = 2^-e, block 1 with its 57
// inputs padded to kDecInPad by zero columns; the output layer in FP32.
// Returns nullptr, or why the weights are refused.
// Weights are stored in the matrix-core operand layout of the decoder
// kernels: half (r, k) of an R x K matrix at dec_frag_half(r, k, K), 16 x 32
// fragments in the order one wave's loads read them.
size_t dec_frag_half(int r, int k, int K);
struct DecoderTables {
  std::vector<uint16_t> w_hi[kDecLayers], w_lo[kDecLayers];  // out x in, fragment layout
  std::vector<float> shift[kDecLayers];
  float inv_scale[kDecLayers];
  std::vector<float> w6, b6;                // PLAN_NP x kDecHidden5, PLAN_NP
};
const char *build_decoder(const plan_decoder &dec, DecoderTables &t);

}  // namespace plan
