// plan_internal.h -- layouts shared by the host engine and the HIP kernels of
// the batched bi-level planner (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/plan.h"

namespace plan {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // lower kernel: 4 waves
constexpr int kSelBlock = 256;       // selection / update kernel (4 waves)
constexpr int kZ = 16;               // free coefficients (8 x + 7 y) padded
constexpr int kBasisCols = 37;       // columns of the per-T basis table
constexpr int kStep1Floats = 16 * 8 + 16 * 4;
constexpr int kProjFloats = 16 * 16 + 16;
constexpr int kMaxCes = 1024;        // LDS bound of the ConstraintEliteSet
constexpr int kMaxEs = 256;          // LDS bound of the EliteSet
// Far entries after the vector-ALU kernel's neighbour table: its lanes read
// their slots' instants unclamped, up to 64 IPL ceil(T / (64 IPL)) - 1 < T + 128.
constexpr int kObsPad = 128;
// Matrix-core (FP16 high/low) lower level.
constexpr int kMfmaMaxT = 128;       // horizon limit of the matrix-core kernel
constexpr int kMfmaMaxPairs = kMfmaMaxT / 8;  // pairs of 4-instant tiles
constexpr int kMfmaSamples = 16;     // samples per workgroup (the MFMA N dimension)
constexpr double kAinvScale = 256.0; // A^-1 is stored times this (exact power of two)
constexpr float kRhsScale = 1.0f / 16.0f;  // the xi-update right-hand side is split times this

// Columns of the per-T basis table (each column holds Tpad floats):
//   0..7   W[:, 3..10]     8..15 Wd[:, 3..10]     16..23 Wdd[:, 3..10]
//   24     W9 + W10        25    Wd9 + Wd10       26     Wdd9 + Wdd10
//   27..29 W[:, 0..2]      30..32 Wd[:, 0..2]     33..35 Wdd[:, 0..2]
//   36     t_k
enum BasisCol {
  kColW = 0, kColWd = 8, kColWdd = 16, kColY7 = 24, kColFix = 27, kColT = 36
};

// Basis table of the matrix-core lower level, per instant t (padded to a
// multiple of 4 instants, zero beyond T), in FP16 halves:
//   [axis x, y][q = position, velocity, acceleration][hi 0..7 | lo 8..15]
// over the 8 free coefficients of the axis (x: c3..c10; y: c3..c8, c9 + c10,
// 0), then a zero pad of 16 halves and 8 unused ones (the stride of 60
// dwords per instant spreads both read patterns over the LDS banks: 3%
// faster than 56). v = hi + lo to about 22 bits.
constexpr int kEvAxisHalfs = 48;          // 3 orders x 16
constexpr int kEvPad = 96;                // offset of the zero pad
constexpr int kEvInstHalfs = 120;         // halves per instant (240 bytes; the 8-half gap spreads LDS banks)
// Basis table of the FP32 matrix-core lower level, per instant t (padded to
// a multiple of 4 instants, zero beyond T), in FP32:
//   [q = position, velocity, acceleration][g = 0..3]
//     (x c_g, x c_{4+g}, y c_g, y c_{4+g})
// over the same 8 free coefficients per axis (x: c3..c10; y: c3..c8,
// c9 + c10, 0): one float4 per (instant, order, lane group).
constexpr int kEv32InstFloats = 48;       // floats per instant (192 bytes)
// How iteration 0 draws its samples.
enum InitMode : int32_t {
  kInitStructured = 0,  // structured initial sampler (lanes + uniform speeds)
  kInitGiven = 1,       // N(mu0, Sigma0) supplied with the request
  kInitSession = 2,     // N(mu, Sigma) stored for the session on the device
  kInitForced = 3       // samples uploaded by the caller (lower-level only)
};

// Device-resident descriptor of one request slot.
struct ReqDesc {
  int32_t T, M, N, n_ces, n_es;
  int32_t t_idx;     // index into the per-T tables
  int32_t tm_idx;    // index into the per-(T, M) tables
  int32_t basis_off;  // float offset of the basis table of t_idx (copied at staging,
  int32_t basis_tpad; //   so the kernels reach the table without another load)
  int32_t mops_off;   // FP16 offset of the matrix-core table of t_idx, or 0
  int32_t init_mode; // InitMode
  int32_t session;    // session store index read at iteration 0, or -1
  int32_t session_wb; // session store index written after the last update, or -1
  int32_t first_iter; // upper-iteration index of the first iteration (sample stream)
  int32_t cur_iter;   // next upper iteration of this request (served mode)
  int64_t row_off;    // first row of this request in the sample-row pool
  uint64_t seed;
  double ego[6];     // x0, y0, vx0, vy0, ax0, ay0
  double kappa;
  double mu0[8];
  double sigma0[64];
  double obs[PLAN_MAX_M][4];
  int32_t n_road;    // road profile: 0 = constant kappa and lane limits
  double road_x0, road_dx;
  double road[PLAN_MAX_ROAD][3];  // kappa, y_lb, y_ub per knot
  double obsv[PLAN_OBS_DIM];      // observation of the decoder sampler
};

// Sampling distribution of one slot (FP64).
struct DistState {
  double mu[8];
  double sigma[64];
  double chol[64];
};

// Result record of one slot (FP64). cost_upper and residual are those of
// the returned trajectory xi, evaluated in FP64.
struct ResultRec {
  int32_t status;
  uint32_t flags;
  int32_t best;
  int32_t iterations;
  double p[8];
  double xi[22];
  double cost_upper;
  double residual;
};

// Scalars of the method (from plan_config), FP64 on the host, passed by value.
struct MethodParams {
  double t_f, rho, ell_a, ell_b;
  double v_min, v_max, a_max, kappa_max, c_max, y_lb, y_ub, v_eps;
  double eta, gamma, cov_jitter;
  double lane_c[3];
  double lane_sigma, vd_lo, vd_hi;
  int32_t K, L;
  int32_t behaviour, sampler;  // plan_behaviour, plan_sampler_t
};

// Arguments of the lower-level kernel.
struct LowerArgs {
  const ReqDesc *desc;
  const int32_t *act_slots;  // slots of this launch
  const int32_t *blk_prefix; // workgroups before each active slot (n_act + 1)
  int32_t n_act;
  int32_t l_uniform;         // upper iteration of every slot, or -1: desc.cur_iter
  const float *basis;        // concatenated per-T tables
  const int32_t *basis_off;  // float offset of table t_idx
  const int32_t *basis_tpad; // column stride of table t_idx
  const float *step1;        // per-T: S (16x8) then R (16x4)
  const float *proj;         // per-(T,M): A^-1 (16x16) then D (16)
  float *p;                  // row pool [rows][8] (written unless forced)
  DistState *dist;           // slot distribution (iterations >= 1; written at iteration 0, see below)
  const double *sess;        // session store (iteration 0 of a warm start)
  float *zs;                 // row pool [rows][16] free coefficients
  float *resid;              // row pool [rows]
  float *cost;               // row pool [rows]
  double *xi_bar_out;        // optional [N][22] (single request only)
  double *xi_star_out;       // optional [N][22] (single request only)
  // matrix-core lower level only
  const uint16_t *mops;      // concatenated per-T basis tables (FP16 bits)
  const int32_t *mops_off;   // offset (in FP16 values) of table t_idx
  const uint16_t *mainv;     // per-(T, M) [2][64][4] high / low of kAinvScale A^-1
};

// Arguments of the selection / update kernel and the init kernel.
struct SelArgs {
  ReqDesc *desc;
  const int32_t *slots;      // slot of each workgroup
  int32_t l_uniform;         // upper iteration of every slot, or -1: desc.cur_iter
  float *p;
  const float *zs;
  const float *resid;
  const float *cost;
  DistState *dist;
  ResultRec *result;
  double *traj;              // [slot][traj_stride][2]: positions of the returned trajectory (FP64)
  int32_t traj_stride;       // instants per slot of traj (the longest horizon of the config)
  double *sess;              // session store [n_sess][72]: mu then Sigma
  // optional trace (per slot and iteration; max_N rows per slot)
  float *tr_p;               // [slot][L][max_N][8]
  float *tr_r;               // [slot][L][max_N]
  float *tr_c;               // [slot][L][max_N]
  int32_t *tr_ces;           // [slot][L][max_ces]
  int32_t *tr_es;            // [slot][L][max_es]
  double *tr_mu;             // [slot][L][8]
  double *tr_sigma;          // [slot][L][64]
  int32_t max_N, max_ces, max_es;
};

// Working memory of plan_lower_solve_static: a file-scope device array (one
// copy per GPU, static_scratch.hip), addressed through the device pointers
// that static_scratch_init takes once per device. Holds one request
// descriptor, the launch arrays and the free-coefficient rows of up to
// kStaticRows samples.
constexpr int kStaticRows = PLAN_MAX_N;
struct StaticScratch {
  ReqDesc *desc = nullptr;
  int32_t *act = nullptr;  // act_slots at [0, 8), blk_prefix at [8, 16)
  float *zs = nullptr;     // [kStaticRows][kZ]
  int32_t rows = 0;
};
// With `device` current: look up the array's address on that device (once
// per device; later calls reuse it) and fill *out.
hipError_t static_scratch_init(int device, StaticScratch *out);
size_t static_scratch_bytes();

// Decoder sampler (App. A decoder MLP at inference). Its samples are the
// rows of the requests being decoded, concatenated: segment s covers
// concatenated rows [row_begin, row_begin + n) = samples 0..n-1 of slot.
// The kernels run on a chunk of at most kDecChunk concatenated rows at a
// time: the hidden activations live in two buffers of FP16 high/low pairs
// (the matrix-core operand layout); block 1 builds its input [o, z], padded
// to kDecInPad, from the requests as it loads it.
constexpr int kDecIn = PLAN_OBS_DIM + PLAN_LATENT_DIM;  // 57
constexpr int kDecInPad = 64;                           // K of block 1 on the matrix cores
constexpr int kDecHidden = PLAN_DEC_HIDDEN;             // 1024
constexpr int kDecHidden5 = PLAN_DEC_HIDDEN5;           // 256
constexpr int kDecLayers = 5;                           // blocks on the matrix cores
constexpr int kDecChunk = 16384;

struct DecSeg {
  int32_t slot, row_begin, n, pad;
};

// One block: out = relu(inv_scale * (W_scaled x) + shift), W_scaled = W' 2^e
// split into FP16 high/low pairs (out x in, row-major), inv_scale = 2^-e,
// W' and shift the Linear layer with its BatchNorm and bias folded in.
struct DecLayer {
  const uint16_t *w_hi, *w_lo;
  const float *shift;
  float inv_scale;
  int32_t n_in, n_out;
};

struct DecArgs {
  const ReqDesc *desc;
  const DecSeg *seg;
  int32_t nseg;
  int32_t r0, nrows;          // chunk: concatenated rows [r0, r0 + nrows)
  DecLayer layer[kDecLayers]; // blocks 1-5 (block 1: n_in = kDecInPad)
  const float *w6, *b6;       // output layer [8][kDecHidden5], [8]
  uint16_t *act_hi[2], *act_lo[2];  // hidden ping-pong [kDecChunk][kDecHidden]
  float *p;                   // row pool [rows][8]
  int32_t behaviour;
};

// Arguments of the closed-loop advance kernel (one workgroup per episode,
// episode e in slot e).
struct AdvArgs {
  ReqDesc *desc;
  const ResultRec *result;
  const DistState *dist;
  const double *obs0;        // [n][PLAN_MAX_M][2] neighbour x, y at the first cycle
  int32_t cycles, cycle, n_exec;
  int32_t warm;              // nonzero: warm start from the session, else the structured sampler
  // device logs (each nullable), laid out as the host's plan_mpc_log
  double *ego, *xi, *mu, *sigma, *cost;
  int32_t *collided, *status;
};

}  // namespace plan
