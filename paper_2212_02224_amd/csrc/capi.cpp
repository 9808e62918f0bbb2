// capi.cpp -- the C ABI of include/plan.h: validation, device memory layout,
// request staging, the launch sequence of Alg. 1 on a HIP stream, and the
// served mode (continuous batching).
//
// One upper iteration of every resident request is two launches:
//   lower_kernel          draw of the iteration, Steps 1-2 of Alg. 1,
//                         residual/cost, for all samples of all requests
//   select_update_kernel  elite sets and the update of mu, Sigma, one
//                         workgroup per request
// Batch mode runs L such pairs for a staged batch; served mode runs one pair
// per plan_progress call for whatever is resident, each request at its own
// iteration (kept on the device in its descriptor). The closed loop
// (plan_mpc_run) runs L pairs per cycle followed by advance_kernel, which
// writes the next cycle's descriptors on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "plan_internal.h"
#include "precompute.h"

namespace plan {
hipError_t launch_lower(const LowerArgs &a, const MethodParams &p, int nblocks, int ipl, bool road, size_t lds,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_lower_mfma(const LowerArgs &a, const MethodParams &p, int nblocks, int tpw, bool road, bool f32,
                             int T, size_t lds, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_select(const SelArgs &a, const MethodParams &p, int nreq, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1);
hipError_t launch_lower_fused(const LowerArgs &a, const SelArgs &sa, const MethodParams &p, uint32_t *ctl,
                              int nblocks, int ipl, bool road, size_t obs_lds, uint64_t wait_ticks, hipStream_t st,
                              hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_advance(const AdvArgs &a, const MethodParams &p, int n, hipStream_t st);
hipError_t launch_decoder(const DecArgs &a, int total_rows, int n_cu, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1);
}  // namespace plan

using namespace plan;
using Clock = std::chrono::steady_clock;

namespace {

thread_local std::string g_create_error;

int round_half_up(double v) { return (int)std::floor(v + 0.5); }

void elite_sizes(const plan_config &c, int N, int &n, int &q) {
  q = std::max(1, round_half_up(c.frac_es * N));
  n = std::max(q, round_half_up(c.frac_ces * N));
  n = std::min(n, N);
  q = std::min(q, n);
}

bool finite_all(const double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int64_t budget_rows(const plan_config &c) {
  return c.sample_budget > 0 ? c.sample_budget : (int64_t)c.max_requests * c.max_N;
}

bool mfma_mode(const plan_config &c) {
  return c.precision == PLAN_PREC_FP16_SPLIT || c.precision == PLAN_PREC_FP32_MFMA;
}
bool mfma_f32(const plan_config &c) { return c.precision == PLAN_PREC_FP32_MFMA; }

// Dynamic LDS of the lower kernels: two neighbours per float4 and instant;
// the matrix-core kernel adds its basis table (kEvInstHalfs halves, or in
// the FP32 form kEv32InstFloats floats, per instant of the padded horizon),
// the fixed trajectory part (two float4 per instant), the N^T g sums of its
// tile pairs and their total.
size_t lds_bytes(int M, int T, bool mfma, bool f32 = false) {
  size_t b = (size_t)((M + 1) / 2) * T * sizeof(float4);
  if (!mfma && M > 0) b += (size_t)kObsPad * sizeof(float4);
  if (mfma) {
    const size_t NT = (size_t)((T + 3) / 4), NI = 4 * NT;
    b += (f32 ? NI * kEv32InstFloats * 4 : NI * kEvInstHalfs * 2) +
         (2 * NI + ((NT + 1) / 2 + 1) * kWave) * sizeof(float4);
  }
  return b;
}

// Horizon class of the VALU kernel: up to 64 instants (one per lane), or
// more (one or two per lane, chosen per launch).
int t_class(int T) { return T > kWave ? 2 : 1; }

// Workgroups of one request. VALU kernel: ceil(T / (64 ipl)) waves per
// sample with ipl instants per lane, 4 waves per group; matrix-core kernel:
// 16 samples per group, or 8 in its one-pair-per-wave layout (half).
int blocks_for(int N, int T, bool mfma, int ipl = 1, bool half = false) {
  if (mfma) {
    const int spb = half ? kMfmaSamples / 2 : kMfmaSamples;
    return (N + spb - 1) / spb;
  }
  const int spb = 4 / ((T + kWave * ipl - 1) / (kWave * ipl));
  return (N + spb - 1) / spb;
}

// Two instants per lane or one? Both give the same results. A workgroup of
// two instants per lane holds 4 samples (one wave each), one of one instant
// per lane 2 samples (two waves each, T = 100), so the first has half the
// waves: it is faster once its launch gives every SIMD about two waves, and
// slower below that, where the latency of each wave's chain is not hidden.
// Lower-kernel time per launch at T = 100 (one instant / two instants per
// lane): 1000 samples 37.1 / 43.2 us (M = 10), 46.8 / 56.1 us (M = 20); 2048
// samples 52.9 / 49.4, 65.8 / 62.3; 4096 samples 89.7 / 88.4, 111.1 / 112.8;
// 8192 samples 161 / 140, 198 / 180; 524288 samples 9.25 / 7.90 ms,
// 11.0 / 10.0 ms. Two instants per lane from 2 workgroups per CU on.
bool use_ipl2(int blocks1, int blocks2, int n_cu) {
  (void)blocks1;
  return blocks2 >= 2 * n_cu;
}

// Lower-level launches of one upper iteration: one per horizon length in the
// matrix-core mode (its workgroup shape depends on T), one per number of
// instants per lane in the VALU mode. Group.T is that key.
struct LaunchSet {
  int n_act = 0, ngroups = 0;
  struct Group {
    int act_off = 0, n = 0, nblocks = 0, T = 0;
    int ipl = 1;        // VALU kernel: instants per lane
    int tpw = 4;        // matrix-core kernel: 4 tiles per wave, or 1 (a tile pair over 8 samples)
    bool road = false;  // requests with a road profile
    size_t lds = 0;
  } grp[8];
};

struct DevBuf {
  char *base = nullptr;
  size_t used = 0, cap = 0;
  void *take(size_t bytes) {
    size_t off = (used + 255) & ~(size_t)255;
    if (off + bytes > cap) return nullptr;
    used = off + bytes;
    return base + off;
  }
};

// Device bytes of every region, in allocation order.
struct Layout {
  size_t basis = 0, step1 = 0, proj = 0, offs = 0, mops = 0, mainv = 0;
  size_t desc = 0, dist = 0, result = 0, traj = 0, act = 0, fctl = 0;
  size_t p = 0, zs = 0, rc = 0, sess = 0, xiout = 0;
  size_t tr_p = 0, tr_rc = 0, tr_idx = 0, tr_dist = 0;
  size_t dec_tab = 0, dec_act = 0, dec_seg = 0;  // decoder sampler
  size_t total() const {
    size_t s = 0;
    for (size_t b : {basis, step1, proj, offs, mops, mainv, desc, dist, result, traj, act, fctl, p, zs, rc, sess, xiout,
                     tr_p, tr_rc, tr_idx, tr_dist, dec_tab, dec_act, dec_seg})
      s += (b + 255) & ~(size_t)255;
    return s;
  }
};

// Pinned host staging of the served ticks (launch-set arrays, decoder
// segments) in a ring: a tick need not wait for the GPU, so the buffers of
// tick t are reused only once the event recorded after tick t - kRing has
// passed.
constexpr int kRing = 4;

int max_sessions(const plan_config &c) { return std::max(64, 2 * c.max_requests); }

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Pieces of the decoder tables, each taken 256-aligned, in carve order:
// blocks 1-5 (W hi, W lo, shift), W6, b6.
const int kDecNin[kDecLayers] = {kDecInPad, kDecHidden, kDecHidden, kDecHidden, kDecHidden};
const int kDecNout[kDecLayers] = {kDecHidden, kDecHidden, kDecHidden, kDecHidden, kDecHidden5};
constexpr int kDecPieces = 3 * kDecLayers + 2;
size_t dec_piece(int i) {
  if (i < 3 * kDecLayers) {
    const int L = i / 3, part = i % 3;
    return part < 2 ? (size_t)kDecNout[L] * kDecNin[L] * 2 : (size_t)kDecNout[L] * 4;
  }
  if (i == 3 * kDecLayers) return (size_t)PLAN_NP * kDecHidden5 * 4;
  return (size_t)PLAN_NP * 4;
}

// Rows of the decoder's activation buffers: a chunk, rounded up to whole
// 16-row blocks (the matrix-core layout stores the last partial block whole).
int dec_chunk(int64_t rows) { return (int)((std::min<int64_t>(rows, kDecChunk) + 15) / 16 * 16); }

// Instants per slot of the returned-trajectory buffer: the longest horizon.
int traj_stride(const plan_config &c) {
  int t = 0;
  for (int i = 0; i < c.n_T; ++i) t = std::max(t, (int)c.T_set[i]);
  return t;
}

Layout compute_layout(const plan_config &c) {
  Layout L;
  const size_t S = (size_t)c.max_requests, N = (size_t)c.max_N, R = (size_t)budget_rows(c);
  for (int i = 0; i < c.n_T; ++i) L.basis += (size_t)kBasisCols * ((c.T_set[i] + 63) / 64 * 64) * 4;
  L.step1 = (size_t)c.n_T * kStep1Floats * 4;
  L.proj = (size_t)c.n_T * c.n_M * kProjFloats * 4;
  L.offs = (size_t)c.n_T * 3 * 4;
  if (mfma_mode(c)) {
    const size_t per_inst = mfma_f32(c) ? kEv32InstFloats * 4 : kEvInstHalfs * 2;
    for (int i = 0; i < c.n_T; ++i) L.mops += (size_t)4 * ((c.T_set[i] + 3) / 4) * per_inst;
    if (!mfma_f32(c)) L.mainv = (size_t)c.n_T * c.n_M * 2 * kWave * 8;
  }
  L.desc = S * sizeof(ReqDesc);
  L.dist = S * sizeof(DistState);
  L.result = S * sizeof(ResultRec);
  L.traj = S * (size_t)traj_stride(c) * 2 * 8;
  L.act = (2 * S + 8) * 4;
  L.fctl = (4 + 2 * S) * 4;
  L.p = R * 8 * 4;
  L.zs = R * kZ * 4;
  L.rc = R * 2 * 4;
  L.sess = (size_t)max_sessions(c) * 72 * 8;
  L.xiout = N * 22 * 2 * 8;
  if (c.trace) {
    int n, q;
    elite_sizes(c, c.max_N, n, q);
    const size_t Lit = (size_t)c.upper_iters;
    L.tr_p = S * Lit * N * 8 * 4;
    L.tr_rc = S * Lit * N * 2 * 4;
    L.tr_idx = S * Lit * (size_t)(n + q) * 4;
    L.tr_dist = S * Lit * 72 * 8;
  }
  if (c.sampler == PLAN_SAMPLER_DECODER) {
    for (int i = 0; i < kDecPieces; ++i) L.dec_tab += round256(dec_piece(i));
    L.dec_act = 4 * round256((size_t)dec_chunk(R) * kDecHidden * 2);
    L.dec_seg = S * sizeof(DecSeg);
  }
  return L;
}

const char *validate_config(const plan_config &c) {
  if (c.n_T < 1 || c.n_T > 4 || c.n_M < 1 || c.n_M > 8) return "n_T must be 1..4 and n_M 1..8";
  for (int i = 0; i < c.n_T; ++i)
    if (c.T_set[i] < 16 || c.T_set[i] > PLAN_MAX_T) return "T must be in [16, PLAN_MAX_T]";
  for (int i = 0; i < c.n_M; ++i)
    if (c.M_set[i] < 0 || c.M_set[i] > PLAN_MAX_M) return "M must be in [0, PLAN_MAX_M]";
  if (c.max_N < 1 || c.max_N > PLAN_MAX_N) return "max_N must be in [1, PLAN_MAX_N]";
  if (c.max_requests < 1 || c.max_requests > 65536) return "max_requests must be in [1, 65536]";
  if (c.sample_budget < 0) return "sample_budget must be >= 0";
  if (c.proj_iters < 1 || c.proj_iters > 10000) return "proj_iters must be >= 1";
  if (c.upper_iters < 1 || c.upper_iters > PLAN_MAX_L) return "upper_iters must be in [1, PLAN_MAX_L]";
  if (!(c.t_f > 0) || !(c.rho > 0) || !(c.gamma > 0) || !(c.eta >= 0 && c.eta <= 1))
    return "t_f, rho, gamma must be > 0 and eta in [0, 1]";
  if (!(c.ell_a > 0) || !(c.ell_b > 0) || !(c.kappa_max > 0) || !(c.v_eps > 0))
    return "ell_a, ell_b, kappa_max, v_eps must be > 0";
  if (!(c.y_lb < c.y_ub) || !(c.v_min <= c.v_max) || !(c.a_max >= 0) || !(c.c_max >= 0))
    return "bounds must satisfy y_lb < y_ub, v_min <= v_max, a_max >= 0, c_max >= 0";
  if (!(c.frac_es > 0) || !(c.frac_ces >= c.frac_es) || c.frac_ces > 1.0)
    return "need 0 < frac_es <= frac_ces <= 1";
  int n, q;
  elite_sizes(c, c.max_N, n, q);
  if (n > kMaxCes) return "ConstraintEliteSet larger than 1024 samples is not supported";
  if (q > kMaxEs) return "EliteSet larger than 256 samples is not supported";
  if (c.behaviour != PLAN_BEHAV_SETPOINTS && c.behaviour != PLAN_BEHAV_GOALS) return "unknown behaviour";
  if (c.sampler != PLAN_SAMPLER_RANDOM && c.sampler != PLAN_SAMPLER_GRID && c.sampler != PLAN_SAMPLER_DECODER)
    return "unknown sampler";
  if (c.served_run_ahead < 0 || c.served_run_ahead > kRing - 1) return "served_run_ahead must be in [0, 3]";
  if (c.fused_iters < 0 || c.fused_iters > 1) return "fused_iters must be 0 or 1";
  if (c.fused_iters != 0 && c.fused_wait_us < 1) return "fused_wait_us must be >= 1";
  if (c.behaviour == PLAN_BEHAV_GOALS && !(c.w_s > 0)) return "goal positions need w_s > 0 (the cost is c_s alone)";
  if (c.precision != PLAN_PREC_FP32 && c.precision != PLAN_PREC_FP16_SPLIT && c.precision != PLAN_PREC_FP32_MFMA)
    return "unsupported precision";
  if (mfma_mode(c))
    for (int i = 0; i < c.n_T; ++i)
      if (c.T_set[i] > kMfmaMaxT) return "the matrix-core precisions support T <= 128";
  return nullptr;
}

// A queued request of the served mode, owning copies of its arrays.
struct Pending {
  uint64_t ticket = 0;
  plan_request req{};  // the scalars; every array it points to is copied into desc
  ReqDesc desc{};      // validated at submit
  Clock::time_point submit;
};

struct Resident {
  uint64_t ticket = 0;
  uint64_t session_key = 0;  // the request's session_id (0: none)
  int slot = -1;
  int64_t row_off = 0;
  int N = 0, T = 0;
  int iters = 0;
  int session_wb = -1;
  Clock::time_point submit;
};

// A served request whose last iteration is on the stream; it is retired
// (result filled, slot and rows freed) once `ev`, recorded after the copies
// of its result, has passed.
struct Retiring {
  Resident rs;
  hipEvent_t ev = nullptr;
};



}  // namespace

struct plan_handle {
  plan_config cfg;
  MethodParams mp;
  std::string err;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_cu = 256;  // compute units of the device
  int device = 0;  // device current at plan_create
  StaticScratch scr;  // plan_lower_solve_static's working memory on that device
  bool own_mem = false;
  DevBuf mem;
  Layout lay;
  int64_t rows = 0;
  // tables
  float *basis = nullptr, *step1 = nullptr, *proj = nullptr;
  int32_t *basis_off = nullptr, *basis_tpad = nullptr, *mops_off = nullptr;
  std::vector<int32_t> table_offs;  // host copy of basis_off / basis_tpad / mops_off
  uint16_t *mops = nullptr, *mainv = nullptr;
  // slots and the row pool
  ReqDesc *desc = nullptr;
  DistState *dist = nullptr;
  ResultRec *result = nullptr;
  double *traj = nullptr;  // [slot][traj_stride][2] positions of the returned trajectory
  int traj_T = 0;          // traj_stride of the config
  int32_t *act_slots = nullptr, *blk_prefix = nullptr;
  uint32_t *fctl = nullptr;  // control words of the fused launches (zero between launches)
  int wall_khz = 100000;     // device wall clock [kHz] (the fused launches' wait bound)
  float *p = nullptr, *zs = nullptr, *resid = nullptr, *cost = nullptr;
  double *sess = nullptr;
  double *xi_out = nullptr;
  float *tr_p = nullptr, *tr_r = nullptr, *tr_c = nullptr;
  int32_t *tr_ces = nullptr, *tr_es = nullptr;
  double *tr_mu = nullptr, *tr_sigma = nullptr;
  int max_ces = 0, max_es = 0;
  // host staging (pinned)
  ReqDesc *h_desc = nullptr;
  int32_t *h_act = nullptr;  // act_slots then blk_prefix (the current ring entry)
  int32_t *h_act_ring[kRing] = {};
  DecSeg *h_seg_ring[kRing] = {};
  hipEvent_t ring_ev[kRing] = {};
  int64_t tick = 0;  // served iterations enqueued so far (tick t stages in ring entry t % kRing)
  std::vector<Retiring> retiring;
  std::vector<hipEvent_t> sync_ev_free;  // events without timing, for retirement
  ResultRec *h_result = nullptr;
  DistState *h_dist = nullptr;
  double *h_traj = nullptr;  // pinned mirror of traj
  // batch mode: staged requests in slots 0..staged-1
  int staged = 0;
  LaunchSet ls;
  std::vector<int> ls_slots;  // make_launch_set: slots ordered by road class
  std::vector<int> staged_req;
  std::vector<int> staged_status;
  int staged_total = 0;
  Clock::time_point t_stage;
  // served mode
  std::map<int64_t, int64_t> free_rows;  // begin -> end of free row ranges
  std::vector<char> slot_busy;
  std::deque<Pending> queue;
  std::vector<Resident> resident;
  std::unordered_map<uint64_t, plan_result> done;
  std::unordered_map<uint64_t, std::vector<double>> done_traj;  // positions of finished tickets (T x 2)
  uint64_t next_ticket = 1;
  // sessions
  std::unordered_map<uint64_t, int> sess_index;
  std::vector<uint64_t> sess_key;
  std::vector<uint64_t> sess_used;
  std::vector<char> sess_valid;
  uint64_t sess_clock = 0;
  // kernel timing
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_count[3] = {0, 0, 0};
  // decoder sampler
  bool dec_ready = false;
  float *dec_w6 = nullptr, *dec_b6 = nullptr;
  uint16_t *dec_whi[kDecLayers] = {}, *dec_wlo[kDecLayers] = {};
  float *dec_shift[kDecLayers] = {};
  float dec_inv_scale[kDecLayers] = {1, 1, 1, 1, 1};
  uint16_t *dec_act[4] = {};  // ping-pong: hi 0, lo 0, hi 1, lo 1
  DecSeg *dec_seg = nullptr, *h_seg = nullptr;
  int dec_nseg = 0, dec_rows = 0;  // segment table on the device
};

namespace {

// Served requests queued, resident, or with their last copies on the stream.
bool served_in_flight(const plan_handle *h) {
  return !h->resident.empty() || !h->queue.empty() || !h->retiring.empty();
}

plan_status fail(plan_handle *h, plan_status st, const std::string &msg) {
  if (h) h->err = msg;
  return st;
}

plan_status hip_fail(plan_handle *h, hipError_t e, const char *what) {
  return fail(h, PLAN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                   \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail((h), e_, #expr); \
  } while (0)

MethodParams method_params(const plan_config &c) {
  MethodParams m;
  m.t_f = c.t_f;
  m.rho = c.rho;
  m.ell_a = c.ell_a;
  m.ell_b = c.ell_b;
  m.v_min = c.v_min;
  m.v_max = c.v_max;
  m.a_max = c.a_max;
  m.kappa_max = c.kappa_max;
  m.c_max = c.c_max;
  m.y_lb = c.y_lb;
  m.y_ub = c.y_ub;
  m.v_eps = c.v_eps;
  m.eta = c.eta;
  m.gamma = c.gamma;
  m.cov_jitter = c.cov_jitter;
  for (int i = 0; i < 3; ++i) m.lane_c[i] = c.lane_c[i];
  m.lane_sigma = c.lane_sigma;
  m.vd_lo = c.vd_lo;
  m.vd_hi = c.vd_hi;
  m.K = c.proj_iters;
  m.L = c.upper_iters;
  m.behaviour = c.behaviour;
  m.sampler = c.sampler;
  return m;
}

int find_T(const plan_config &c, int T) {
  for (int i = 0; i < c.n_T; ++i)
    if (c.T_set[i] == T) return i;
  return -1;
}
int find_M(const plan_config &c, int M) {
  for (int i = 0; i < c.n_M; ++i)
    if (c.M_set[i] == M) return i;
  return -1;
}

// Validate one request; fill its descriptor (warm start and rows are set by
// the caller).
const char *check_request(const plan_handle *h, const plan_request &r, ReqDesc &d) {
  const plan_config &c = h->cfg;
  if (r.N < 1 || r.N > c.max_N) return "N out of range";
  const int ti = find_T(c, r.T), mi = find_M(c, r.M);
  if (ti < 0) return "T not in T_set";
  if (mi < 0) return "M not in M_set";
  if (lds_bytes(r.M, r.T, false) > 60 * 1024) return "M * T too large for the LDS table";
  if (mfma_mode(c) && lds_bytes(r.M, r.T, true, mfma_f32(c)) > 64 * 1024)
    return "M * T too large for the LDS table";
  if (!finite_all(r.ego, 6) || !std::isfinite(r.kappa_road)) return "non-finite ego state";
  if (r.M > 0 && r.obstacles == nullptr) return "obstacles missing";
  if (r.M > 0 && !finite_all(r.obstacles, 4 * r.M)) return "non-finite obstacle";
  if ((r.mu0 == nullptr) != (r.sigma0 == nullptr)) return "mu0 and sigma0 must be given together";
  if (r.mu0 && (!finite_all(r.mu0, 8) || !finite_all(r.sigma0, 64))) return "non-finite mu0/sigma0";
  if (r.first_iter < 0 || r.first_iter > (1 << 20)) return "first_iter out of range";
  if (c.sampler == PLAN_SAMPLER_DECODER) {
    if (!h->dec_ready) return "decoder weights not set (plan_set_decoder)";
    if (!r.observation) return "observation missing (the decoder sampler needs one)";
    if (!finite_all(r.observation, PLAN_OBS_DIM)) return "non-finite observation";
  }
  if (r.n_road < 0 || r.n_road > PLAN_MAX_ROAD) return "n_road out of range";
  if (r.n_road > 0) {
    if (!r.road) return "road profile missing";
    if (!finite_all(r.road, 3 * r.n_road) || !std::isfinite(r.road_x0) || !std::isfinite(r.road_dx))
      return "non-finite road profile";
    if (r.n_road > 1 && !(r.road_dx > 0)) return "road_dx must be > 0";
    for (int i = 0; i < r.n_road; ++i)
      if (!(r.road[3 * i + 1] < r.road[3 * i + 2])) return "road profile needs y_lb < y_ub at every knot";
  }
  std::memset(&d, 0, sizeof(d));
  d.T = r.T;
  d.M = r.M;
  d.N = r.N;
  elite_sizes(c, r.N, d.n_ces, d.n_es);
  d.t_idx = ti;
  d.tm_idx = ti * c.n_M + mi;
  d.basis_off = h->table_offs[ti];
  d.basis_tpad = h->table_offs[c.n_T + ti];
  d.mops_off = h->table_offs[2 * c.n_T + ti];
  d.session = -1;
  d.session_wb = -1;
  d.first_iter = r.first_iter;
  d.cur_iter = 0;
  d.seed = r.seed;
  std::memcpy(d.ego, r.ego, sizeof(d.ego));
  d.kappa = r.kappa_road;
  d.n_road = r.n_road;
  d.road_x0 = r.road_x0;
  d.road_dx = r.n_road > 1 ? r.road_dx : 1.0;
  for (int i = 0; i < r.n_road; ++i)
    for (int k = 0; k < 3; ++k) d.road[i][k] = r.road[3 * i + k];
  if (c.sampler == PLAN_SAMPLER_DECODER)
    for (int k = 0; k < PLAN_OBS_DIM; ++k) d.obsv[k] = r.observation[k];
  for (int i = 0; i < r.M; ++i)
    for (int k = 0; k < 4; ++k) d.obs[i][k] = r.obstacles[4 * i + k];
  if (r.mu0) {
    std::memcpy(d.mu0, r.mu0, sizeof(d.mu0));
    std::memcpy(d.sigma0, r.sigma0, sizeof(d.sigma0));
    d.init_mode = kInitGiven;
  } else {
    d.init_mode = kInitStructured;
  }
  return nullptr;
}

int session_slot(plan_handle *h, uint64_t key) {
  auto it = h->sess_index.find(key);
  if (it != h->sess_index.end()) {
    h->sess_used[it->second] = ++h->sess_clock;
    return it->second;
  }
  const int ns = (int)h->sess_key.size();
  int victim = 0;
  for (int i = 1; i < ns; ++i)
    if (h->sess_used[i] < h->sess_used[victim]) victim = i;
  if (h->sess_key[victim] != 0) h->sess_index.erase(h->sess_key[victim]);
  h->sess_key[victim] = key;
  h->sess_used[victim] = ++h->sess_clock;
  h->sess_valid[victim] = 0;
  h->sess_index[key] = victim;
  return victim;
}

// Warm start from the session store when the request brings none.
void resolve_session(plan_handle *h, uint64_t key, ReqDesc &d, bool write_back) {
  if (key == 0) return;
  const int s = session_slot(h, key);
  if (d.init_mode == kInitStructured && h->sess_valid[s]) {
    d.init_mode = kInitSession;
    d.session = s;
  }
  if (write_back) d.session_wb = s;
}

SelArgs sel_args(plan_handle *h, int l_uniform) {
  SelArgs a;
  a.desc = h->desc;
  a.slots = h->act_slots;
  a.l_uniform = l_uniform;
  a.p = h->p;
  a.zs = h->zs;
  a.resid = h->resid;
  a.cost = h->cost;
  a.dist = h->dist;
  a.result = h->result;
  a.traj = h->traj;
  a.traj_stride = h->traj_T;
  a.sess = h->sess;
  a.tr_p = h->tr_p;
  a.tr_r = h->tr_r;
  a.tr_c = h->tr_c;
  a.tr_ces = h->tr_ces;
  a.tr_es = h->tr_es;
  a.tr_mu = h->tr_mu;
  a.tr_sigma = h->tr_sigma;
  a.max_N = h->cfg.max_N;
  a.max_ces = h->max_ces;
  a.max_es = h->max_es;
  return a;
}

LowerArgs lower_args(plan_handle *h, int n_act, int l_uniform) {
  LowerArgs a;
  a.desc = h->desc;
  a.act_slots = h->act_slots;
  a.blk_prefix = h->blk_prefix;
  a.n_act = n_act;
  a.l_uniform = l_uniform;
  a.basis = h->basis;
  a.basis_off = h->basis_off;
  a.basis_tpad = h->basis_tpad;
  a.step1 = h->step1;
  a.proj = h->proj;
  a.p = h->p;
  a.dist = h->dist;
  a.sess = h->sess;
  a.zs = h->zs;
  a.resid = h->resid;
  a.cost = h->cost;
  a.xi_bar_out = nullptr;
  a.xi_star_out = nullptr;
  a.mops = h->mops;
  a.mops_off = h->mops_off;
  a.mainv = h->mainv;
  return a;
}

// Event pair for one launch when profiling (kind: 0 lower, 1 select); the
// dispatch records both events.
hipError_t prof_pair(plan_handle *h, int kind, std::pair<hipEvent_t, hipEvent_t> &ev) {
  if (h->ev_free.empty()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    h->ev_free.push_back({a, b});
  }
  ev = h->ev_free.back();
  h->ev_free.pop_back();
  h->ev_pending.push_back({kind, ev});
  return hipSuccess;
}

template <class F>
plan_status timed(plan_handle *h, int kind, F &&launch, const char *what) {
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (h->profiling) HIP_TRY(h, prof_pair(h, kind, ev));
  hipError_t e = launch(ev.first, ev.second);
  if (e != hipSuccess) return hip_fail(h, e, what);
  return PLAN_OK;
}

// Workgroup prefix of the launch-set entries act[a0..a1) of group k (stored
// at prefix[i + k], the total at prefix[a1 + k]) with blocks(request) each;
// returns the total.
template <class F>
int set_prefix(const plan_handle *h, const int32_t *act, int32_t *prefix, int a0, int a1, int k, F blocks) {
  int total = 0;
  for (int i = a0; i < a1; ++i) {
    prefix[i + k] = total;
    total += blocks(h->h_desc[act[i]]);
  }
  prefix[a1 + k] = total;
  return total;
}
// Launch groups of the slots slots[0..n), all with or all without a road
// profile, appended to ls: group k's slots at act[off..off+n), its workgroup
// prefix counts at prefix[off + k .. off + k + n].
void add_launch_groups(plan_handle *h, const int *slots, int n, bool road, LaunchSet &ls) {
  if (n == 0) return;
  const bool mf = mfma_mode(h->cfg);
  int32_t *act = h->h_act, *prefix = h->h_act + h->cfg.max_requests;
  const int k0 = ls.ngroups, pos0 = ls.n_act;
  int keys[4];
  int nkeys = 0;
  for (int i = 0; i < n; ++i) {
    const int key = mf ? h->h_desc[slots[i]].T : t_class(h->h_desc[slots[i]].T);
    bool seen = false;
    for (int k = 0; k < nkeys; ++k) seen |= keys[k] == key;
    if (!seen) keys[nkeys++] = key;
  }
  std::sort(keys, keys + nkeys);
  int pos = pos0;
  for (int kk = 0; kk < nkeys; ++kk) {
    const int k = k0 + kk;
    LaunchSet::Group &gr = ls.grp[k];
    gr = LaunchSet::Group();
    gr.road = road;
    gr.act_off = pos;
    int blocks = 0;
    for (int i = 0; i < n; ++i) {
      const ReqDesc &d = h->h_desc[slots[i]];
      if ((mf ? d.T : t_class(d.T)) != keys[kk]) continue;
      act[pos] = slots[i];
      prefix[pos + k] = blocks;
      blocks += blocks_for(d.N, d.T, mf);
      gr.lds = std::max(gr.lds, lds_bytes(d.M, d.T, mf, mfma_f32(h->cfg)));
      ++pos;
    }
    gr.n = pos - gr.act_off;
    gr.nblocks = blocks;
    prefix[pos + k] = blocks;
    gr.T = keys[kk];
    if (mf && blocks < 2 * h->n_cu) {
      // lighter load: two tiles per wave, or while the 8-sample workgroups
      // all fit the chip at once (one per CU), one tile pair per wave (twice
      // the workgroups, half the serial work of each); the same arithmetic
      int blocks8 = 0;
      for (int i = gr.act_off; i < pos; ++i) blocks8 += blocks_for(h->h_desc[act[i]].N, 0, true, 1, true);
      gr.tpw = 2;
      if (blocks8 <= h->n_cu) {
        gr.tpw = 1;
        gr.nblocks = set_prefix(h, act, prefix, gr.act_off, pos, k,
                                [](const ReqDesc &d) { return blocks_for(d.N, d.T, true, 1, true); });
      }
    }
    if (!mf && keys[kk] == 2) {
      int blocks2 = 0;
      for (int i = gr.act_off; i < pos; ++i) {
        const ReqDesc &d = h->h_desc[act[i]];
        blocks2 += blocks_for(d.N, d.T, false, 2);
      }
      if (use_ipl2(blocks, blocks2, h->n_cu)) {
        gr.ipl = 2;
        gr.nblocks = set_prefix(h, act, prefix, gr.act_off, pos, k,
                                [](const ReqDesc &d) { return blocks_for(d.N, d.T, false, 2); });
      }
    }
  }
  ls.n_act = pos;
  ls.ngroups = k0 + nkeys;
  // One launch for the whole class: VALU mode when the longer horizon class
  // runs one instant per lane (then every request, whatever its T, fits a
  // launch of one instant per lane); matrix-core mode when the load is light
  // (the launch is shaped for the longest horizon, waves without a tile pair
  // only join the barriers), so its groups do not wait for each other. The
  // arithmetic per request is the same in any launch.
  int total = 0;
  if (mf) {
    for (int i = pos0; i < pos0 + n; ++i) total += blocks_for(h->h_desc[act[i]].N, h->h_desc[act[i]].T, true);
  } else {
    for (int kk = 0; kk < nkeys; ++kk) total += ls.grp[k0 + kk].nblocks;
  }
  const bool merge = nkeys > 1 && (mf ? total < 2 * h->n_cu : ls.grp[k0 + nkeys - 1].ipl == 1);
  if (!merge) return;
  LaunchSet::Group all;
  all.road = road;
  all.act_off = pos0;
  all.n = n;
  all.T = mf ? ls.grp[k0 + nkeys - 1].T : 1;
  // matrix-core: merged only under light load; one tile pair per wave while
  // the 8-sample workgroups all fit the chip at once, else two tiles per wave
  bool half = false;
  if (mf) {
    int blocks8 = 0;
    for (int i = pos0; i < pos0 + n; ++i) blocks8 += blocks_for(h->h_desc[act[i]].N, 0, true, 1, true);
    half = blocks8 <= h->n_cu;
    all.tpw = half ? 1 : 2;
  }
  int blocks = 0;
  for (int i = pos0; i < pos0 + n; ++i) {
    const ReqDesc &d = h->h_desc[act[i]];
    prefix[i + k0] = blocks;
    blocks += blocks_for(d.N, d.T, mf, 1, half);
    all.lds = std::max(all.lds, lds_bytes(d.M, d.T, mf, mfma_f32(h->cfg)));
  }
  prefix[pos0 + n + k0] = blocks;
  all.nblocks = blocks;
  ls.grp[k0] = all;
  ls.ngroups = k0 + 1;
}

// Order the slots into launch groups and fill the host act / prefix arrays.
// Requests with a road profile run in launches of their own (a kernel
// variant with the profile lookup), after those without; the variant depends
// on the request alone, so a request's results do not depend on its batch.
void make_launch_set(plan_handle *h, const int *slots, int n, LaunchSet &ls) {
  ls = LaunchSet();
  int *flat = h->ls_slots.data();
  int nf = 0;
  for (int i = 0; i < n; ++i)
    if (h->h_desc[slots[i]].n_road == 0) flat[nf++] = slots[i];
  int nr = nf;
  for (int i = 0; i < n; ++i)
    if (h->h_desc[slots[i]].n_road != 0) flat[nr++] = slots[i];
  add_launch_groups(h, flat, nf, false, ls);
  add_launch_groups(h, flat + nf, n - nf, true, ls);
}

plan_status upload_launch_set(plan_handle *h, const LaunchSet &ls) {
  if (ls.n_act == 0) return PLAN_OK;
  const int32_t *act = h->h_act, *prefix = h->h_act + h->cfg.max_requests;
  HIP_TRY(h, hipMemcpyAsync(h->act_slots, act, sizeof(int32_t) * ls.n_act, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->blk_prefix, prefix, sizeof(int32_t) * (ls.n_act + ls.ngroups),
                            hipMemcpyHostToDevice, h->stream));
  return PLAN_OK;
}

// Lower-level launch of group k of a launch set at upper iteration l_uniform
// (-1: each slot's cur_iter).
plan_status launch_lower_group(plan_handle *h, const LaunchSet &ls, int k, int l_uniform, double *xi_bar,
                               double *xi_star) {
  const LaunchSet::Group &gr = ls.grp[k];
  LowerArgs la = lower_args(h, gr.n, l_uniform);
  la.act_slots += gr.act_off;
  la.blk_prefix += gr.act_off + k;
  la.xi_bar_out = xi_bar;
  la.xi_star_out = xi_star;
  const bool mf = mfma_mode(h->cfg);
  return timed(
      h, 0,
      [&](hipEvent_t a, hipEvent_t b) {
        // matrix cores: 4, 2 or 1 tiles per wave by load (same arithmetic)
        return mf ? launch_lower_mfma(la, h->mp, gr.nblocks, gr.tpw, gr.road, mfma_f32(h->cfg), gr.T, gr.lds,
                                      h->stream, a, b)
                  : launch_lower(la, h->mp, gr.nblocks, gr.ipl, gr.road, gr.lds, h->stream, a, b);
      },
      mf ? "lower_mfma_kernel" : "lower_kernel");
}

plan_status launch_lower_set(plan_handle *h, const LaunchSet &ls, int l_uniform, double *xi_bar, double *xi_star) {
  for (int k = 0; k < ls.ngroups; ++k) {
    plan_status st = launch_lower_group(h, ls, k, l_uniform, xi_bar, xi_star);
    if (st != PLAN_OK) return st;
  }
  return PLAN_OK;
}

// One upper iteration of the resident slots of a launch set (its arrays are
// on the device): the lower kernel(s) then select_update_kernel.
plan_status launch_iteration(plan_handle *h, const LaunchSet &ls, int l_uniform) {
  plan_status st = launch_lower_set(h, ls, l_uniform, nullptr, nullptr);
  if (st == PLAN_OK) {
    const SelArgs sa = sel_args(h, l_uniform);
    st = timed(
        h, 1, [&](hipEvent_t a, hipEvent_t b) { return launch_select(sa, h->mp, ls.n_act, h->stream, a, b); },
        "select_update_kernel");
  }
  return st;
}

// Do the launch groups run as fused launches (fused_iters)? Only the FP32
// vector-ALU lower level has the fused form.
bool fused_mode(const plan_config &c) { return c.fused_iters != 0 && !mfma_mode(c); }

// Every upper iteration of a launch set (arrays on the device, decoder
// samples launched), all slots from iteration 0: one lower-level and one
// selection launch per iteration, or (fused_iters) one fused launch per
// launch group.
plan_status launch_solve(plan_handle *h, const LaunchSet &ls) {
  plan_status st = PLAN_OK;
  if (!fused_mode(h->cfg)) {
    for (int l = 0; st == PLAN_OK && l < h->cfg.upper_iters; ++l) st = launch_iteration(h, ls, l);
    return st;
  }
  const uint64_t wait_ticks = (uint64_t)h->cfg.fused_wait_us * (uint64_t)h->wall_khz / 1000u;
  for (int k = 0; st == PLAN_OK && k < ls.ngroups; ++k) {
    const LaunchSet::Group &gr = ls.grp[k];
    LowerArgs la = lower_args(h, gr.n, -1);
    la.act_slots += gr.act_off;
    la.blk_prefix += gr.act_off + k;
    const SelArgs sa = sel_args(h, -1);
    st = timed(
        h, 0,
        [&](hipEvent_t a, hipEvent_t b) {
          return launch_lower_fused(la, sa, h->mp, h->fctl, gr.nblocks, gr.ipl, gr.road, gr.lds, wait_ticks,
                                    h->stream, a, b);
        },
        "lower_fused_kernel");
  }
  return st;
}

plan_status upload_dec_segments(plan_handle *h, const int *slots, int n);

// Batch mode: stage requests into slots 0..k-1 with consecutive rows.
plan_status stage_impl(plan_handle *h, const plan_request *reqs, int n, int first) {
  h->dec_nseg = h->dec_rows = 0;
  if (served_in_flight(h))
    return fail(h, PLAN_E_BUSY, "served requests are in flight; drain them before batch calls");
  h->staged = 0;
  h->ls = LaunchSet();
  h->staged_req.clear();
  h->staged_status.assign(n, PLAN_OK);
  h->staged_total = n;
  std::unordered_map<uint64_t, int> last_of_session;
  for (int i = 0; i < n; ++i)
    if (reqs[i].session_id != 0) last_of_session[reqs[i].session_id] = i;
  int64_t row = 0;
  std::vector<int> slots;
  for (int i = 0; i < n; ++i) {
    if (h->staged >= h->cfg.max_requests) return fail(h, PLAN_E_INVALID, "more requests than max_requests");
    ReqDesc &d = h->h_desc[h->staged];
    if (const char *why = check_request(h, reqs[i], d)) {
      h->staged_status[i] = PLAN_E_INVALID;
      h->err = "request " + std::to_string(first + i) + ": " + why;
      continue;
    }
    if (d.N > h->rows) {
      // larger than the whole sample budget: this request fails alone
      h->staged_status[i] = PLAN_E_NOMEM;
      h->err = "request " + std::to_string(first + i) + ": N larger than the sample budget";
      continue;
    }
    if (row + d.N > h->rows) return fail(h, PLAN_E_NOMEM, "batch exceeds the sample budget");
    const uint64_t sk = reqs[i].session_id;
    resolve_session(h, sk, d, sk != 0 && last_of_session[sk] == i);
    d.row_off = row;
    row += d.N;
    const int slot = h->staged++;
    h->staged_req.push_back(i);
    slots.push_back(slot);
  }
  if (h->staged == 0) return PLAN_OK;
  make_launch_set(h, slots.data(), h->staged, h->ls);
  HIP_TRY(h, hipMemcpyAsync(h->desc, h->h_desc, sizeof(ReqDesc) * h->staged, hipMemcpyHostToDevice, h->stream));
  plan_status st = upload_launch_set(h, h->ls);
  if (st == PLAN_OK) st = upload_dec_segments(h, slots.data(), h->staged);
  return st;
}

// Decoder sampler, segment table: every listed slot that starts from the
// initial sampler (no given distribution, no warm start) gets its rows; the
// table is uploaded on the stream (the caller keeps h_seg untouched until
// the stream has passed the copy: staging and the served tick synchronise).
plan_status upload_dec_segments(plan_handle *h, const int *slots, int n) {
  h->dec_nseg = h->dec_rows = 0;
  if (h->cfg.sampler != PLAN_SAMPLER_DECODER) return PLAN_OK;
  for (int i = 0; i < n; ++i) {
    const ReqDesc &d = h->h_desc[slots[i]];
    if (d.init_mode != kInitStructured) continue;
    h->h_seg[h->dec_nseg++] = DecSeg{slots[i], h->dec_rows, d.N, 0};
    h->dec_rows += d.N;
  }
  if (h->dec_nseg > 0)
    HIP_TRY(h, hipMemcpyAsync(h->dec_seg, h->h_seg, sizeof(DecSeg) * h->dec_nseg, hipMemcpyHostToDevice,
                              h->stream));
  return PLAN_OK;
}

// Decoder sampler: the samples of the uploaded segments, written into the
// slots' sample rows before the lower level reads them.
plan_status launch_dec_segments(plan_handle *h) {
  if (h->cfg.sampler != PLAN_SAMPLER_DECODER || h->dec_nseg == 0) return PLAN_OK;
  const int nseg = h->dec_nseg, rows = h->dec_rows;
  DecArgs a{};
  a.desc = h->desc;
  a.seg = h->dec_seg;
  a.nseg = nseg;
  for (int L = 0; L < kDecLayers; ++L)
    a.layer[L] = DecLayer{h->dec_whi[L], h->dec_wlo[L], h->dec_shift[L], h->dec_inv_scale[L], kDecNin[L],
                          kDecNout[L]};
  a.w6 = h->dec_w6;
  a.b6 = h->dec_b6;
  a.act_hi[0] = h->dec_act[0];
  a.act_lo[0] = h->dec_act[1];
  a.act_hi[1] = h->dec_act[2];
  a.act_lo[1] = h->dec_act[3];
  a.p = h->p;
  a.behaviour = h->cfg.behaviour;
  return timed(
      h, 2, [&](hipEvent_t e0, hipEvent_t e1) { return launch_decoder(a, rows, h->n_cu, h->stream, e0, e1); },
      "decoder sampler");
}

plan_status launch_impl(plan_handle *h) {
  if (h->staged == 0) return PLAN_OK;
  plan_status st = launch_dec_segments(h);  // table uploaded at staging
  if (st == PLAN_OK) st = launch_solve(h, h->ls);
  return st;
}

// Fill o from the slot's records; the caller's trajectory buffer (o.traj_xy,
// nullable) keeps its pointer and receives the T x 2 positions traj.
void fill_result(plan_result &o, const ResultRec &R, const DistState &ds, double latency, const double *traj,
                 int T) {
  double *traj_xy = o.traj_xy;
  std::memset(&o, 0, sizeof(o));
  o.traj_xy = traj_xy;
  if (traj_xy && traj && R.status == 0) std::memcpy(traj_xy, traj, sizeof(double) * 2 * T);
  o.status = R.status;
  o.flags = R.flags;
  o.best_index = R.best;
  o.iterations = R.iterations;
  std::memcpy(o.p_best, R.p, sizeof(o.p_best));
  std::memcpy(o.xi_best, R.xi, sizeof(o.xi_best));
  o.cost_upper = R.cost_upper;
  o.residual = R.residual;
  std::memcpy(o.mu, ds.mu, sizeof(o.mu));
  std::memcpy(o.sigma, ds.sigma, sizeof(o.sigma));
  o.latency_s = latency;
}

// Wait for the staged batch and copy results into out[0..staged_total).
plan_status collect_impl(plan_handle *h, plan_result *out, double elapsed) {
  if (h->staged > 0) {
    HIP_TRY(h, hipMemcpyAsync(h->h_result, h->result, sizeof(ResultRec) * h->staged, hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->h_dist, h->dist, sizeof(DistState) * h->staged, hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->h_traj, h->traj, sizeof(double) * 2 * h->traj_T * h->staged,
                              hipMemcpyDeviceToHost, h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  plan_status worst = PLAN_OK;
  for (int i = 0; i < h->staged_total; ++i) {
    double *traj_xy = out[i].traj_xy;
    std::memset(&out[i], 0, sizeof(plan_result));
    out[i].traj_xy = traj_xy;
    out[i].status = h->staged_status[i];
    out[i].best_index = -1;
    if (out[i].status != PLAN_OK) worst = std::min(worst, (plan_status)out[i].status);
  }
  for (int s = 0; s < h->staged; ++s) {
    plan_result &o = out[h->staged_req[s]];
    fill_result(o, h->h_result[s], h->h_dist[s], elapsed, h->h_traj + (size_t)s * 2 * h->traj_T, h->h_desc[s].T);
    if (o.status == PLAN_E_TIMEOUT)
      h->err = "fused launch: a device-side wait exceeded fused_wait_us; requests whose iterations did not all run "
               "failed with PLAN_E_TIMEOUT";
    if (o.status != 0) worst = std::min(worst, (plan_status)o.status);
    else if (h->h_desc[s].session_wb >= 0) h->sess_valid[h->h_desc[s].session_wb] = 1;
  }
  return worst;
}

// ---- served mode: first-fit allocation of contiguous sample rows

bool take_rows(plan_handle *h, int N, int64_t &off) {
  for (auto it = h->free_rows.begin(); it != h->free_rows.end(); ++it) {
    if (it->second - it->first >= N) {
      off = it->first;
      const int64_t end = it->second;
      h->free_rows.erase(it);
      if (off + N < end) h->free_rows[off + N] = end;
      return true;
    }
  }
  return false;
}

void give_rows(plan_handle *h, int64_t off, int N) {
  int64_t b = off, e = off + N;
  auto next = h->free_rows.lower_bound(b);
  if (next != h->free_rows.end() && next->first == e) {
    e = next->second;
    next = h->free_rows.erase(next);
  }
  if (next != h->free_rows.begin()) {
    auto prev = std::prev(next);
    if (prev->second == b) {
      b = prev->first;
      h->free_rows.erase(prev);
    }
  }
  h->free_rows[b] = e;
}

// Retire the served requests whose result copies have arrived: fill their
// results (latency measured now), free their slots and rows.
plan_status retire_done(plan_handle *h) {
  for (size_t i = 0; i < h->retiring.size();) {
    const hipError_t q = hipEventQuery(h->retiring[i].ev);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (q != hipSuccess) return hip_fail(h, q, "served result copy");
    const Resident rs = h->retiring[i].rs;
    plan_result o{};
    fill_result(o, h->h_result[rs.slot], h->h_dist[rs.slot],
                std::chrono::duration<double>(Clock::now() - rs.submit).count(), nullptr, 0);
    if (o.status == 0 && rs.session_wb >= 0) h->sess_valid[rs.session_wb] = 1;
    const double *tr = h->h_traj + (size_t)rs.slot * 2 * h->traj_T;
    h->done_traj[rs.ticket].assign(tr, tr + 2 * rs.T);
    h->done[rs.ticket] = o;
    h->slot_busy[rs.slot] = 0;
    give_rows(h, rs.row_off, rs.N);
    h->sync_ev_free.push_back(h->retiring[i].ev);
    h->retiring.erase(h->retiring.begin() + i);
  }
  return PLAN_OK;
}

// Served admission: first come first served while a slot and N contiguous
// rows are free; appends the admitted slots.
void admit_queued(plan_handle *h, std::vector<int> &admitted) {
  const int S = h->cfg.max_requests;
  while (!h->queue.empty()) {
    Pending &pd = h->queue.front();
    // a request of a session waits (and the queue behind it) until the
    // session's request in flight has retired, so it starts from that
    // request's final distribution, whatever the timing
    if (pd.req.session_id != 0) {
      bool busy = false;
      for (const auto &rs : h->resident) busy |= rs.session_key == pd.req.session_id;
      for (const auto &rt : h->retiring) busy |= rt.rs.session_key == pd.req.session_id;
      if (busy) break;
    }
    int slot = -1;
    for (int s = 0; s < S; ++s)
      if (!h->slot_busy[s]) {
        slot = s;
        break;
      }
    int64_t off = 0;
    if (slot < 0 || !take_rows(h, pd.req.N, off)) break;
    const plan_request &r = pd.req;
    ReqDesc &d = h->h_desc[slot];
    d = pd.desc;
    resolve_session(h, r.session_id, d, r.session_id != 0);
    d.row_off = off;
    d.cur_iter = 0;
    h->slot_busy[slot] = 1;
    Resident rs;
    rs.ticket = pd.ticket;
    rs.session_key = r.session_id;
    rs.slot = slot;
    rs.row_off = off;
    rs.N = r.N;
    rs.T = r.T;
    rs.session_wb = d.session_wb;
    rs.submit = pd.submit;
    h->resident.push_back(rs);
    admitted.push_back(slot);
    h->queue.pop_front();
  }
}

void free_handle(plan_handle *h) {
  if (!h) return;
  // best effort: a failure while releasing cannot be reported to anyone
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (auto &e : h->ev_free) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto &e : h->ev_pending) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  if (h->own_mem && h->mem.base) (void)hipFree(h->mem.base);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  if (h->h_desc) (void)hipHostFree(h->h_desc);
  for (int r = 0; r < kRing; ++r) {
    if (h->h_act_ring[r]) (void)hipHostFree(h->h_act_ring[r]);
    if (h->h_seg_ring[r]) (void)hipHostFree(h->h_seg_ring[r]);
    if (h->ring_ev[r]) (void)hipEventDestroy(h->ring_ev[r]);
  }
  for (auto &rt : h->retiring) (void)hipEventDestroy(rt.ev);
  for (hipEvent_t e : h->sync_ev_free) (void)hipEventDestroy(e);
  if (h->h_result) (void)hipHostFree(h->h_result);
  if (h->h_dist) (void)hipHostFree(h->h_dist);
  if (h->h_traj) (void)hipHostFree(h->h_traj);
  delete h;
}

}  // namespace

extern "C" {

void plan_config_init(plan_config *c) {
  std::memset(c, 0, sizeof(*c));
  c->T_set[0] = 50;
  c->T_set[1] = 100;
  c->n_T = 2;
  c->M_set[0] = 4;
  c->M_set[1] = 10;
  c->M_set[2] = 20;
  c->n_M = 3;
  c->t_f = 5.0;
  c->max_N = 1024;
  c->max_requests = 1;
  c->proj_iters = 20;
  c->upper_iters = 5;
  c->frac_ces = 0.15;
  c->frac_es = 0.05;
  c->eta = 0.6;
  c->gamma = 0.9;
  c->rho = 1.0;
  c->k_p = 1.0;
  c->k_v = 2.0;
  c->w_s = c->w_l = c->w_v = 1.0;
  c->cov_jitter = 1e-6;
  c->v_min = 0.0;
  c->v_max = 30.0;
  c->a_max = 8.0;
  c->kappa_max = 0.2;
  c->c_max = 4.0;
  c->y_lb = -7.0;
  c->y_ub = 7.0;
  c->ell_a = 4.5;
  c->ell_b = 2.0;
  c->v_eps = 0.1;
  c->lane_c[0] = -3.5;
  c->lane_c[1] = 0.0;
  c->lane_c[2] = 3.5;
  c->lane_sigma = 0.3;
  c->vd_lo = 5.0;
  c->vd_hi = 25.0;
  c->precision = PLAN_PREC_FP32;
  c->fused_iters = 0;
  c->fused_wait_us = 1000000;
}

size_t plan_workspace_bytes(const plan_config *cfg) {
  if (!cfg || validate_config(*cfg)) return 0;
  return compute_layout(*cfg).total() + 4096;
}

const char *plan_last_error(const plan_handle *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

plan_status plan_elite_sizes(const plan_config *cfg, int32_t N, int32_t *n_ces, int32_t *n_es) {
  if (!cfg || !n_ces || !n_es || N < 1 || N > cfg->max_N) return PLAN_E_INVALID;
  int n, q;
  elite_sizes(*cfg, N, n, q);
  *n_ces = n;
  *n_es = q;
  return PLAN_OK;
}

plan_status plan_create(const plan_config *cfg, plan_handle **out) {
  if (!cfg || !out) {
    g_create_error = "null argument";
    return PLAN_E_INVALID;
  }
  *out = nullptr;
  if (const char *why = validate_config(*cfg)) {
    g_create_error = why;
    return PLAN_E_INVALID;
  }
  plan_handle *h = new plan_handle();
  h->cfg = *cfg;
  h->mp = method_params(*cfg);
  h->rows = budget_rows(*cfg);
  const plan_config &c = h->cfg;
  // ---- FP64 precompute, once per T and per (T, M)
  std::vector<BasisTable> bts(c.n_T);
  std::vector<Step1Table> s1(c.n_T);
  std::vector<ProjTable> pj((size_t)c.n_T * c.n_M);
  try {
    const CostWeights cw{c.k_p, c.k_v, c.w_s, c.w_l, c.w_v};
    for (int i = 0; i < c.n_T; ++i) {
      build_basis(c.T_set[i], c.t_f, bts[i]);
      const bool goals = c.behaviour == PLAN_BEHAV_GOALS;
      build_step1(bts[i], cw, c.t_f, goals, s1[i]);
      for (int m = 0; m < c.n_M; ++m)
        build_proj(bts[i], c.M_set[m], c.rho, goals, pj[(size_t)i * c.n_M + m]);
    }
  } catch (const std::exception &e) {
    g_create_error = std::string("precompute failed: ") + e.what();
    delete h;
    return PLAN_E_INVALID;
  }
  // ---- device memory: caller's workspace or our own allocation
  h->lay = compute_layout(c);
  const size_t need = h->lay.total() + 4096;
  if (c.device_workspace) {
    if (c.workspace_bytes < need) {
      g_create_error = "workspace too small: need " + std::to_string(need) + " bytes";
      delete h;
      return PLAN_E_NOMEM;
    }
    h->mem.base = (char *)c.device_workspace;
    h->mem.cap = c.workspace_bytes;
  } else {
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess) {
      g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
      delete h;
      return e == hipErrorOutOfMemory ? PLAN_E_NOMEM : PLAN_E_DEVICE;
    }
    h->mem.base = (char *)ptr;
    h->mem.cap = need;
    h->own_mem = true;
  }
  const Layout &L = h->lay;
  const size_t S = (size_t)c.max_requests, R = (size_t)h->rows;
  h->basis = (float *)h->mem.take(L.basis);
  h->step1 = (float *)h->mem.take(L.step1);
  h->proj = (float *)h->mem.take(L.proj);
  h->basis_off = (int32_t *)h->mem.take(L.offs);
  h->basis_tpad = h->basis_off + c.n_T;
  h->mops_off = h->basis_off + 2 * c.n_T;
  if (L.mops) {
    h->mops = (uint16_t *)h->mem.take(L.mops);
    if (L.mainv) h->mainv = (uint16_t *)h->mem.take(L.mainv);
  }
  h->desc = (ReqDesc *)h->mem.take(L.desc);
  h->dist = (DistState *)h->mem.take(L.dist);
  h->result = (ResultRec *)h->mem.take(L.result);
  h->traj_T = traj_stride(c);
  h->traj = (double *)h->mem.take(L.traj);
  h->act_slots = (int32_t *)h->mem.take(L.act);
  h->blk_prefix = h->act_slots + S;
  h->fctl = (uint32_t *)h->mem.take(L.fctl);
  h->p = (float *)h->mem.take(L.p);
  h->zs = (float *)h->mem.take(L.zs);
  h->resid = (float *)h->mem.take(L.rc);
  h->cost = h->resid + R;
  h->sess = (double *)h->mem.take(L.sess);
  h->xi_out = (double *)h->mem.take(L.xiout);
  elite_sizes(c, c.max_N, h->max_ces, h->max_es);
  if (c.trace) {
    h->tr_p = (float *)h->mem.take(L.tr_p);
    h->tr_r = (float *)h->mem.take(L.tr_rc);
    h->tr_c = h->tr_r + S * c.upper_iters * c.max_N;
    h->tr_ces = (int32_t *)h->mem.take(L.tr_idx);
    h->tr_es = h->tr_ces + S * c.upper_iters * h->max_ces;
    h->tr_mu = (double *)h->mem.take(L.tr_dist);
    h->tr_sigma = h->tr_mu + S * c.upper_iters * 8;
  }
  if (c.sampler == PLAN_SAMPLER_DECODER) {
    void *piece[kDecPieces];
    for (int i = 0; i < kDecPieces; ++i) piece[i] = h->mem.take(dec_piece(i));
    for (int Lr = 0; Lr < kDecLayers; ++Lr) {
      h->dec_whi[Lr] = (uint16_t *)piece[3 * Lr];
      h->dec_wlo[Lr] = (uint16_t *)piece[3 * Lr + 1];
      h->dec_shift[Lr] = (float *)piece[3 * Lr + 2];
    }
    h->dec_w6 = (float *)piece[3 * kDecLayers];
    h->dec_b6 = (float *)piece[3 * kDecLayers + 1];
    const int chunk = dec_chunk(R);
    for (int i = 0; i < 4; ++i) h->dec_act[i] = (uint16_t *)h->mem.take((size_t)chunk * kDecHidden * 2);
    h->dec_seg = (DecSeg *)h->mem.take(L.dec_seg);
  }
  if (!h->xi_out || !h->fctl || (c.trace && !h->tr_mu) || (c.sampler == PLAN_SAMPLER_DECODER && !h->dec_seg)) {
    g_create_error = "internal: workspace carve failed";
    free_handle(h);
    return PLAN_E_NOMEM;
  }
  h->sess_key.assign(max_sessions(c), 0);
  h->sess_used.assign(max_sessions(c), 0);
  h->sess_valid.assign(max_sessions(c), 0);
  h->slot_busy.assign(S, 0);
  h->ls_slots.assign(S, 0);
  h->free_rows[0] = h->rows;
  // ---- stream and pinned staging
  hipError_t e = hipSuccess;
  {
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      h->n_cu = cus;
    int khz = 0;
    if (e == hipSuccess && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      h->wall_khz = khz;
    h->device = dev;
    // the static scratch array's address on this device (once per device)
    if (e == hipSuccess) e = static_scratch_init(dev, &h->scr);
  }
  if (e == hipSuccess && c.stream) {
    h->stream = (hipStream_t)c.stream;
  } else if (e == hipSuccess) {
    e = hipStreamCreate(&h->stream);
    h->own_stream = e == hipSuccess;
  }
  if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_desc, sizeof(ReqDesc) * S);
  for (int r = 0; e == hipSuccess && r < kRing; ++r) {
    e = hipHostMalloc((void **)&h->h_act_ring[r], sizeof(int32_t) * (2 * S + 8));
    if (e == hipSuccess && c.sampler == PLAN_SAMPLER_DECODER)
      e = hipHostMalloc((void **)&h->h_seg_ring[r], sizeof(DecSeg) * S);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ring_ev[r], hipEventDisableTiming);
  }
  h->h_act = h->h_act_ring[0];
  h->h_seg = h->h_seg_ring[0];
  if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_result, sizeof(ResultRec) * S);
  if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_dist, sizeof(DistState) * S);
  if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_traj, L.traj);
  // ---- upload tables
  if (e == hipSuccess) {
    std::vector<float> basis_all;
    std::vector<uint16_t> mops_all, mainv_all, tmp;
    std::vector<int32_t> offs(3 * c.n_T);
    for (int i = 0; i < c.n_T; ++i) {
      offs[i] = (int32_t)basis_all.size();
      offs[c.n_T + i] = bts[i].Tpad;
      basis_all.insert(basis_all.end(), bts[i].table.begin(), bts[i].table.end());
      if (h->mops) {
        offs[2 * c.n_T + i] = (int32_t)mops_all.size();
        if (mfma_f32(c)) build_mfma32_basis(bts[i], tmp);
        else build_mfma_basis(bts[i], tmp);
        mops_all.insert(mops_all.end(), tmp.begin(), tmp.end());
      }
    }
    if (h->mainv)
      for (auto &t : pj) {
        build_mfma_inverse(t, tmp);
        mainv_all.insert(mainv_all.end(), tmp.begin(), tmp.end());
      }
    std::vector<float> s1all, pjall;
    for (auto &t : s1) s1all.insert(s1all.end(), t.table.begin(), t.table.end());
    for (auto &t : pj) pjall.insert(pjall.end(), t.table.begin(), t.table.end());
    e = hipMemcpyAsync(h->basis, basis_all.data(), basis_all.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->basis_off, offs.data(), offs.size() * 4, hipMemcpyHostToDevice, h->stream);
    h->table_offs = offs;
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->step1, s1all.data(), s1all.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->proj, pjall.data(), pjall.size() * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && h->mops)
      e = hipMemcpyAsync(h->mops, mops_all.data(), mops_all.size() * 2, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && h->mainv)
      e = hipMemcpyAsync(h->mainv, mainv_all.data(), mainv_all.size() * 2, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->sess, 0, L.sess, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->fctl, 0, L.fctl, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  }
  if (e != hipSuccess) {
    g_create_error = std::string("device setup: ") + hipGetErrorString(e);
    free_handle(h);
    return PLAN_E_DEVICE;
  }
  *out = h;
  return PLAN_OK;
}

void plan_destroy(plan_handle *h) { free_handle(h); }

plan_status plan_stage(plan_handle *h, const plan_request *reqs, int32_t n) {
  if (!h || (n > 0 && !reqs) || n < 0) return fail(h, PLAN_E_INVALID, "bad arguments");
  if (n > h->cfg.max_requests) return fail(h, PLAN_E_INVALID, "more requests than max_requests");
  h->t_stage = Clock::now();
  plan_status st = stage_impl(h, reqs, n, 0);
  if (st != PLAN_OK) return st;
  return hipStreamSynchronize(h->stream) == hipSuccess ? PLAN_OK : fail(h, PLAN_E_DEVICE, "stage sync");
}

plan_status plan_launch(plan_handle *h) {
  if (!h) return PLAN_E_INVALID;
  return launch_impl(h);
}

plan_status plan_collect(plan_handle *h, plan_result *out) {
  if (!h || !out) return fail(h, PLAN_E_INVALID, "bad arguments");
  const double el = std::chrono::duration<double>(Clock::now() - h->t_stage).count();
  return collect_impl(h, out, el);
}

plan_status plan_solve_batch(plan_handle *h, const plan_request *reqs, int32_t n, plan_result *out) {
  if (!h || n < 0 || (n > 0 && (!reqs || !out))) return fail(h, PLAN_E_INVALID, "bad arguments");
  plan_status worst = PLAN_OK;
  int first = 0;
  while (first < n) {
    // a group: at most max_requests requests whose samples fit the budget
    int m = 0;
    int64_t rows = 0;
    while (first + m < n && m < h->cfg.max_requests) {
      const int Nr = reqs[first + m].N;
      const bool counted = Nr >= 1 && Nr <= h->cfg.max_N;
      if (m > 0 && counted && rows + Nr > h->rows) break;
      if (counted) rows += Nr;
      ++m;
    }
    const auto t0 = Clock::now();
    plan_status st = stage_impl(h, reqs + first, m, first);
    if (st == PLAN_OK) st = launch_impl(h);
    hipError_t e = st == PLAN_OK ? hipStreamSynchronize(h->stream) : hipSuccess;
    if (e != hipSuccess) st = hip_fail(h, e, "solve");
    if (st != PLAN_OK) {
      // this group and the ones after it did not run: each says why
      for (int i = first; i < n; ++i) {
        double *traj_xy = out[i].traj_xy;
        std::memset(&out[i], 0, sizeof(plan_result));
        out[i].traj_xy = traj_xy;
        out[i].status = st;
        out[i].best_index = -1;
      }
      return st;
    }
    const double el = std::chrono::duration<double>(Clock::now() - t0).count();
    st = collect_impl(h, out + first, el);
    worst = std::min(worst, st);
    first += m;
  }
  return worst;
}

plan_status plan_mpc_run(plan_handle *h, const plan_request *reqs, int32_t n, int32_t cycles, int32_t n_exec,
                         int32_t init, plan_mpc_log *log, plan_result *out) {
  if (!h || !reqs || n < 1) return fail(h, PLAN_E_INVALID, "bad arguments");
  if (n > h->cfg.max_requests) return fail(h, PLAN_E_INVALID, "more episodes than max_requests");
  if (cycles < 1 || cycles > (1 << 20)) return fail(h, PLAN_E_INVALID, "cycles out of range");
  if (init != PLAN_MPC_SAMPLER && init != PLAN_MPC_WARM) return fail(h, PLAN_E_INVALID, "unknown init mode");
  if (h->cfg.sampler == PLAN_SAMPLER_DECODER)
    return fail(h, PLAN_E_UNSUPPORTED, "the closed loop has no per-cycle observation for the decoder sampler");
  std::unordered_map<uint64_t, int> seen;
  for (int i = 0; i < n; ++i) {
    if (n_exec < 1 || n_exec > reqs[i].T - 1)
      return fail(h, PLAN_E_INVALID, "episode " + std::to_string(i) + ": n_exec out of [1, T - 1]");
    if (reqs[i].session_id == 0 && init == PLAN_MPC_WARM)
      return fail(h, PLAN_E_INVALID, "episode " + std::to_string(i) + ": no session_id");
    if (reqs[i].session_id != 0 && !seen.emplace(reqs[i].session_id, i).second)
      return fail(h, PLAN_E_INVALID, "episode " + std::to_string(i) + ": session_id repeated");
  }
  plan_status st = stage_impl(h, reqs, n, 0);
  if (st != PLAN_OK) return st;
  for (int i = 0; i < n; ++i)
    if (h->staged_status[i] != PLAN_OK) return fail(h, (plan_status)h->staged_status[i], h->err);

  // Device memory of the call: first-cycle neighbour positions and the logs
  // that were asked for.
  const size_t nc = (size_t)n * cycles;
  const plan_mpc_log lg = log ? *log : plan_mpc_log{};
  struct Part {
    void *host;
    size_t bytes;
    size_t off;
  } parts[8] = {{nullptr, (size_t)n * PLAN_MAX_M * 2 * 8, 0},
                {lg.ego, (size_t)n * (cycles + 1) * 6 * 8, 0},
                {lg.xi, nc * 22 * 8, 0},
                {lg.mu, nc * 8 * 8, 0},
                {lg.sigma, nc * 64 * 8, 0},
                {lg.cost, nc * 2 * 8, 0},
                {lg.collided, nc * 4, 0},
                {lg.status, nc * 4, 0}};
  size_t total = 0;
  for (int k = 0; k < 8; ++k) {
    if (k > 0 && parts[k].host == nullptr) continue;
    parts[k].off = total;
    total += (parts[k].bytes + 255) & ~(size_t)255;
  }
  char *buf = nullptr;
  if (hipMalloc(&buf, total) != hipSuccess) return fail(h, PLAN_E_NOMEM, "closed-loop log memory");
  auto dev = [&](int k) -> void * { return (k == 0 || parts[k].host) ? buf + parts[k].off : nullptr; };
  std::vector<double> o0((size_t)n * PLAN_MAX_M * 2, 0.0);
  for (int i = 0; i < n; ++i) {
    const ReqDesc &d = h->h_desc[i];
    for (int m = 0; m < d.M; ++m) {
      o0[((size_t)i * PLAN_MAX_M + m) * 2] = d.obs[m][0];
      o0[((size_t)i * PLAN_MAX_M + m) * 2 + 1] = d.obs[m][1];
    }
  }
  AdvArgs aa;
  aa.desc = h->desc;
  aa.result = h->result;
  aa.dist = h->dist;
  aa.obs0 = (const double *)dev(0);
  aa.cycles = cycles;
  aa.n_exec = n_exec;
  aa.warm = init == PLAN_MPC_WARM ? 1 : 0;
  aa.ego = (double *)dev(1);
  aa.xi = (double *)dev(2);
  aa.mu = (double *)dev(3);
  aa.sigma = (double *)dev(4);
  aa.cost = (double *)dev(5);
  aa.collided = (int32_t *)dev(6);
  aa.status = (int32_t *)dev(7);
  const auto t0 = Clock::now();
  hipError_t e = hipMemcpyAsync(buf, o0.data(), o0.size() * 8, hipMemcpyHostToDevice, h->stream);
  for (int c = 0; e == hipSuccess && st == PLAN_OK && c < cycles; ++c) {
    st = launch_impl(h);
    aa.cycle = c;
    if (st == PLAN_OK) e = launch_advance(aa, h->mp, n, h->stream);
  }
  if (e == hipSuccess && st == PLAN_OK) e = hipStreamSynchronize(h->stream);
  for (int k = 1; e == hipSuccess && st == PLAN_OK && k < 8; ++k)
    if (parts[k].host) e = hipMemcpy(parts[k].host, buf + parts[k].off, parts[k].bytes, hipMemcpyDeviceToHost);
  const double el = std::chrono::duration<double>(Clock::now() - t0).count();
  if (e == hipSuccess && st == PLAN_OK && lg.ego) {
    // the first cycle's state is the request's (the kernel writes the rest)
    for (int i = 0; i < n; ++i) std::memcpy(lg.ego + (size_t)i * (cycles + 1) * 6, reqs[i].ego, 6 * 8);
  }
  if (e == hipSuccess && st == PLAN_OK) {
    std::vector<plan_result> tmp(out ? 0 : n);
    st = collect_impl(h, out ? out : tmp.data(), el);
  }
  // release the loop's buffer on every path; the call's status is already decided
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(buf);
  h->staged = 0;
  h->staged_total = 0;
  if (e != hipSuccess) return hip_fail(h, e, "closed loop");
  return st;
}

plan_status plan_lower_solve(plan_handle *h, const plan_request *req, const double *p, int32_t N,
                             double *xi_bar, double *xi_star, double *resid, double *cost_upper) {
  if (!h || !req || !p) return fail(h, PLAN_E_INVALID, "bad arguments");
  if (served_in_flight(h))
    return fail(h, PLAN_E_BUSY, "served requests are in flight; drain them before batch calls");
  plan_request r = *req;
  r.N = N;
  r.mu0 = r.sigma0 = nullptr;
  r.session_id = 0;
  ReqDesc &d = h->h_desc[0];
  if (const char *why = check_request(h, r, d)) return fail(h, PLAN_E_INVALID, why);
  if (N > h->rows) return fail(h, PLAN_E_NOMEM, "N larger than the sample budget");
  if (!finite_all(p, 8 * N)) return fail(h, PLAN_E_INVALID, "non-finite p");
  d.init_mode = kInitForced;
  d.row_off = 0;
  std::vector<float> pf((size_t)N * 8);
  for (size_t i = 0; i < pf.size(); ++i) pf[i] = (float)p[i];
  const int slot0 = 0;
  LaunchSet ls;
  make_launch_set(h, &slot0, 1, ls);
  HIP_TRY(h, hipMemcpyAsync(h->desc, h->h_desc, sizeof(ReqDesc), hipMemcpyHostToDevice, h->stream));
  plan_status ust = upload_launch_set(h, ls);
  if (ust != PLAN_OK) return ust;
  HIP_TRY(h, hipMemcpyAsync(h->p, pf.data(), pf.size() * 4, hipMemcpyHostToDevice, h->stream));
  double *xi_bar_d = h->xi_out, *xi_star_d = h->xi_out + (size_t)h->cfg.max_N * 22;
  ust = launch_lower_set(h, ls, 0, xi_bar_d, xi_star_d);
  if (ust != PLAN_OK) return ust;
  std::vector<double> xo((size_t)N * 22 * 2);
  std::vector<float> rc((size_t)N * 2);
  HIP_TRY(h, hipMemcpyAsync(xo.data(), xi_bar_d, (size_t)N * 22 * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(xo.data() + (size_t)N * 22, xi_star_d, (size_t)N * 22 * 8, hipMemcpyDeviceToHost,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(rc.data(), h->resid, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(rc.data() + N, h->cost, (size_t)N * 4, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (xi_bar) std::memcpy(xi_bar, xo.data(), (size_t)N * 22 * 8);
  if (xi_star) std::memcpy(xi_star, xo.data() + (size_t)N * 22, (size_t)N * 22 * 8);
  for (int j = 0; j < N; ++j) {
    if (resid) resid[j] = rc[j];
    if (cost_upper) cost_upper[j] = rc[N + j];
  }
  h->staged = 0;  // slot 0 was overwritten
  return PLAN_OK;
}

plan_status plan_lower_solve_static(plan_handle *h, const plan_request *req, const float *p, int32_t N,
                                    double *xi_bar, double *xi_star, float *resid, float *cost_upper) {
  if (!h || !req || !p || !resid || !cost_upper) return fail(h, PLAN_E_INVALID, "bad arguments");
  if ((xi_bar == nullptr) != (xi_star == nullptr))
    return fail(h, PLAN_E_INVALID, "xi_bar and xi_star must both be given or both be NULL");
  if (served_in_flight(h))
    return fail(h, PLAN_E_BUSY, "served requests are in flight; drain them before batch calls");
  if (N > h->scr.rows)
    return fail(h, PLAN_E_NOMEM, "N larger than the static scratch (" + std::to_string(h->scr.rows) + " rows)");
  plan_request r = *req;
  r.N = N;
  r.mu0 = r.sigma0 = nullptr;
  r.session_id = 0;
  ReqDesc &d = h->h_desc[0];
  if (const char *why = check_request(h, r, d)) return fail(h, PLAN_E_INVALID, why);
  d.init_mode = kInitForced;
  d.row_off = 0;
  const int slot0 = 0;
  LaunchSet ls;
  make_launch_set(h, &slot0, 1, ls);
  if (ls.n_act != 1 || ls.n_act + ls.ngroups > 8) return fail(h, PLAN_E_INVALID, "internal: launch set");
  h->staged = 0;  // slot 0's host descriptor now holds this request
  // descriptor and launch arrays into the scratch array (pinned host sources,
  // and the call waits below, so the next call cannot overwrite them early)
  const int32_t *act = h->h_act, *prefix = h->h_act + h->cfg.max_requests;
  HIP_TRY(h, hipMemcpyAsync(h->scr.desc, h->h_desc, sizeof(ReqDesc), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->scr.act, act, sizeof(int32_t) * ls.n_act, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->scr.act + 8, prefix, sizeof(int32_t) * (ls.n_act + ls.ngroups),
                            hipMemcpyHostToDevice, h->stream));
  const bool mf = mfma_mode(h->cfg);
  for (int k = 0; k < ls.ngroups; ++k) {
    const LaunchSet::Group &gr = ls.grp[k];
    LowerArgs la = lower_args(h, gr.n, 0);
    la.desc = h->scr.desc;
    la.act_slots = h->scr.act + gr.act_off;
    la.blk_prefix = h->scr.act + 8 + gr.act_off + k;
    la.p = const_cast<float *>(p);  // read only: the samples are the caller's (kInitForced)
    la.dist = nullptr;              // not read for caller's samples
    la.sess = nullptr;
    la.zs = h->scr.zs;
    la.resid = resid;
    la.cost = cost_upper;
    la.xi_bar_out = xi_bar;
    la.xi_star_out = xi_star;
    const hipError_t e =
        mf ? launch_lower_mfma(la, h->mp, gr.nblocks, gr.tpw, gr.road, mfma_f32(h->cfg), gr.T, gr.lds, h->stream,
                               nullptr, nullptr)
           : launch_lower(la, h->mp, gr.nblocks, gr.ipl, gr.road, gr.lds, h->stream, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(h, e, mf ? "lower_mfma_kernel" : "lower_kernel");
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return PLAN_OK;
}

plan_status plan_get_trace(plan_handle *h, int32_t i, double *p, double *resid, double *cost_upper,
                           int32_t *ces, int32_t *es, double *mu, double *sigma) {
  if (!h) return PLAN_E_INVALID;
  if (!h->cfg.trace) return fail(h, PLAN_E_UNSUPPORTED, "trace was not enabled in plan_config");
  int slot = -1;
  for (int s = 0; s < h->staged; ++s)
    if (h->staged_req[s] == i) slot = s;
  if (slot < 0) return fail(h, PLAN_E_INVALID, "request not in the last staged batch");
  const ReqDesc &d = h->h_desc[slot];
  const size_t L = h->cfg.upper_iters, Nmax = h->cfg.max_N, N = d.N;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (size_t l = 0; l < L; ++l) {
    const size_t tb = ((size_t)slot * L + l) * Nmax;
    if (p) {
      std::vector<float> f(N * 8);
      HIP_TRY(h, hipMemcpy(f.data(), h->tr_p + tb * 8, N * 8 * 4, hipMemcpyDeviceToHost));
      for (size_t k = 0; k < N * 8; ++k) p[l * N * 8 + k] = f[k];
    }
    if (resid || cost_upper) {
      std::vector<float> f(N);
      if (resid) {
        HIP_TRY(h, hipMemcpy(f.data(), h->tr_r + tb, N * 4, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < N; ++k) resid[l * N + k] = f[k];
      }
      if (cost_upper) {
        HIP_TRY(h, hipMemcpy(f.data(), h->tr_c + tb, N * 4, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < N; ++k) cost_upper[l * N + k] = f[k];
      }
    }
    const size_t ib = (size_t)slot * L + l;
    if (ces)
      HIP_TRY(h, hipMemcpy(ces + l * d.n_ces, h->tr_ces + ib * h->max_ces, d.n_ces * 4, hipMemcpyDeviceToHost));
    if (es) HIP_TRY(h, hipMemcpy(es + l * d.n_es, h->tr_es + ib * h->max_es, d.n_es * 4, hipMemcpyDeviceToHost));
    if (mu) HIP_TRY(h, hipMemcpy(mu + l * 8, h->tr_mu + ib * 8, 64, hipMemcpyDeviceToHost));
    if (sigma) HIP_TRY(h, hipMemcpy(sigma + l * 64, h->tr_sigma + ib * 64, 512, hipMemcpyDeviceToHost));
  }
  return PLAN_OK;
}

// ---- served mode

plan_status plan_submit(plan_handle *h, const plan_request *req, uint64_t *ticket) {
  if (!h || !req || !ticket) return fail(h, PLAN_E_INVALID, "bad arguments");
  Pending pd;
  if (const char *why = check_request(h, *req, pd.desc)) return fail(h, PLAN_E_INVALID, why);
  if (req->N > h->rows) return fail(h, PLAN_E_NOMEM, "request larger than the sample budget");
  pd.ticket = h->next_ticket++;
  pd.req = *req;
  pd.req.obstacles = nullptr;
  pd.req.mu0 = pd.req.sigma0 = nullptr;
  pd.req.road = nullptr;
  pd.submit = Clock::now();
  *ticket = pd.ticket;
  h->queue.push_back(std::move(pd));
  return PLAN_OK;
}

// Result copies of a served request whose last iteration is enqueued, and
// its move to the retiring list (retired by retire_done once the copies
// have arrived).
plan_status enqueue_retire(plan_handle *h, const Resident &rs) {
  HIP_TRY(h, hipMemcpyAsync(h->h_result + rs.slot, h->result + rs.slot, sizeof(ResultRec), hipMemcpyDeviceToHost,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->h_dist + rs.slot, h->dist + rs.slot, sizeof(DistState), hipMemcpyDeviceToHost,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->h_traj + (size_t)rs.slot * 2 * h->traj_T, h->traj + (size_t)rs.slot * 2 * h->traj_T,
                            sizeof(double) * 2 * rs.T, hipMemcpyDeviceToHost, h->stream));
  Retiring rt;
  rt.rs = rs;
  if (!h->sync_ev_free.empty()) {
    rt.ev = h->sync_ev_free.back();
    h->sync_ev_free.pop_back();
  } else {
    HIP_TRY(h, hipEventCreateWithFlags(&rt.ev, hipEventDisableTiming));
  }
  HIP_TRY(h, hipEventRecord(rt.ev, h->stream));
  h->retiring.push_back(rt);
  return PLAN_OK;
}

// Served mode with fused iterations: each call enqueues the whole solve of
// the requests it admits (one launch set, every iteration), so a request's
// iterations follow each other on the device without host ticks. At most
// kRing such solves are in flight (the pinned launch arrays of the one
// enqueued kRing calls ago are reused once it has finished).
plan_status progress_fused(plan_handle *h, int32_t *n_active, int32_t *n_queued) {
  if (h->tick >= kRing) HIP_TRY(h, hipEventSynchronize(h->ring_ev[(h->tick - kRing) % kRing]));
  plan_status st = retire_done(h);
  if (st != PLAN_OK) return st;
  std::vector<int> admitted;
  admit_queued(h, admitted);
  if (admitted.empty() && !h->retiring.empty()) {
    // nothing to launch: wait for the oldest result instead (the stream
    // completes them in order), so that every call makes progress
    HIP_TRY(h, hipEventSynchronize(h->retiring.front().ev));
    st = retire_done(h);
    if (st != PLAN_OK) return st;
    admit_queued(h, admitted);
  }
  if (!admitted.empty()) {
    std::sort(admitted.begin(), admitted.end());
    for (size_t a = 0; a < admitted.size();) {
      size_t b = a + 1;
      while (b < admitted.size() && admitted[b] == admitted[b - 1] + 1) ++b;
      HIP_TRY(h, hipMemcpyAsync(h->desc + admitted[a], h->h_desc + admitted[a], sizeof(ReqDesc) * (b - a),
                                hipMemcpyHostToDevice, h->stream));
      a = b;
    }
    const int rg = (int)(h->tick % kRing);
    h->h_act = h->h_act_ring[rg];
    h->h_seg = h->h_seg_ring[rg];
    LaunchSet ls;
    make_launch_set(h, admitted.data(), (int)admitted.size(), ls);
    st = upload_launch_set(h, ls);
    if (st == PLAN_OK) st = upload_dec_segments(h, admitted.data(), (int)admitted.size());
    if (st == PLAN_OK) st = launch_dec_segments(h);
    if (st == PLAN_OK) st = launch_solve(h, ls);
    if (st != PLAN_OK) return st;
    HIP_TRY(h, hipEventRecord(h->ring_ev[rg], h->stream));
    ++h->tick;
    for (int i = (int)h->resident.size() - 1; i >= 0; --i) {
      Resident &rs = h->resident[i];
      rs.iters = h->cfg.upper_iters;
      st = enqueue_retire(h, rs);
      if (st != PLAN_OK) return st;
      h->resident.erase(h->resident.begin() + i);
    }
  }
  if (n_active) *n_active = (int32_t)(h->resident.size() + h->retiring.size());
  if (n_queued) *n_queued = (int32_t)h->queue.size();
  return PLAN_OK;
}

plan_status plan_progress(plan_handle *h, int32_t *n_active, int32_t *n_queued) {
  if (!h) return PLAN_E_INVALID;
  h->staged = 0;  // batch slots are reused
  if (fused_mode(h->cfg)) return progress_fused(h, n_active, n_queued);
  // Run-ahead limit: tick t is enqueued once tick t - 1 - run_ahead has
  // finished (which also frees ring entry t % kRing, last used by tick
  // t - kRing).
  const int ra = h->cfg.served_run_ahead;
  if (h->tick >= 1 + ra) HIP_TRY(h, hipEventSynchronize(h->ring_ev[(h->tick - 1 - ra) % kRing]));
  // Requests whose results have arrived free their slots and rows first.
  plan_status st = retire_done(h);
  if (st != PLAN_OK) return st;
  std::vector<int> admitted;
  admit_queued(h, admitted);
  if (h->resident.empty() && !h->retiring.empty()) {
    // nothing to launch: wait for the oldest result instead (the stream
    // completes them in order), so that every call makes progress
    HIP_TRY(h, hipEventSynchronize(h->retiring.front().ev));
    st = retire_done(h);
    if (st != PLAN_OK) return st;
    admit_queued(h, admitted);
  }
  // descriptors of the admitted slots, one copy per run of consecutive slots
  // (a slot's host descriptor is written again only after the slot retired)
  std::sort(admitted.begin(), admitted.end());
  for (size_t a = 0; a < admitted.size();) {
    size_t b = a + 1;
    while (b < admitted.size() && admitted[b] == admitted[b - 1] + 1) ++b;
    HIP_TRY(h, hipMemcpyAsync(h->desc + admitted[a], h->h_desc + admitted[a], sizeof(ReqDesc) * (b - a),
                              hipMemcpyHostToDevice, h->stream));
    a = b;
  }
  const int n_act = (int)h->resident.size();
  if (n_act > 0) {
    // One upper iteration for every resident request, staged through the
    // next ring entry of pinned host memory.
    const int rg = (int)(h->tick % kRing);
    h->h_act = h->h_act_ring[rg];
    h->h_seg = h->h_seg_ring[rg];
    std::vector<int> slots(n_act);
    for (int i = 0; i < n_act; ++i) slots[i] = h->resident[i].slot;
    LaunchSet ls;
    make_launch_set(h, slots.data(), n_act, ls);
    st = upload_launch_set(h, ls);
    if (st == PLAN_OK && h->cfg.sampler == PLAN_SAMPLER_DECODER) {
      std::vector<int> first;
      for (int i = 0; i < n_act; ++i)
        if (h->resident[i].iters == 0) first.push_back(h->resident[i].slot);
      st = upload_dec_segments(h, first.data(), (int)first.size());
      if (st == PLAN_OK) st = launch_dec_segments(h);
    }
    if (st == PLAN_OK) st = launch_iteration(h, ls, -1);
    if (st != PLAN_OK) return st;
    HIP_TRY(h, hipEventRecord(h->ring_ev[rg], h->stream));
    ++h->tick;
    // Requests that ran their last iteration: copy their results back and
    // retire them once the copies have arrived (retire_done); the host does
    // not wait for the GPU here.
    for (int i = n_act - 1; i >= 0; --i) {
      Resident &rs = h->resident[i];
      if (++rs.iters < h->cfg.upper_iters) continue;
      st = enqueue_retire(h, rs);
      if (st != PLAN_OK) return st;
      h->resident.erase(h->resident.begin() + i);
    }
  }
  if (n_active) *n_active = (int32_t)(h->resident.size() + h->retiring.size());
  if (n_queued) *n_queued = (int32_t)h->queue.size();
  return PLAN_OK;
}

plan_status plan_poll(plan_handle *h, uint64_t ticket, plan_result *out) {
  if (!h || !out) return fail(h, PLAN_E_INVALID, "bad arguments");
  plan_status st = retire_done(h);
  if (st != PLAN_OK) return st;
  auto it = h->done.find(ticket);
  if (it != h->done.end()) {
    double *traj_xy = out->traj_xy;
    *out = it->second;
    out->traj_xy = traj_xy;
    auto tt = h->done_traj.find(ticket);
    if (traj_xy && tt != h->done_traj.end() && out->status == 0)
      std::memcpy(traj_xy, tt->second.data(), sizeof(double) * tt->second.size());
    if (tt != h->done_traj.end()) h->done_traj.erase(tt);
    h->done.erase(it);
    return PLAN_OK;
  }
  for (const auto &rs : h->resident)
    if (rs.ticket == ticket) return PLAN_E_BUSY;
  for (const auto &rt : h->retiring)
    if (rt.rs.ticket == ticket) return PLAN_E_BUSY;
  for (const auto &pd : h->queue)
    if (pd.ticket == ticket) return PLAN_E_BUSY;
  return fail(h, PLAN_E_INVALID, "unknown ticket");
}

plan_status plan_poll_done(plan_handle *h, uint64_t *tickets, plan_result *out, int32_t max_n, int32_t *n_done) {
  if (!h || !n_done || max_n < 0 || (max_n > 0 && (!tickets || !out))) return fail(h, PLAN_E_INVALID, "bad arguments");
  *n_done = 0;
  plan_status st = retire_done(h);
  if (st != PLAN_OK) return st;
  // finished tickets in ticket (submission) order, up to max_n
  std::vector<uint64_t> ready;
  ready.reserve(h->done.size());
  for (const auto &kv : h->done) ready.push_back(kv.first);
  std::sort(ready.begin(), ready.end());
  int32_t k = 0;
  for (uint64_t t : ready) {
    if (k == max_n) break;
    auto it = h->done.find(t);
    double *traj_xy = out[k].traj_xy;
    out[k] = it->second;
    out[k].traj_xy = traj_xy;
    auto tt = h->done_traj.find(t);
    if (traj_xy && tt != h->done_traj.end() && out[k].status == 0)
      std::memcpy(traj_xy, tt->second.data(), sizeof(double) * tt->second.size());
    if (tt != h->done_traj.end()) h->done_traj.erase(tt);
    h->done.erase(it);
    tickets[k++] = t;
  }
  *n_done = k;
  return PLAN_OK;
}

plan_status plan_set_decoder(plan_handle *h, const plan_decoder *dec) {
  if (!h || !dec) return fail(h, PLAN_E_INVALID, "bad arguments");
  if (h->cfg.sampler != PLAN_SAMPLER_DECODER)
    return fail(h, PLAN_E_INVALID, "the config's sampler is not PLAN_SAMPLER_DECODER");
  if (served_in_flight(h))
    return fail(h, PLAN_E_BUSY, "served requests are in flight; drain them first");
  DecoderTables t;
  if (const char *why = build_decoder(*dec, t)) return fail(h, PLAN_E_INVALID, why);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->dec_ready = false;  // until every table of the new weights is on the device
  auto up = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream);
  };
  hipError_t e = hipSuccess;
  for (int L = 0; e == hipSuccess && L < kDecLayers; ++L) {
    e = up(h->dec_whi[L], t.w_hi[L].data(), t.w_hi[L].size() * 2);
    if (e == hipSuccess) e = up(h->dec_wlo[L], t.w_lo[L].data(), t.w_lo[L].size() * 2);
    if (e == hipSuccess) e = up(h->dec_shift[L], t.shift[L].data(), t.shift[L].size() * 4);
  }
  if (e == hipSuccess) e = up(h->dec_w6, t.w6.data(), t.w6.size() * 4);
  if (e == hipSuccess) e = up(h->dec_b6, t.b6.data(), t.b6.size() * 4);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "decoder upload");
  for (int L = 0; L < kDecLayers; ++L) h->dec_inv_scale[L] = t.inv_scale[L];
  h->dec_ready = true;
  return PLAN_OK;
}

plan_status plan_profile(plan_handle *h, int32_t enable) {
  if (!h) return PLAN_E_INVALID;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto &e : h->ev_pending) h->ev_free.push_back(e.second);
  h->ev_pending.clear();
  for (int k = 0; k < 3; ++k) {
    h->prof_ms[k] = 0.0;
    h->prof_count[k] = 0;
  }
  h->profiling = enable != 0;
  return PLAN_OK;
}

plan_status plan_profile_read(plan_handle *h, double ms[3], int64_t count[3]) {
  if (!h || !ms || !count) return fail(h, PLAN_E_INVALID, "bad arguments");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto &e : h->ev_pending) {
    float t = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&t, e.second.first, e.second.second));
    h->prof_ms[e.first] += t;
    h->prof_count[e.first] += 1;
    h->ev_free.push_back(e.second);
  }
  h->ev_pending.clear();
  for (int k = 0; k < 3; ++k) {
    ms[k] = h->prof_ms[k];
    count[k] = h->prof_count[k];
  }
  return PLAN_OK;
}

}  // extern "C"
