// decoder.hip -- the decoder sampler on the device: the learned initial
// sampler of Sec. III-D at inference (App. A, decoder table). Sample j of a
// request is p_j = MLP([o, z_j]) with o the request's observation and z_j the
// Box-Muller pair of Philox block (j, 0, 0, 0) under its seed.
//
// The rows being decoded (every sample of every request that starts from
// the decoder at this upper iteration) are processed in chunks of up to
// kDecChunk rows, as one batch for all requests (the weights are shared):
//   blocks 1-5  64 -> 1024, 1024 -> 1024 (three times), 1024 -> 256: matrix
//             cores; block 1 builds its input [o, z] (57, padded to 64)
//             while loading its operands. Every
//             operand is an FP16 high/low pair and each product is
//             hi*hi + hi*lo + lo*hi with FP32 accumulation
//             (v_mfma_f32_16x16x32_f16), about 22 significant bits. The
//             epilogue applies 2^-e, the folded BatchNorm/bias shift and the
//             ReLU, and splits the result for the next layer.
//   output    256 -> 8: FP32, one wave per row, written into the sample rows
//             the lower level reads at iteration 0.
// The BatchNorm of each block (inference form) and the Linear bias are
// folded into the Linear weights and one shift per output on the host, in
// FP64. Everything is in a fixed order: the same rows give the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_internal.h"
#include "rng.h"

namespace plan {
namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Segment of concatenated row r (segments in increasing row_begin).
__device__ __forceinline__ int find_seg(const DecSeg *seg, int nseg, int r) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid].row_begin <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// v = hi + lo: hi is v cut to 11 significant bits (exact in FP16 in its
// normal range), lo the remainder after the FP16 hi, rounded to FP16.
__device__ __forceinline__ void split_act(float v, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)__uint_as_float(__float_as_uint(v) & 0xFFFFE000u);
  lo = (_Float16)(v - (float)hi);
}

// Tile of this workgroup, XCD-aware: workgroups are dispatched round-robin
// over the 8 XCDs (each with its own L2), so workgroup b runs on XCD b % 8.
// split2d (the 1024 -> 1024 layers, whose weights and activations are about
// the same size) and a tile grid that splits evenly: XCD x takes one block
// of a 4 x 2 split of the grid (a quarter of the output features, half of
// the rows), so each L2 reads a quarter of the weights and half of the
// activations instead of all the weights (measured: 37.8 -> 24 MB fetched
// per layer at 1000 rows). Otherwise logical tiles go to XCDs in contiguous
// ranges (n fastest, then rows), which keeps each XCD on its own rows: best
// where the weights are the smaller operand. The remainder of the grid keeps
// the identity map. Tiles are independent: the map changes where a tile
// runs, not its result.
__device__ __forceinline__ void xcd_tile(bool split2d, int &tx, int &ty) {
  const int gx = gridDim.x, gy = gridDim.y, T = gx * gy, b = blockIdx.y * gx + blockIdx.x;
  if (split2d && gx % 4 == 0 && gy % 2 == 0) {
    const int x = b % 8, i = b / 8, qx = gx / 4, hy = gy / 2;
    tx = (x % 4) * qx + i % qx;
    ty = (x / 4) * hy + i / qx;
    return;
  }
  const int per = T / 8;
  const int t = b < 8 * per ? (b % 8) * per + b / 8 : b;
  tx = t % gx;
  ty = t / gx;
}

// Operand layout of the matrix-core layers ("fragment-major"): a matrix of
// R rows (a multiple of 16) and K columns (a multiple of 32) of FP16 halves
// is stored as 16 x 32 fragments, fragment (r / 16, k / 32) at h8 offset
// ((r / 16) (K / 32) + k / 32) 64, and inside it the 8 halves k .. k + 7 (k
// a multiple of 8) of row r at h8 (r % 16) + 16 ((k / 8) % 4): exactly the
// 16 bytes lane (r % 16) + 16 ((k / 8) % 4) of v_mfma_f32_16x16x32_f16
// supplies. One operand load of a wave is then 1 KB of contiguous memory.
__device__ __forceinline__ size_t frag_half(int r, int k, int K) {
  return ((((size_t)(r >> 4) * (K >> 5) + (k >> 5)) * 64 + (r & 15) + 16 * ((k >> 3) & 3)) << 3) + (k & 7);
}

// ReLU that keeps a NaN: an activation beyond the FP16 range splits into
// +-inf halves, whose products give NaN in the next layer; it must reach the
// samples (and fail the request there) instead of being cut to 0.
__device__ __forceinline__ float relu_keep_nan(float v) { return v > 0.f ? v : (v == v ? 0.f : v); }

// Where block 1's input comes from: the requests' observations and the
// latent draws of their samples (rows r0.. of the chunk).
struct DecIn {
  const ReqDesc *desc;
  const DecSeg *seg;
  int nseg, r0;
};

// Halves k0 .. k0 + 7 of block 1's input for chunk row rl: [o, z_j] of the
// row's request and sample (z_j the Box-Muller pair of Philox block
// (j, 0, 0, 0)), zero past the 57 inputs, split into FP16 high/low.
__device__ __forceinline__ void input_h8(const DecIn &in, int rl, int k0, h8 &hi, h8 &lo) {
  const int r = in.r0 + rl;
  const DecSeg sg = in.seg[find_seg(in.seg, in.nseg, r)];
  const ReqDesc &D = in.desc[sg.slot];
  float z0 = 0.f, z1 = 0.f;
  if (k0 + 8 > PLAN_OBS_DIM && k0 < kDecIn) {
    uint32_t w[4];
    rng_block(D.seed, r - sg.row_begin, 0, 0, w);
    normals2(w[0], w[1], z0, z1);
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e;
    const float v = k < PLAN_OBS_DIM ? (float)D.obsv[k] : (k == PLAN_OBS_DIM ? z0 : (k < kDecIn ? z1 : 0.f));
    _Float16 h, l;
    split_act(v, h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

// Blocks 1-5: out = relu(inv_scale (W x) + shift) as C^T = W X^T on the
// matrix cores, operands and result in the fragment-major layout. In
// v_mfma_f32_16x16x32_f16 lane l supplies 8 consecutive k of W row (feature)
// l % 16 and of X row (sample) l % 16 and gets back features
// 4 (l / 16) .. + 3 of sample l % 16. KSPLIT = 1: the four waves of a
// workgroup own 2 x 2 tiles of 16 TN features x 16 TM rows. KSPLIT = 4: they
// share one tile and split its K-steps in four; the partials meet in LDS and
// wave 0 adds them in wave order (((w0 + w1) + w2) + w3) before the
// epilogue (more waves per tile hide the operand loads at small row counts).
// The summation order depends on KSPLIT only, never on the tile shape. The
// next D K-steps' operands are loaded while a step's products run. INPUT:
// block 1, whose input operand is built from the requests while loading.
template <int TN, int TM, int KSTEPS, int KSPLIT, bool INPUT>
__global__ void __launch_bounds__(kWave *(KSPLIT > 4 ? KSPLIT : 4)) dec_gemm_kernel(DecLayer Ly, const uint16_t *in_hi, const uint16_t *in_lo,
                                                       DecIn in, uint16_t *out_hi, uint16_t *out_lo, int nrows) {
  constexpr int KW = KSTEPS / KSPLIT;  // K-steps of one wave
  constexpr int D = 2;
  __shared__ f4 s_part[KSPLIT > 1 ? KSPLIT - 1 : 1][TN][TM][kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  int tx, ty;
  xcd_tile(Ly.n_in == Ly.n_out, tx, ty);
  const int wn = KSPLIT == 1 ? (wave & 1) : 0, wm = KSPLIT == 1 ? (wave >> 1) : 0;
  const int n_base = (tx * (KSPLIT == 1 ? 2 : 1) + wn) * 16 * TN;
  const int m_base = (ty * (KSPLIT == 1 ? 2 : 1) + wm) * 16 * TM;
  const int s0 = KSPLIT == 1 ? 0 : wave * KW;  // first K-step of this wave
  const h8 *whi = reinterpret_cast<const h8 *>(Ly.w_hi), *wlo = reinterpret_cast<const h8 *>(Ly.w_lo);
  const h8 *xhi = reinterpret_cast<const h8 *>(in_hi), *xlo = reinterpret_cast<const h8 *>(in_lo);
  // row blocks past the chunk read its last block (in bounds) and are not stored
  const int mb_last = (nrows - 1) >> 4;
  const h8 *xh[TM], *xl[TM];
  const h8 *wh[TN], *wl[TN];
#pragma unroll
  for (int bm = 0; bm < TM; ++bm) {
    const int mb = min((m_base >> 4) + bm, mb_last);
    const size_t off = ((size_t)mb * KSTEPS + s0) * 64 + lane;
    xh[bm] = INPUT ? nullptr : xhi + off;  // block 1 reads no input buffer
    xl[bm] = INPUT ? nullptr : xlo + off;
  }
#pragma unroll
  for (int bn = 0; bn < TN; ++bn) {
    const size_t off = ((size_t)((n_base >> 4) + bn) * KSTEPS + s0) * 64 + lane;
    wh[bn] = whi + off;
    wl[bn] = wlo + off;
  }
  f4 acc[TN][TM];
#pragma unroll
  for (int bn = 0; bn < TN; ++bn)
#pragma unroll
    for (int bm = 0; bm < TM; ++bm) acc[bn][bm] = f4{0.f, 0.f, 0.f, 0.f};
  h8 ah[D][TN], al[D][TN], bh[D][TM], bl[D][TM];
  auto load = [&](int step, int d) {
    const int o = 64 * step;
#pragma unroll
    for (int bn = 0; bn < TN; ++bn) {
      ah[d][bn] = wh[bn][o];
      al[d][bn] = wl[bn][o];
    }
#pragma unroll
    for (int bm = 0; bm < TM; ++bm) {
      if constexpr (INPUT) {
        // block 1 builds its input operand from the requests (KSPLIT = 1)
        input_h8(in, min(m_base + 16 * bm + i16, nrows - 1), 32 * step + 8 * g, bh[d][bm], bl[d][bm]);
      } else {
        bh[d][bm] = xh[bm][o];
        bl[d][bm] = xl[bm][o];
      }
    }
  };
#pragma unroll
  for (int d = 0; d < D && d < KW; ++d) load(d, d);
#pragma unroll
  for (int step = 0; step < KW; ++step) {
    const int d = step % D;
#pragma unroll
    for (int bn = 0; bn < TN; ++bn)
#pragma unroll
      for (int bm = 0; bm < TM; ++bm) {
        acc[bn][bm] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[d][bn], bh[d][bm], acc[bn][bm], 0, 0, 0);
        acc[bn][bm] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[d][bn], bl[d][bm], acc[bn][bm], 0, 0, 0);
        acc[bn][bm] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[d][bn], bh[d][bm], acc[bn][bm], 0, 0, 0);
      }
    if (step + D < KW) load(step + D, d);
  }
  if constexpr (KSPLIT > 1) {
    if (wave > 0) {
#pragma unroll
      for (int bn = 0; bn < TN; ++bn)
#pragma unroll
        for (int bm = 0; bm < TM; ++bm) s_part[wave - 1][bn][bm][lane] = acc[bn][bm];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int bn = 0; bn < TN; ++bn)
#pragma unroll
      for (int bm = 0; bm < TM; ++bm)
#pragma unroll
        for (int w = 0; w < KSPLIT - 1; ++w) acc[bn][bm] += s_part[w][bn][bm][lane];
  }
  const int Kn = Ly.n_out;  // K of the next layer's input
#pragma unroll
  for (int bn = 0; bn < TN; ++bn) {
    const int n = n_base + 16 * bn + 4 * g;
    const float4 sh = *reinterpret_cast<const float4 *>(Ly.shift + n);
    const float shv[4] = {sh.x, sh.y, sh.z, sh.w};
#pragma unroll
    for (int bm = 0; bm < TM; ++bm) {
      const int m = m_base + 16 * bm + i16;
      if (m >= nrows) continue;
      h4 hi, lo;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float v = relu_keep_nan(fmaf(acc[bn][bm][u], Ly.inv_scale, shv[u]));
        _Float16 h, l;
        split_act(v, h, l);
        hi[u] = h;
        lo[u] = l;
      }
      const size_t o = frag_half(m, n, Kn);  // n % 8 is 0 or 4: four consecutive halves
      *reinterpret_cast<h4 *>(out_hi + o) = hi;
      *reinterpret_cast<h4 *>(out_lo + o) = lo;
    }
  }
}

// Output layer: p = W6 h5 + b6 (FP32), one wave per row, lane l holding
// features 4l .. 4l + 3; the eight dot products are summed over the wave in
// a fixed butterfly order and written into the request's sample row.
__global__ void __launch_bounds__(256) dec_out_kernel(DecArgs A, const uint16_t *h_hi, const uint16_t *h_lo) {
  const int lane = threadIdx.x & 63;
  const int rl = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (rl >= A.nrows) return;
  const size_t base = frag_half(rl, 4 * lane, kDecHidden5);
  const h4 hh = *reinterpret_cast<const h4 *>(h_hi + base);
  const h4 hl = *reinterpret_cast<const h4 *>(h_lo + base);
  float h[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) h[u] = (float)hh[u] + (float)hl[u];
  float s[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const float4 w = *reinterpret_cast<const float4 *>(A.w6 + a * kDecHidden5 + 4 * lane);
    float v = w.x * h[0];
    v = fmaf(w.y, h[1], v);
    v = fmaf(w.z, h[2], v);
    v = fmaf(w.w, h[3], v);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    s[a] = v;
  }
  if (lane == 0) {
    const int r = A.r0 + rl;
    const DecSeg sg = A.seg[find_seg(A.seg, A.nseg, r)];
    const ReqDesc &D = A.desc[sg.slot];
    float *dst = A.p + (size_t)(D.row_off + (r - sg.row_begin)) * 8;
    const bool goals = A.behaviour == PLAN_BEHAV_GOALS;
    float out[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) out[a] = (goals && a >= 2) ? 0.f : s[a] + A.b6[a];
    reinterpret_cast<float4 *>(dst)[0] = make_float4(out[0], out[1], out[2], out[3]);
    reinterpret_cast<float4 *>(dst)[1] = make_float4(out[4], out[5], out[6], out[7]);
  }
}

template <int TN, int TM, int KSTEPS, int KSPLIT, bool INPUT = false>
hipError_t gemm_launch(const DecLayer &Ly, const uint16_t *ih, const uint16_t *il, const DecIn &in, uint16_t *oh,
                       uint16_t *ol, int nrows, hipStream_t st) {
  constexpr int tn = (KSPLIT == 1 ? 32 : 16) * TN, tm = (KSPLIT == 1 ? 32 : 16) * TM;
  if (Ly.n_in != 32 * KSTEPS || Ly.n_out % tn != 0) return hipErrorInvalidValue;
  const dim3 grid(Ly.n_out / tn, (nrows + tm - 1) / tm);
  hipLaunchKernelGGL((dec_gemm_kernel<TN, TM, KSTEPS, KSPLIT, INPUT>), grid, dim3(kWave * (KSPLIT > 4 ? KSPLIT : 4)),
                     0, st, Ly, ih, il, in, oh, ol, nrows);
  return hipGetLastError();
}

// Block 1 (K = 64): four waves on 2 x 2 tiles of 32 x 16 (measured best
// at 1000 rows: 3.6 us). Blocks 2-5 (K = 1024): K split in four, tile
// 32 x 64 while that gives two workgroups per CU, else 32 x 32 while it
// fills each CU once, else 32 x 16 (measured at 1000 and 16384 rows: 15 and
// 179 us for 1024 -> 1024, 6.3 us for 1024 -> 256 at 1000 rows).
hipError_t gemm_layer(const DecLayer &Ly, const uint16_t *ih, const uint16_t *il, const DecIn &in, uint16_t *oh,
                      uint16_t *ol, int nrows, int n_cu, hipStream_t st) {
  if (Ly.n_in == kDecInPad) return gemm_launch<2, 1, kDecInPad / 32, 1, true>(Ly, ih, il, in, oh, ol, nrows, st);
  if (Ly.n_in != kDecHidden) return hipErrorInvalidValue;
  auto wgs = [&](int tn, int tm) { return (long)(Ly.n_out / (16 * tn)) * ((nrows + 16 * tm - 1) / (16 * tm)); };
  constexpr int KS = kDecHidden / 32;
  if (wgs(2, 4) >= 2L * n_cu) return gemm_launch<2, 4, KS, 4>(Ly, ih, il, in, oh, ol, nrows, st);
  if (wgs(2, 2) >= (long)n_cu) return gemm_launch<2, 2, KS, 4>(Ly, ih, il, in, oh, ol, nrows, st);
  return gemm_launch<2, 1, KS, 4>(Ly, ih, il, in, oh, ol, nrows, st);
}

}  // namespace

// All decoder kernels for total_rows concatenated rows, chunk by chunk, on
// stream st; ev0/ev1 (optional) are recorded around the whole sequence.
hipError_t launch_decoder(const DecArgs &a0, int total_rows, int n_cu, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1) {
  static const int n_in[kDecLayers] = {kDecInPad, kDecHidden, kDecHidden, kDecHidden, kDecHidden};
  static const int n_out[kDecLayers] = {kDecHidden, kDecHidden, kDecHidden, kDecHidden, kDecHidden5};
  for (int i = 0; i < kDecLayers; ++i)
    if (a0.layer[i].n_in != n_in[i] || a0.layer[i].n_out != n_out[i]) return hipErrorInvalidValue;
  if (ev0) {
    const hipError_t e = hipEventRecord(ev0, st);
    if (e != hipSuccess) return e;
  }
  for (int r0 = 0; r0 < total_rows; r0 += kDecChunk) {
    DecArgs a = a0;
    a.r0 = r0;
    a.nrows = total_rows - r0 < kDecChunk ? total_rows - r0 : kDecChunk;
    const DecIn in{a.desc, a.seg, a.nseg, a.r0};
    hipError_t e = gemm_layer(a.layer[0], nullptr, nullptr, in, a.act_hi[0], a.act_lo[0], a.nrows, n_cu, st);
    int cur = 0;
    for (int i = 1; e == hipSuccess && i < kDecLayers; ++i) {
      e = gemm_layer(a.layer[i], a.act_hi[cur], a.act_lo[cur], in, a.act_hi[cur ^ 1], a.act_lo[cur ^ 1], a.nrows,
                     n_cu, st);
      cur ^= 1;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dec_out_kernel, dim3((a.nrows + 3) / 4), dim3(256), 0, st, a, a.act_hi[cur], a.act_lo[cur]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev1) return hipEventRecord(ev1, st);
  return hipSuccess;
}

}  // namespace plan
