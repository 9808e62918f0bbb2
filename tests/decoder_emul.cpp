// CPU emulation of the decoder sampler's tables and arithmetic.
//
// Builds the decoder tables with the library's own host code (build_decoder:
// BatchNorm folding, power-of-two scaling, FP16 high/low split, fragment-
// major packing), then runs the device arithmetic in software: the input
// split, five matrix-core layers read through the documented operand layout
// (fragment (r / 16, k / 32) at h8 ((r / 16) (K / 32) + k / 32) 64, lane
// (r % 16) + 16 ((k / 8) % 4) holding halves k .. k + 7 of row r), the
// hi*hi + hi*lo + lo*hi products summed in FP32 with the K split of the
// kernels, the epilogue (2^-e, shift, ReLU, split) and the FP32 output
// layer. Compares
//   * every packed weight, hi + lo, with the folded FP64 weight times 2^e,
//   * the samples p with the FP64 reference written by the test,
// and exits non-zero if a bound is exceeded.
//
// usage: decoder_emul <dir> <rows>; <dir> holds raw little-endian float64
// files W0..W5, b0..b5, g0..g4, be0..be4, m0..m4, v0..v4 (weights), eps, x
// (rows x 57 inputs [o, z]) and p_ref (rows x 8).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "precompute.h"

using namespace plan;

namespace {

std::vector<double> read_f64(const std::string &path, size_t n) {
  std::vector<double> v(n, 0.0);
  FILE *f = std::fopen(path.c_str(), "rb");
  if (!f || std::fread(v.data(), 8, n, f) != n) {
    std::fprintf(stderr, "cannot read %s\n", path.c_str());
    std::exit(2);
  }
  std::fclose(f);
  return v;
}

float half_to_float(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (float)h;
}

// the device's activation split: hi = v cut to 11 significant bits, lo = the
// remainder after the FP16 hi, rounded to FP16
void split_act(float v, float &hi, float &lo) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  u &= 0xFFFFE000u;
  float c;
  std::memcpy(&c, &u, 4);
  hi = (float)(_Float16)c;
  lo = (float)(_Float16)(v - hi);
}

// half k of row r of a K-column matrix stored in the fragment layout, read
// the way lane (r % 16) + 16 ((k / 8) % 4) of one operand load reads it
size_t lane_half(int r, int k, int K) {
  const size_t frag = (size_t)(r / 16) * (K / 32) + k / 32;
  const int lane = (r % 16) + 16 * ((k / 8) % 4);
  return (frag * 64 + lane) * 8 + (k % 8);
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 3) return 2;
  const std::string dir = argv[1];
  const int rows = std::atoi(argv[2]);
  static const int n_in[6] = {kDecIn, kDecHidden, kDecHidden, kDecHidden, kDecHidden, kDecHidden5};
  static const int n_out[6] = {kDecHidden, kDecHidden, kDecHidden, kDecHidden, kDecHidden5, PLAN_NP};
  std::vector<double> W[6], b[6], g[5], be[5], mu[5], var[5];
  plan_decoder dec{};
  for (int i = 0; i < 6; ++i) {
    W[i] = read_f64(dir + "/W" + std::to_string(i), (size_t)n_out[i] * n_in[i]);
    b[i] = read_f64(dir + "/b" + std::to_string(i), n_out[i]);
    dec.W[i] = W[i].data();
    dec.b[i] = b[i].data();
  }
  for (int i = 0; i < 5; ++i) {
    g[i] = read_f64(dir + "/g" + std::to_string(i), n_out[i]);
    be[i] = read_f64(dir + "/be" + std::to_string(i), n_out[i]);
    mu[i] = read_f64(dir + "/m" + std::to_string(i), n_out[i]);
    var[i] = read_f64(dir + "/v" + std::to_string(i), n_out[i]);
    dec.bn_gamma[i] = g[i].data();
    dec.bn_beta[i] = be[i].data();
    dec.bn_mean[i] = mu[i].data();
    dec.bn_var[i] = var[i].data();
  }
  dec.bn_eps = read_f64(dir + "/eps", 1)[0];
  const std::vector<double> x = read_f64(dir + "/x", (size_t)rows * kDecIn);
  const std::vector<double> p_ref = read_f64(dir + "/p_ref", (size_t)rows * PLAN_NP);

  DecoderTables t;
  if (const char *why = build_decoder(dec, t)) {
    std::printf("build_decoder refused: %s\n", why);
    return 1;
  }

  // 1. packed weights against the folded FP64 weights
  double w_err = 0.0;
  for (int i = 0; i < kDecLayers; ++i) {
    const int K = i == 0 ? kDecInPad : n_in[i];
    const double s2 = 1.0 / t.inv_scale[i];
    for (int n = 0; n < n_out[i]; ++n) {
      const double sc = g[i][n] / std::sqrt(var[i][n] + dec.bn_eps);
      for (int k = 0; k < K; ++k) {
        const size_t q = lane_half(n, k, K);
        const double got = (double)half_to_float(t.w_hi[i][q]) + (double)half_to_float(t.w_lo[i][q]);
        const double want = k < n_in[i] ? sc * W[i][(size_t)n * n_in[i] + k] * s2 : 0.0;
        w_err = std::max(w_err, std::fabs(got - want));
      }
      const double sh = sc * (b[i][n] - mu[i][n]) + be[i][n];
      if (std::fabs(t.shift[i][n] - sh) > 1e-6 * (1.0 + std::fabs(sh))) {
        std::printf("shift of layer %d output %d: %g vs %g\n", i, n, t.shift[i][n], sh);
        return 1;
      }
    }
  }

  // 2. the device arithmetic on the inputs
  std::vector<float> ahi((size_t)rows * kDecInPad, 0.f), alo((size_t)rows * kDecInPad, 0.f);
  for (int r = 0; r < rows; ++r)
    for (int k = 0; k < kDecIn; ++k) split_act((float)x[(size_t)r * kDecIn + k], ahi[(size_t)r * kDecInPad + k],
                                               alo[(size_t)r * kDecInPad + k]);
  int K = kDecInPad;
  for (int i = 0; i < kDecLayers; ++i) {
    const int N = n_out[i];
    const int split = i == 0 ? 1 : 4, steps = K / 32, per = steps / split;
    std::vector<float> nhi((size_t)rows * N), nlo((size_t)rows * N);
    std::vector<float> whi((size_t)N * K), wlo((size_t)N * K);
    for (int n = 0; n < N; ++n)
      for (int k = 0; k < K; ++k) {
        whi[(size_t)n * K + k] = half_to_float(t.w_hi[i][lane_half(n, k, K)]);
        wlo[(size_t)n * K + k] = half_to_float(t.w_lo[i][lane_half(n, k, K)]);
      }
    for (int r = 0; r < rows; ++r)
      for (int n = 0; n < N; ++n) {
        float total = 0.f;
        for (int w = 0; w < split; ++w) {
          float acc = 0.f;
          for (int s = w * per; s < (w + 1) * per; ++s) {
            float sh = 0.f, sl = 0.f, sl2 = 0.f;
            for (int k = 32 * s; k < 32 * s + 32; ++k) {
              const float xh = ahi[(size_t)r * K + k], xl = alo[(size_t)r * K + k];
              sh += whi[(size_t)n * K + k] * xh;
              sl += whi[(size_t)n * K + k] * xl;
              sl2 += wlo[(size_t)n * K + k] * xh;
            }
            acc = ((acc + sh) + sl) + sl2;
          }
          total = w == 0 ? acc : total + acc;
        }
        float v = std::fmaf(total, t.inv_scale[i], t.shift[i][n]);
        v = v > 0.f ? v : 0.f;
        split_act(v, nhi[(size_t)r * N + n], nlo[(size_t)r * N + n]);
      }
    ahi.swap(nhi);
    alo.swap(nlo);
    K = N;
  }
  double p_err = 0.0;
  std::vector<double> pmax(PLAN_NP, 0.0);
  for (int r = 0; r < rows; ++r)
    for (int a = 0; a < PLAN_NP; ++a) pmax[a] = std::max(pmax[a], std::fabs(p_ref[(size_t)r * PLAN_NP + a]));
  bool ok = w_err <= 1e-6;
  for (int r = 0; r < rows; ++r)
    for (int a = 0; a < PLAN_NP; ++a) {
      float s = 0.f;
      for (int k = 0; k < kDecHidden5; ++k)
        s = std::fmaf(t.w6[(size_t)a * kDecHidden5 + k], ahi[(size_t)r * K + k] + alo[(size_t)r * K + k], s);
      const double p = (double)(s + t.b6[a]);
      const double e = std::fabs(p - p_ref[(size_t)r * PLAN_NP + a]);
      p_err = std::max(p_err, e);
      if (e > 1e-5 + 2e-6 * (1.0 + pmax[a])) ok = false;
    }
  std::printf("packed weights: max |hi + lo - W' 2^e| = %.3e; samples: max |p - p_ref| = %.3e (%s)\n", w_err, p_err,
              ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}
