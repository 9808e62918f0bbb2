// rng.h -- counter-based random numbers of the samplers (device code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plan {

// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the request
// seed; counter (sample, upper iteration, block, 0). Box-Muller turns pairs of
// uniforms in (0, 1] into normals.

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c[0];
    uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2];
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void rng_block(uint64_t seed, int j, int l, int blk, uint32_t w[4]) {
  w[0] = (uint32_t)j;
  w[1] = (uint32_t)l;
  w[2] = (uint32_t)blk;
  w[3] = 0u;
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ float u01(uint32_t x) {
  return (float)((x >> 8) + 1u) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ void normals2(uint32_t a, uint32_t b, float &n0, float &n1) {
  float rad = sqrtf(-2.0f * logf(u01(a)));
  float s, c;
  sincospif(2.0f * u01(b), &s, &c);
  n0 = rad * c;
  n1 = rad * s;
}

}  // namespace plan
