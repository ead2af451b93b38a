// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11) and the Box-Muller transform, device side.
//
// Each round multiplies words 0 and 2 by two fixed odd constants, keeps the
// high and low 32-bit halves of the products, and mixes the high halves with
// words 1 and 3 and the round key; the key advances by two Weyl increments
// (golden-ratio and sqrt(3)-1 fractions) after every round.  Ten rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace vip {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  const uint32_t w0 = 0x9E3779B9u, w1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = m0 * c[0], hi0 = __umulhi(m0, c[0]);
    uint32_t lo1 = m1 * c[2], hi1 = __umulhi(m1, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += w0;
    k1 += w1;
  }
}

// Four standard normals for quad q of the stream (elements 4q .. 4q+3):
// counter (q lo, q hi, stream lo, stream hi), key (seed lo, seed hi).
__device__ __forceinline__ void philox_normals4(uint64_t q, uint32_t k0, uint32_t k1, uint32_t s0,
                                                uint32_t s1, float z[4]) {
  uint32_t c[4] = {uint32_t(q), uint32_t(q >> 32), s0, s1};
  philox4x32_10(c, k0, k1);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float u1 = (float(c[2 * p]) + 1.0f) * 2.3283064365386963e-10f;   // (x + 1) 2^-32, in (0, 1]
    float u2 = float(c[2 * p + 1]) * 2.3283064365386963e-10f;        // x 2^-32, in [0, 1)
    float r = sqrtf(-2.0f * logf(u1));
    float s, co;
    sincosf(6.2831853071795865f * u2, &s, &co);
    z[2 * p] = r * co;
    z[2 * p + 1] = r * s;
  }
}

}  // namespace vip
