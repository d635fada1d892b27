// Counter-based random numbers of the device code: Philox4x32-10 (Salmon,
// Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11), counter (row, block, stream, problem), key (seed low word, seed
// high word).  Word i of a stream is word i%4 of block i/4; uniform i takes
// 53 bits from the two words of half block i%2 of block i/2; a standard
// normal is the cosine branch of Box-Muller from uniform i of two streams.
#pragma once
#include "internal.h"

namespace sb {

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ inline uint32_t rng_word(uint64_t seed, uint32_t problem, uint32_t ray, uint32_t stream,
                                    uint32_t i) {
  uint32_t c[4] = {ray, i >> 2, stream, problem};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return c[i & 3u];
}

__device__ inline double rng_uniform(uint64_t seed, uint32_t problem, uint32_t ray,
                                     uint32_t stream, uint32_t i) {
  uint32_t c[4] = {ray, i >> 1, stream, problem};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t a = c[2u * (i & 1u)], b = c[2u * (i & 1u) + 1u];
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Standard normal i of counter row `row`: uniforms i of streams `stream` and
// `stream` + 1 (the sunburst rays draw their directions the same way).
__device__ inline double rng_normal(uint64_t seed, uint32_t problem, uint32_t row,
                                    uint32_t stream, uint32_t i) {
  const double u1 = rng_uniform(seed, problem, row, stream, i);
  const double u2 = rng_uniform(seed, problem, row, stream + 1u, i);
  return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
}

}  // namespace sb
