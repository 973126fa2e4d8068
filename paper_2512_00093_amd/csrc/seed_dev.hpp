// Device-side initialisation of a RANMAR state from an integer seed
// (Haramoto & Suzuki, arXiv 2512.00093, Appendix A, Algorithm 3), one lane per
// seed.
//
// The initialisation runs two small generators for 97 x 24 steps:
//   - a three-term multiplicative generator mod 179,  m = i*j*k mod 179
//     (the printed Quotient(i*j,179) is read as Remainder: with the quotient,
//     seed 1 would give m = 0 for ever and an all-zero state);
//   - a linear congruential generator l <- (53 l + 1) mod 169,
// and sets bit (23 - step) of word u_ii when (l*m) mod 64 >= 32.  Word u_ii
// (ii = 1..97) lands in state slot x[97 - ii]: Algorithm 2 starts with i = 97
// as its oldest word, so u_97 is the oldest (x[0]) and u_1 the newest.
#pragma once

#include "common.hpp"

namespace ranmar {

// x mod 179 for x < 2^23 (all products i*j*k of residues in [1,178] are
// below 178^3 < 2^23): q = floor(2x * 11997116 / 2^32) = floor(x / 179)
// on that range (11997116 = ceil(2^31 / 179)).
__device__ __forceinline__ uint32_t mod179(uint32_t x) {
  const uint32_t q = mulhi24(x << 1, 11997116u);
  return x - mul24(q, 179u);  // q < 2^16: the full-rate 24-bit multiply is exact
}

// y mod 169 for y < 15196: q = floor(y * 6205 / 2^20), 6205 = ceil(2^20/169).
__device__ __forceinline__ uint32_t mod169(uint32_t y) {
  uint32_t q = mul24(y, 6205u) >> 20;
  return y - 169u * q;
}

// Writes the 97 words and c of the seeded state to dst[0..97] (stride
// `stride` words between consecutive words).  Returns false for a seed out of
// [1, 9e8]; then nothing is written.
__device__ __forceinline__ bool seed_state(int32_t seed, uint32_t* dst, int stride = 1) {
  if (seed < 1 || seed > 900000000) return false;
  const uint32_t s1 = (uint32_t)seed - 1u;
  const uint32_t ij = s1 / 30082u;
  const uint32_t kl = s1 - 30082u * ij;
  uint32_t i = (ij / 177u) % 177u + 2u;
  uint32_t j = ij % 177u + 2u;
  uint32_t k = (kl / 169u) % 178u + 1u;
  uint32_t l = kl % 169u;
  for (int ii = 1; ii <= 97; ++ii) {
    uint32_t acc = 0;
#pragma unroll
    for (int jj = 0; jj < 24; jj += 3) {
      // Three steps per round so that (i, j, k) rotate by renaming.
      uint32_t m0 = mod179(mul24(mul24(i, j), k));
      l = mod169(mad24(l, 53u, 1u));
      acc = (acc << 1) | ((mul24(l, m0) >> 5) & 1u);
      uint32_t m1 = mod179(mul24(mul24(j, k), m0));
      l = mod169(mad24(l, 53u, 1u));
      acc = (acc << 1) | ((mul24(l, m1) >> 5) & 1u);
      uint32_t m2 = mod179(mul24(mul24(k, m0), m1));
      l = mod169(mad24(l, 53u, 1u));
      acc = (acc << 1) | ((mul24(l, m2) >> 5) & 1u);
      i = m0;
      j = m1;
      k = m2;
    }
    dst[(97 - ii) * stride] = acc;
  }
  dst[97 * stride] = kC0;
  return true;
}

}  // namespace ranmar
