// Device-side exact jump-ahead of RANMAR (Haramoto & Suzuki, arXiv
// 2512.00093, Sec. 3.1 and 3.2), one request per lane, everything in VGPRs.
//
//   P_J(t) = t^J mod phi(t) in (Z/2^24)[t],  phi = t^97 + t^64 - 1
// by left-to-right square-and-multiply.  A squaring is a 97x97 schoolbook
// product using the symmetry c_k = 2 sum_{i<k-i} a_i a_{k-i} + a_{k/2}^2
// (4753 multiply-adds), reduced with t^97 = 1 - t^64.  Coefficients are kept
// unreduced mod 2^32: every multiply reads only the low 24 bits of its
// operands, and reduction mod 2^32 -> mod 2^24 is a ring homomorphism, so
// masking once at the end gives the exact residues.
//
// The state is then moved by Horner's rule (Sec. 3.1):
//   uP(A) = (...((b_96 uA + b_95 u)A + b_94 u)A + ... ) + b_0 u,
// where vA = f_1(v) = (v_2, ..., v_97, v_1 - v_65).
#pragma once

#include "common.hpp"

namespace ranmar {


// Coefficients K and K-1 of a*a (both before reduction), two chains
// interleaved so that consecutive multiply-adds are independent.
template <int K>
__device__ __forceinline__ void sq_pair(const uint32_t (&a)[97], uint32_t& s0, uint32_t& s1) {
  constexpr int lo0 = (K - 96) > 0 ? K - 96 : 0;
  constexpr int lo1 = (K - 97) > 0 ? K - 97 : 0;
  constexpr int n0 = (K + 1) / 2 - lo0;  // pairs i < K-i with i >= lo0
  constexpr int n1 = K / 2 - lo1;        // pairs i < K-1-i with i >= lo1
  constexpr int nmax = n0 > n1 ? n0 : n1;
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (int t = 0; t < nmax; ++t) {
    if (t < n0) s0 = mad24(a[lo0 + t], a[K - lo0 - t], s0);
    if (t < n1) s1 = mad24(a[lo1 + t], a[K - 1 - lo1 - t], s1);
  }
  s0 <<= 1;
  s1 <<= 1;
  if ((K & 1) == 0)
    s0 = mad24(a[K / 2], a[K / 2], s0);
  else
    s1 = mad24(a[(K - 1) / 2], a[(K - 1) / 2], s1);
}

// High half of the square: h[k-97] = c_k for k = 97..192.
template <int K>
struct SqHigh {
  __device__ __forceinline__ static void run(const uint32_t (&a)[97], uint32_t (&h)[96]) {
    uint32_t s0, s1;
    sq_pair<K>(a, s0, s1);
    h[K - 97] = s0;
    h[K - 98] = s1;
    SqHigh<K - 2>::run(a, h);
  }
};
template <>
struct SqHigh<96> {
  __device__ __forceinline__ static void run(const uint32_t (&)[97], uint32_t (&)[96]) {}
};

// Low half, computed from the top down so that a[k] can be overwritten as
// soon as c_k is known (c_j for j < k reads only a[0..j]).  After the high
// half has been folded onto itself (see sqr_mod), coefficient c_k of the
// reduced square is c_k + h'_{k+97} (k <= 95) - h'_{k+33} (k >= 64).
template <int K>
struct SqLow {
  __device__ __forceinline__ static void run(uint32_t (&a)[97], const uint32_t (&h)[96]) {
    uint32_t s0, s1;
    sq_pair<K>(a, s0, s1);
    if (K <= 95) s0 += h[K];
    if (K >= 64) s0 -= h[K - 64];
    if (K - 1 <= 95) s1 += h[K - 1];
    if (K - 1 >= 64) s1 -= h[K - 65];
    a[K] = s0;
    a[K - 1] = s1;
    SqLow<K - 2>::run(a, h);
  }
};
template <>
struct SqLow<0> {
  __device__ __forceinline__ static void run(uint32_t (&a)[97], const uint32_t (&h)[96]) {
    a[0] = mad24(a[0], a[0], h[0]);
  }
};

// a <- a^2 mod phi.
__device__ __forceinline__ void sqr_mod(uint32_t (&a)[97]) {
  uint32_t h[96];
  SqHigh<192>::run(a, h);
  // Fold the top of the high half into itself, highest power first:
  // t^k = t^(k-97) - t^(k-33); for k >= 130 the second term is still >= 97.
#pragma unroll
  for (int k = 192; k >= 130; --k) h[k - 130] -= h[k - 97];
  SqLow<96>::run(a, h);
}

// a <- t*a mod phi on lanes where `bit` is set: shift up one power and fold
// the overflowing t^97 = 1 - t^64.
__device__ __forceinline__ void mul_t_if(uint32_t (&a)[97], bool bit) {
  const uint32_t top = a[96];
#pragma unroll
  for (int k = 96; k >= 1; --k) a[k] = bit ? a[k - 1] : a[k];
  a[0] = bit ? top : a[0];
  a[64] -= bit ? top : 0u;
}

// Coefficient k (< 97) of a product of degree <= 192, prod[0..192], reduced
// mod phi (unmasked).  With h_j = prod[97 + j] and t^97 = 1 - t^64, t^(97+j)
// in low powers is: j <= 32: t^j - t^(64+j); 33..65: t^j - t^(j-33) +
// t^(j+31); 66..95: t^j - t^(j-33) + t^(j-66) - t^(j-2).
__device__ __forceinline__ uint32_t fold_phi(const uint32_t* prod, int k) {
  const uint32_t* h = prod + 97;
  uint32_t v = prod[k];
  if (k <= 95) v += h[k];
  if (k >= 64) v = v - h[k - 64] + h[k - 31];
  if (k <= 62) v -= h[k + 33];
  if (k <= 29) v += h[k + 66];
  if (k >= 64 && k <= 93) v -= h[k + 2];
  return v;
}

// 128-bit helpers on four 32-bit limbs.
__device__ __forceinline__ int u128_bitlen(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3) {
  if (j3) return 128 - __clz(j3);
  if (j2) return 96 - __clz(j2);
  if (j1) return 64 - __clz(j1);
  if (j0) return 32 - __clz(j0);
  return 0;
}

__device__ __forceinline__ uint32_t u128_bit(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3, int b) {
  const uint32_t limb = b < 32 ? j0 : b < 64 ? j1 : b < 96 ? j2 : j3;
  return (limb >> (b & 31)) & 1u;
}

// (J >> start) & 63 for a wave-uniform start in [0, 122].
__device__ __forceinline__ uint32_t u128_window6(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3, int start) {
  const uint64_t lo = ((uint64_t)j1 << 32) | j0;
  const uint64_t hi = ((uint64_t)j3 << 32) | j2;
  uint64_t w;
  if (start >= 64)
    w = hi >> (start - 64);
  else if (start == 0)
    w = lo;
  else
    w = (lo >> start) | (hi << (64 - start));
  return (uint32_t)w & 63u;
}

// a = t^J mod phi (unmasked; mask with kMask before export).  The loop runs
// over the wave's longest exponent: shorter exponents have leading zeros and
// the window starts at t^(top six bits), a monomial since 63 < 97.
__device__ __forceinline__ void xpow_lane(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3, uint32_t (&a)[97]) {
  const int B = wave_max_i32(u128_bitlen(j0, j1, j2, j3));
  const int start = B > 6 ? B - 6 : 0;
  const uint32_t top = u128_window6(j0, j1, j2, j3, start);
#pragma unroll
  for (int k = 0; k < 97; ++k) a[k] = (k == (int)top) ? 1u : 0u;
  for (int b = start - 1; b >= 0; --b) {
    sqr_mod(a);
    const bool bit = u128_bit(j0, j1, j2, j3, b) != 0;
    if (__any(bit)) mul_t_if(a, bit);
  }
}

// v = u P(A) by Horner's rule with the coefficients read from memory
// (bcoef[i], i = 0..96; consecutive coefficients `bstride` words apart).
// The shift of f_1 is folded into the register naming of the multiply-adds:
// new v[k] = b u[k] + old v[k+1] is computed in increasing k, so old v[k+1]
// is still intact when it is read.
__device__ __forceinline__ void horner_apply(const uint32_t (&u)[97], const uint32_t* bcoef, int bstride,
                                             uint32_t (&v)[97]) {
  uint32_t b = bcoef[96 * bstride];
#pragma unroll
  for (int k = 0; k < 97; ++k) v[k] = mul24(b, u[k]);
  uint32_t bnext = bcoef[95 * bstride];
  for (int i = 95; i >= 0; --i) {
    b = bnext;
    if (i > 0) bnext = bcoef[(i - 1) * bstride];
    const uint32_t fb = v[0] - v[kRS];
#pragma unroll
    for (int k = 0; k < 96; ++k) v[k] = mad24(b, u[k], v[k + 1]);
    v[96] = mad24(b, u[96], fb);
  }
}

// In-place f^J on one state record per lane (valid lanes only; every lane of
// the wave must call it, since the powering loop is wave-uniform).  The jump
// polynomial is parked in the record itself while the state words are held in
// registers, so no workspace is needed.
__device__ __forceinline__ void jump_record_lane(uint32_t* slot, bool valid, uint32_t j0, uint32_t j1, uint32_t j2,
                                                 uint32_t j3) {
  uint32_t a[97];
  xpow_lane(j0, j1, j2, j3, a);
  if (valid) {
    uint32_t u[97], v[97];
#pragma unroll
    for (int k = 0; k < 97; ++k) u[k] = slot[k];
    const uint32_t c = slot[97];
#pragma unroll
    for (int k = 0; k < 97; ++k) slot[k] = a[k];
    horner_apply(u, slot, 1, v);
#pragma unroll
    for (int k = 0; k < 97; ++k) slot[k] = v[k] & kMask;
    slot[97] = c_jump(c, u128_mod_m(j0, j1, j2, j3));
  }
}

}  // namespace ranmar
