// Half-wave cooperative seeding and jump-ahead: one request per 32 lanes,
// state in LDS.  Low latency for single requests, and no per-lane 200-register
// working set.
//
// Seeding (Appendix A, Algorithm 3) in parallel over the 97 words.  Word ii
// (0-based) is produced by steps 24 ii .. 24 ii + 23 of two small generators,
// and both can be jumped in closed form:
//   - the multiplicative step (i, j, k) <- (j, k, i j k mod 179): with
//     a = log_2 i etc. (2 is a primitive root mod 179) it is the linear map
//     (a, b, c) <- (b, c, a + b + c) mod 178, i.e. a 3x3 matrix M, so the
//     state before word ii is M^(24 ii) applied to the initial logs;
//   - l <- 53 l + 1 mod 169 is affine, l_(24 ii) = mu_ii l_0 + nu_ii mod 169.
// Lane l starts words l, l+32, l+64 (and lane 0 word 96) from those closed
// forms and runs the 24 ordinary steps of each.  The bits are exactly those of
// the sequential procedure.
//
// Jump (Sec. 3): with the exponent J written in 8-bit digits d_w,
// t^J = prod_w t^(d_w 2^(8w)) (mod phi), and applying these factors to the
// state one after the other gives f^J exactly (the jumps compose).  The table
// T[w][d] = t^(d 2^(8w)) mod phi (16 x 256 polynomials, 1.6 MB, computed once
// per device by the square-and-multiply kernel) turns a 120-bit jump into 15
// applications instead of ~119 squarings.  Each application is the Hankel
// product  x'_o = sum_i b_i X_(i+o)  with X the window extended by 96 steps;
// lane l computes outputs 3l..3l+3 with a sliding register window, so each
// multiply-add costs half an LDS read.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "seed_dev.hpp"

namespace ranmar {

// ---------------------------------------------------------------------------
// Seeding tables (computed at compile time)
// ---------------------------------------------------------------------------
struct SeedTables {
  uint8_t exp2[178];    // 2^e mod 179
  uint8_t log2[179];    // log_2 x mod 178 (index 0 unused)
  uint8_t m[97][9];     // M^(24 ii) mod 178, row-major
  uint8_t mu[97], nu[97];  // l_(24 ii) = mu l_0 + nu mod 169
};

constexpr SeedTables make_seed_tables() {
  SeedTables t{};
  uint32_t v = 1;
  for (int e = 0; e < 178; ++e) {
    t.exp2[e] = (uint8_t)v;
    t.log2[v] = (uint8_t)e;
    v = v * 2 % 179;
  }
  // M24 = M^24 with M = [[0,1,0],[0,0,1],[1,1,1]] (mod 178)
  uint32_t M[9] = {0, 1, 0, 0, 0, 1, 1, 1, 1};
  uint32_t P[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int s = 0; s < 24; ++s) {
    uint32_t Q[9] = {};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        uint32_t acc = 0;
        for (int x = 0; x < 3; ++x) acc += M[r * 3 + x] * P[x * 3 + c];
        Q[r * 3 + c] = acc % 178;
      }
    for (int q = 0; q < 9; ++q) P[q] = Q[q];
  }
  uint32_t C[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  uint32_t mu = 1, nu = 0;
  for (int ii = 0; ii < 97; ++ii) {
    for (int q = 0; q < 9; ++q) t.m[ii][q] = (uint8_t)C[q];
    t.mu[ii] = (uint8_t)mu;
    t.nu[ii] = (uint8_t)nu;
    uint32_t Q[9] = {};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        uint32_t acc = 0;
        for (int x = 0; x < 3; ++x) acc += P[r * 3 + x] * C[x * 3 + c];
        Q[r * 3 + c] = acc % 178;
      }
    for (int q = 0; q < 9; ++q) C[q] = Q[q];
    for (int s = 0; s < 24; ++s) {
      mu = mu * 53 % 169;
      nu = (nu * 53 + 1) % 169;
    }
  }
  return t;
}

static __constant__ const SeedTables kSeedTab = make_seed_tables();

// One word of Algorithm 3 from the generators' state before it.
__device__ __forceinline__ uint32_t seed_word(uint32_t i, uint32_t j, uint32_t k, uint32_t l) {
  uint32_t acc = 0;
#pragma unroll
  for (int jj = 0; jj < 24; jj += 3) {
    const uint32_t m0 = mod179(mul24(mul24(i, j), k));
    l = mod169(mad24(l, 53u, 1u));
    acc = (acc << 1) | ((mul24(l, m0) >> 5) & 1u);
    const uint32_t m1 = mod179(mul24(mul24(j, k), m0));
    l = mod169(mad24(l, 53u, 1u));
    acc = (acc << 1) | ((mul24(l, m1) >> 5) & 1u);
    const uint32_t m2 = mod179(mul24(mul24(k, m0), m1));
    l = mod169(mad24(l, 53u, 1u));
    acc = (acc << 1) | ((mul24(l, m2) >> 5) & 1u);
    i = m0;
    j = m1;
    k = m2;
  }
  return acc;
}

__device__ __forceinline__ uint32_t seed_word_at(int ii, uint32_t a0, uint32_t b0, uint32_t c0, uint32_t l0) {
  const uint8_t* M = kSeedTab.m[ii];
  const uint32_t a = (M[0] * a0 + M[1] * b0 + M[2] * c0) % 178u;
  const uint32_t b = (M[3] * a0 + M[4] * b0 + M[5] * c0) % 178u;
  const uint32_t c = (M[6] * a0 + M[7] * b0 + M[8] * c0) % 178u;
  const uint32_t l = (kSeedTab.mu[ii] * l0 + kSeedTab.nu[ii]) % 169u;
  return seed_word(kSeedTab.exp2[a], kSeedTab.exp2[b], kSeedTab.exp2[c], l);
}

// The 32 lanes of a half-wave (lane index l) write the seeded state to
// X[0..96] and c to X[97].  Returns false (and writes nothing) for a seed out
// of [1, 9e8]; the result is uniform over the half.
// Algorithm 3's starting values (i, j, k as discrete logs base 2 mod 179,
// and l) for a seed in [1, 9e8].
__device__ __forceinline__ void seed_start(int32_t seed, uint32_t& a0, uint32_t& b0, uint32_t& c0, uint32_t& l0) {
  const uint32_t s1 = (uint32_t)seed - 1u;
  const uint32_t ij = s1 / 30082u;
  const uint32_t kl = s1 - 30082u * ij;
  a0 = kSeedTab.log2[(ij / 177u) % 177u + 2u];
  b0 = kSeedTab.log2[ij % 177u + 2u];
  c0 = kSeedTab.log2[(kl / 169u) % 178u + 1u];
  l0 = kl % 169u;
}

__device__ __forceinline__ bool seed_half(int32_t seed, uint32_t* X, uint32_t l) {
  if (seed < 1 || seed > 900000000) return false;
  uint32_t a0, b0, c0, l0;
  seed_start(seed, a0, b0, c0, l0);
  // u_(ii+1) goes to x[96 - ii].
  X[96 - l] = seed_word_at(l, a0, b0, c0, l0);
  X[64 - l] = seed_word_at(l + 32, a0, b0, c0, l0);
  X[32 - l] = seed_word_at(l + 64, a0, b0, c0, l0);
  if (l == 0) {
    X[0] = seed_word_at(96, a0, b0, c0, l0);
    X[97] = kC0;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Windowed jump
// ---------------------------------------------------------------------------
constexpr int kWinBits = 8;
constexpr int kWinDigits = 1 << kWinBits;   // 256
constexpr int kWindows = 128 / kWinBits;    // 16

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// X[0..96] <- X P(A) for the polynomial in B[0..96]; X must have room for
// 193 words (the window is extended in place).  Half-wave cooperative.
__device__ __forceinline__ void apply_half(uint32_t* X, const uint32_t* B, uint32_t l) {
  // X_(97+i) = X_i - X_(i+64), 32 terms per step.
#pragma unroll
  for (uint32_t s0 = 0; s0 < 96; s0 += 32) {
    X[97 + s0 + l] = X[s0 + l] - X[s0 + l + 64];
    wave_sync();
  }
  // Outputs o = 3l .. 3l+3 (o = 96 only kept by lane 31).
  const uint32_t* Xl = X + 3u * l;
  uint32_t w0 = Xl[0], w1 = Xl[1], w2 = Xl[2];
  uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 4
  for (int i = 0; i < 97; ++i) {
    const uint32_t w3 = Xl[i + 3];
    const uint32_t b = B[i];
    a0 = mad24(b, w0, a0);
    a1 = mad24(b, w1, a1);
    a2 = mad24(b, w2, a2);
    a3 = mad24(b, w3, a3);
    w0 = w1;
    w1 = w2;
    w2 = w3;
  }
  wave_sync();
  X[3 * l] = a0 & kMask;
  X[3 * l + 1] = a1 & kMask;
  X[3 * l + 2] = a2 & kMask;
  if (l == 31) X[96] = a3 & kMask;
  wave_sync();
}

// In place: X[0..96] <- f_1^J applied to X (the c part is left to the caller).
// T: the window table, T + (w * 256 + d) * 97.  J given as 32-bit limbs.
// `nwin`: number of low windows to consider (uniform over the wave); windows
// whose digit is zero in every lane of the wave are skipped.  The next
// window's row is loaded while the current one is applied.
// Digit w of J in base 2^WB (WB = 8, 16, 20 or 24, J as four 32-bit limbs).
// A 20- or 24-bit digit may straddle two limbs; the last one (bits 120..127)
// has 8 bits.
template <int WB = kWinBits>
__device__ __forceinline__ uint32_t window_digit(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3, int w) {
  const int bit = w * WB;
  const uint32_t lo = bit < 32 ? j0 : bit < 64 ? j1 : bit < 96 ? j2 : j3;
  if constexpr (32 % WB == 0) {
    return (lo >> (bit & 31)) & ((1u << WB) - 1u);
  } else {
    const uint32_t hi = bit < 32 ? j1 : bit < 64 ? j2 : bit < 96 ? j3 : 0u;
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (bit & 31)) & ((1u << WB) - 1u);
  }
}

// Row of the factor t^(d 2^(WB w)) in a table of 2^WB rows per window (the
// last window of a 20- or 24-bit table has only 2^8).
template <int WB = kWinBits>
__device__ __forceinline__ const uint32_t* window_row(const uint32_t* __restrict__ T, uint32_t j0, uint32_t j1,
                                                      uint32_t j2, uint32_t j3, int w) {
  return T + (((uint64_t)w << WB) + window_digit<WB>(j0, j1, j2, j3, w)) * 97u;
}

// First window >= w whose digit is nonzero in some lane of the wave (nwin if
// none).  A zero digit's factor is T[w][0] = 1, so skipping it is exact.
template <int WB = kWinBits>
__device__ __forceinline__ int next_window(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3, int w, int nwin) {
  while (w < nwin && !__any(window_digit<WB>(j0, j1, j2, j3, w) != 0u)) ++w;
  return w;
}

template <int WB = kWinBits>
__device__ __forceinline__ void jump_half(uint32_t* X, uint32_t* B, const uint32_t* __restrict__ T, uint32_t j0,
                                          uint32_t j1, uint32_t j2, uint32_t j3, int nwin, uint32_t l) {
  int w = next_window<WB>(j0, j1, j2, j3, 0, nwin);
  if (w >= nwin) return;
  const uint32_t* row = window_row<WB>(T, j0, j1, j2, j3, w);
  uint32_t r0 = row[l], r1 = row[l + 32], r2 = row[l + 64], r3 = row[96];
  while (w < nwin) {
    B[l] = r0;
    B[l + 32] = r1;
    B[l + 64] = r2;
    if (l == 0) B[96] = r3;
    wave_sync();
    const int wn = next_window<WB>(j0, j1, j2, j3, w + 1, nwin);
    if (wn < nwin) {
      row = window_row<WB>(T, j0, j1, j2, j3, wn);
      r0 = row[l];
      r1 = row[l + 32];
      r2 = row[l + 64];
      r3 = row[96];
    }
    apply_half(X, B, l);
    w = wn;
  }
}

// ---------------------------------------------------------------------------
// Group form: one request per G lanes (G = 8, 16 or 32, a divisor of 96).
// Lane l computes outputs K l .. K l + K of the Hankel product, K = 96 / G (the
// extra one, o = 96, kept by lane G-1 only), so 97 of G (K + 1) accumulator
// slots are useful: 97/104 for G = 8, 97/112 for G = 16, 97/128 for G = 32.
// Each step of the sliding window is K + 1 multiply-adds per 2 LDS reads.
// ---------------------------------------------------------------------------

// Seeding by G lanes: lane l computes words l, l+G, ..., and lane 0 word 96.
template <int G>
__device__ __forceinline__ bool seed_group(int32_t seed, uint32_t* X, uint32_t l) {
  if (seed < 1 || seed > 900000000) return false;
  const uint32_t s1 = (uint32_t)seed - 1u;
  const uint32_t ij = s1 / 30082u;
  const uint32_t kl = s1 - 30082u * ij;
  const uint32_t a0 = kSeedTab.log2[(ij / 177u) % 177u + 2u];
  const uint32_t b0 = kSeedTab.log2[ij % 177u + 2u];
  const uint32_t c0 = kSeedTab.log2[(kl / 169u) % 178u + 1u];
  const uint32_t l0 = kl % 169u;
#pragma unroll
  for (uint32_t k = 0; k < 96; k += G) X[96 - (l + k)] = seed_word_at(l + k, a0, b0, c0, l0);
  if (l == 0) {
    X[0] = seed_word_at(96, a0, b0, c0, l0);
    X[97] = kC0;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Seeding by table steps (the same bits as seed_group, fewer instructions)
// ---------------------------------------------------------------------------
// Step n of the initialisation needs only m_n mod 64 and l_n mod 64: the bit
// is bit 5 of l_n m_n mod 64.  In the exponent form m_n = 2^(e_n) mod 179 with
// e_n = e_(n-3) + e_(n-2) + e_(n-1) mod 178, so a step is one table lookup
// indexed by that sum x < 534: entry x holds m mod 64 in bits 0..5 and
// x mod 178 from bit 8 on (bit 10 in the 32-bit table).  Adding three entries
// adds both fields without carries between them (3 * 63 < 256), so the sum
// shifted right by 8 is the next entry's byte offset in the 32-bit table (in
// the 16-bit one: half of it), and the low field never matters for the bit
// (its multiples of 256 vanish mod 64).  The congruential generator has full
// period 169, so l_n = C[(pos(l_0) + n) mod 169] with its cycle C from 0; a
// word's 24 steps read 24 consecutive entries of the cycle (repeated past 169
// so that no step wraps).
struct SeedStepTables {
  uint32_t emt[534];   // (x mod 178) << 10 | (2^(x mod 178) mod 179) mod 64
  uint8_t l64[192];    // C[i mod 169] mod 64
  uint8_t pos[169];    // pos(l): C[pos(l)] = l
};

constexpr SeedStepTables make_seed_step_tables() {
  SeedStepTables t{};
  uint32_t p2[178] = {};
  uint32_t v = 1;
  for (int e = 0; e < 178; ++e) {
    p2[e] = v;
    v = v * 2 % 179;
  }
  for (int x = 0; x < 534; ++x) t.emt[x] = (uint32_t)(x % 178) << 10 | (p2[x % 178] % 64);
  uint32_t cyc[169] = {};
  uint32_t c = 0;
  for (int p = 0; p < 169; ++p) {
    cyc[p] = c;
    t.pos[c] = (uint8_t)p;
    c = (53 * c + 1) % 169;
  }
  for (int i = 0; i < 192; ++i) t.l64[i] = (uint8_t)(cyc[i % 169] % 64);
  return t;
}

static __constant__ const SeedStepTables kSeedStep = make_seed_step_tables();

// The step tables in LDS, filled by the nthreads threads of a workgroup
// (followed by a workgroup barrier in the caller).  WIDE: 32-bit entries (one
// shift per step); otherwise 16-bit entries holding x mod 178 from bit 8 on
// (half the LDS, one more shift per step).
template <bool WIDE>
struct SeedLds {
  typedef typename std::conditional<WIDE, uint32_t, uint16_t>::type entry;
  entry emt[534];
  uint8_t l64[192];
  static constexpr int kShift = WIDE ? 10 : 8;  // bit of the x field in an entry
};

template <bool WIDE>
__device__ __forceinline__ void seed_lds_fill(SeedLds<WIDE>& s, uint32_t t, uint32_t nthreads) {
  for (uint32_t i = t; i < 534; i += nthreads)
    s.emt[i] = (typename SeedLds<WIDE>::entry)(WIDE ? kSeedStep.emt[i] : (kSeedStep.emt[i] >> 10) << 8 | (kSeedStep.emt[i] & 63u));
  for (uint32_t i = t; i < 192; i += nthreads) s.l64[i] = kSeedStep.l64[i];
}

// Words k0 .. k0 + P - 1 of lane l's list (word k of the list is l + k G for
// k < 96 / G, and word 96 after them), stepped together so that their
// lookups overlap.
template <int G, int K0, int P, bool WIDE>
__device__ __forceinline__ void seed_words_tab(uint32_t* X, uint32_t l, const SeedLds<WIDE>& tab, uint32_t a0,
                                               uint32_t b0, uint32_t c0, uint32_t p0) {
  constexpr int W = 96 / G;
  const uint8_t* emt = (const uint8_t*)tab.emt;
  uint32_t ta[P], tb[P], tc[P], pw[P], acc[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int k = K0 + i;
    const uint32_t w = k < W ? l + (uint32_t)(k * G) : 96u;
    const uint8_t* M = kSeedTab.m[w];
    const uint32_t a = (M[0] * a0 + M[1] * b0 + M[2] * c0) % 178u;
    const uint32_t b = (M[3] * a0 + M[4] * b0 + M[5] * c0) % 178u;
    const uint32_t c = (M[6] * a0 + M[7] * b0 + M[8] * c0) % 178u;
    ta[i] = tab.emt[a];
    tb[i] = tab.emt[b];
    tc[i] = tab.emt[c];
    pw[i] = (p0 + 24u * w + 1u) % 169u;  // cycle position of the word's first step
    acc[i] = 0;
  }
#pragma unroll
  for (int bit = 0; bit < 24; ++bit)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const uint32_t sum = ta[i] + tb[i] + tc[i];
      const uint32_t tn = WIDE ? *(const uint32_t*)(emt + (sum >> 8))
                               : (uint32_t) * (const uint16_t*)(emt + ((sum >> 8) << 1));
      const uint32_t lv = tab.l64[pw[i] + bit];
      acc[i] = (acc[i] << 1) | __builtin_amdgcn_ubfe(mul24(lv, tn), 5u, 1u);
      ta[i] = tb[i];
      tb[i] = tc[i];
      tc[i] = tn;
    }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int k = K0 + i;
    if (k < W)
      X[96 - (l + (uint32_t)(k * G))] = acc[i];
    else if (l == 0)
      X[0] = acc[i];  // word 96 (the other lanes made a spare copy)
  }
}

// Words k0 .. N - 1 of the lane's list in passes of at most PMAX.
template <int G, int K0, int N, int PMAX, bool WIDE>
__device__ __forceinline__ void seed_passes_tab(uint32_t* X, uint32_t l, const SeedLds<WIDE>& tab, uint32_t a0,
                                                uint32_t b0, uint32_t c0, uint32_t p0) {
  constexpr int P = N - K0 < PMAX ? N - K0 : PMAX;
  seed_words_tab<G, K0, P, WIDE>(X, l, tab, a0, b0, c0, p0);
  if constexpr (K0 + P < N) seed_passes_tab<G, K0 + P, N, PMAX, WIDE>(X, l, tab, a0, b0, c0, p0);
}

// seed_group's result with the step tables: lane l of the G-lane group makes
// words l, l + G, ... and word 96, at most PMAX of them at a time (more
// overlap the lookups better, fewer need fewer registers).
template <int G, int PMAX, bool WIDE>
__device__ __forceinline__ bool seed_group_tab(int32_t seed, uint32_t* X, uint32_t l, const SeedLds<WIDE>& tab) {
  if (seed < 1 || seed > 900000000) return false;
  constexpr int N = 96 / G + 1;  // words per lane, word 96 included
  constexpr int PM = N <= PMAX ? N : (N + (N + PMAX - 1) / PMAX - 1) / ((N + PMAX - 1) / PMAX);  // even passes
  const uint32_t s1 = (uint32_t)seed - 1u;
  const uint32_t ij = s1 / 30082u;
  const uint32_t kl = s1 - 30082u * ij;
  const uint32_t a0 = kSeedTab.log2[(ij / 177u) % 177u + 2u];
  const uint32_t b0 = kSeedTab.log2[ij % 177u + 2u];
  const uint32_t c0 = kSeedTab.log2[(kl / 169u) % 178u + 1u];
  const uint32_t p0 = kSeedStep.pos[kl % 169u];
  seed_passes_tab<G, 0, N, PM, WIDE>(X, l, tab, a0, b0, c0, p0);
  if (l == 0) X[97] = kC0;
  return true;
}

// X[0..96] <- X P(A) for the polynomial in B[0..96]; X has room for 193 words.
template <int G>
__device__ __forceinline__ void apply_group(uint32_t* X, const uint32_t* B, uint32_t l) {
  constexpr int K = 96 / G;
  // X_(97+i) = X_i - X_(i+64): terms within a block of 33 are independent
  // (each reads words at least 33 back), so only the blocks are ordered.
#pragma unroll
  for (uint32_t b0 = 0; b0 < 96; b0 += 33) {
    const uint32_t b1 = b0 + 33 < 96 ? b0 + 33 : 96;
#pragma unroll
    for (uint32_t i = b0 + l; i < b1; i += G) X[97 + i] = X[i] - X[i + 64];
    wave_sync();
  }
  const uint32_t* Xl = X + (uint32_t)K * l;
  uint32_t w[K], a[K];
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = Xl[k];
#pragma unroll
  for (int k = 0; k < K; ++k) a[k] = 0;
#pragma unroll K
  for (int i = 0; i < 97; ++i) {
    const uint32_t wn = Xl[i + K];
    const uint32_t b = B[i];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = mad24(b, w[k], a[k]);
#pragma unroll
    for (int k = 0; k + 1 < K; ++k) w[k] = w[k + 1];
    w[K - 1] = wn;
  }
  // Output 96 (the 97th of G K = 96 tiled ones) as a dot product split over
  // the group: lane l takes terms K l .. K l + K - 1, the last lane term 96
  // too; a butterfly over the G lanes sums them.
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) d = mad24(B[K * l + k], X[96 + K * l + k], d);
  d = mad24(l == G - 1 ? B[96] : 0u, X[192], d);
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) d += (uint32_t)__shfl_xor((int)d, off);
  wave_sync();
  uint32_t* Xo = X + (uint32_t)K * l;
#pragma unroll
  for (int k = 0; k < K; ++k) Xo[k] = a[k] & kMask;
  if (l == G - 1) X[96] = d & kMask;
  wave_sync();
}

struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

// jump_half for G lanes, with a table of WB-bit windows.  `issued` runs once,
// by the whole wave, after the first factor's loads have been issued (or at
// once if there is none): a memory operation it starts there is waited for
// only by loads issued after it, that is from the second factor on.
template <int G, int WB, class Hook = NoHook>
__device__ __forceinline__ void jump_group(uint32_t* X, uint32_t* B, const uint32_t* __restrict__ T, uint32_t j0,
                                           uint32_t j1, uint32_t j2, uint32_t j3, int nwin, uint32_t l,
                                           Hook issued = Hook{}) {
  constexpr int K = 96 / G;
  int w = next_window<WB>(j0, j1, j2, j3, 0, nwin);
  if (w >= nwin) {
    issued();
    return;
  }
  const uint32_t* row = window_row<WB>(T, j0, j1, j2, j3, w);
  uint32_t r[K + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] = row[l + G * k];
  r[K] = row[96];
  issued();
  while (w < nwin) {
#pragma unroll
    for (int k = 0; k < K; ++k) B[l + G * k] = r[k];
    if (l == 0) B[96] = r[K];
    wave_sync();
    const int wn = next_window<WB>(j0, j1, j2, j3, w + 1, nwin);
    if (wn < nwin) {
      row = window_row<WB>(T, j0, j1, j2, j3, wn);
#pragma unroll
      for (int k = 0; k < K; ++k) r[k] = row[l + G * k];
      r[K] = row[96];
    }
    apply_group<G>(X, B, l);
    w = wn;
  }
}

// Number of WB-bit windows holding the wave's longest exponent.
template <int WB = kWinBits>
__device__ __forceinline__ int wave_windows(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3) {
  int bl = 0;
  if (j3)
    bl = 128 - __clz(j3);
  else if (j2)
    bl = 96 - __clz(j2);
  else if (j1)
    bl = 64 - __clz(j1);
  else if (j0)
    bl = 32 - __clz(j0);
  return (wave_max_i32(bl) + WB - 1) / WB;
}

}  // namespace ranmar
