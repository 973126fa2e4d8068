// General lagged-Fibonacci generators: the combined generator of Sec. 2 for
// any lags 1 <= s < r, precision e <= 32 and arithmetic sequence (m, d), which
// Sec. 5 anticipates for larger r.  RANMAR is (97, 33, 24, 2^24 - 3, 7654321);
// the specialised kernels elsewhere in this library serve that case faster.
//
// Jump (Sec. 3.1, 3.2): P_J = t^J mod phi, phi = t^r + t^{r-s} - 1, over
// Z/2^e by left-to-right binary powering in LDS, one workgroup per J; the new
// words are the Hankel product sum_i b_i x_{i+l} over the state extended by
// r - 1 steps, and c moves by the closed form (c - J d) mod m.
//
// Generate (Algorithm 2 with general lags): the last r words of each stream
// live in an LDS ring of Z >= r + W words (Z a power of two); W lanes of a
// wave (W = min(s, 64) rounded down to a power of two) produce W consecutive
// words per step, since x_n .. x_{n+W-1} depend only on words older than x_n
// when W <= s; U steps (U W <= s, U <= 4) read all their operands before any
// is written.  Up to 64 / W streams share a wave (fewer when their rings would
// not fit), and each stream's W draws of a step form one contiguous store.
//
// Families (Sec. 1, block splitting): ~sqrt(n) direct jumps and ~sqrt(n)
// shared polynomials, every other start one polynomial applied to a direct
// start.
//
// Arithmetic is kept mod 2^32 and masked to e bits on output: for e <= 24 the
// products use v_mad_u32_u24 (exact in the low 24 bits), for e > 24 the full
// 32-bit multiply.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.hpp"
#include "internal.hpp"

namespace ranmar {
namespace {

struct LfgDev {
  uint32_t r, s, mask, m, d;
};

__device__ __forceinline__ void lane_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool W32>
__device__ __forceinline__ uint32_t mac(uint32_t a, uint32_t b, uint32_t acc) {
  if constexpr (W32)
    return a * b + acc;
  else
    return mad24(a, b, acc);
}

// J mod m for J = hi 2^64 + lo; m < 2^32 so every product fits 64 bits.
__device__ __forceinline__ uint32_t j_mod_m(ranmar_u128 J, uint32_t m) {
  const uint64_t M = m;
  const uint64_t t32 = (1ull << 32) % M;
  const uint64_t t64 = (t32 * t32) % M;
  return (uint32_t)(((J.hi % M) * t64 + J.lo % M) % M);
}

// Reduces Q[0 .. 2r-2] modulo phi in place (coefficients k >= r become zero
// in effect; only Q[0 .. r-1] is read afterwards).  t^k = t^{k-r} - t^{k-s}
// for k >= r.  The top coefficients are folded in blocks of at most s, from
// the top: inside a block the targets k - r and k - s all lie below the
// block, so one pass per target kind has no conflicts; the k - s targets of
// one block may be folded again by a lower block.
__device__ __forceinline__ void fold_phi(uint32_t* Q, int r, int s, int top, int tid, int bs) {
  for (int hi = top; hi >= r;) {
    const int lo = hi - s + 1 > r ? hi - s + 1 : r;
    for (int k = lo + tid; k <= hi; k += bs) Q[k - r] += Q[k];
    __syncthreads();
    for (int k = lo + tid; k <= hi; k += bs) Q[k - s] -= Q[k];
    __syncthreads();
    hi = lo - 1;
  }
}

// Squares and applications work on tiles of kTile consecutive outputs, the
// square as Q[k] = 2 sum_{i < k - i} P_i P_{k-i} + [k even] P_{k/2}^2.  P is
// read through a zero-padded view (P[i] = 0 for i < 0 and i >= r), so the
// ranges need no bounds tests: blocks of kTile terms i, each with the
// 2 kTile - 1 words P[k0 - i ..] they meet held in registers (six 16-byte LDS
// reads per kTile^2 multiply-adds instead of two 4-byte reads per multiply-add).
constexpr int kTile = 8;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The kTile coefficients P[ib ..] and the 2 kTile - 1 words P[k0 - ib - kTile + 1 ..]
// of one block, as 16-byte LDS reads: every start is a multiple of kTile words
// from a 32-byte aligned base, and lanes kTile words apart hit distinct banks.
__device__ __forceinline__ void load_block(const uint32_t* Pp, int ib, int k0, uint32_t (&a)[kTile],
                                           uint32_t (&x)[2 * kTile - 1]) {
  const u32x4* pa = (const u32x4*)(Pp + ib);
  const u32x4* px = (const u32x4*)(Pp + k0 - ib - kTile);
  uint32_t xx[2 * kTile];
#pragma unroll
  for (int v = 0; v < kTile / 4; ++v) {
    const u32x4 t = pa[v];
    a[4 * v] = t.x, a[4 * v + 1] = t.y, a[4 * v + 2] = t.z, a[4 * v + 3] = t.w;
  }
#pragma unroll
  for (int v = 0; v < kTile / 2; ++v) {
    const u32x4 t = px[v];
    xx[4 * v] = t.x, xx[4 * v + 1] = t.y, xx[4 * v + 2] = t.z, xx[4 * v + 3] = t.w;
  }
#pragma unroll
  for (int q = 0; q < 2 * kTile - 1; ++q) x[q] = xx[q + 1];
}

// Sum over the 8 lanes of an aligned lane group, left in every lane of it:
// DPP swaps of neighbours (quad_perm 1,0,3,2), of pairs (quad_perm 2,3,0,1)
// and of the two halves of the 8 (row_half_mirror).
__device__ __forceinline__ uint32_t group8_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
  return v;
}

// Sum over the 4 lanes of an aligned quad, left in every lane of it.
__device__ __forceinline__ uint32_t group4_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
  return v;
}

// One tile of the square, its term blocks split over the 4 lanes of a quad:
// lane l takes the blocks ib0 + kTile (l + 4 m) among those whose every term
// has 2 i < k0, i.e. belongs to all kTile outputs of the tile, so the blocks
// need no predicate.  After the quad sum, lane l owns outputs k0 + l and
// k0 + l + 4; the terms ib_stop <= i < k - i left for each all lie in the one
// block starting at ib_stop (k0 is a multiple of kTile), which the lane adds
// with a predicate per term.
template <bool W32>
__device__ __forceinline__ void square_tile(const uint32_t* Pp, uint32_t* Q, int r, int k0, int l) {
  uint32_t acc[kTile];
#pragma unroll
  for (int u = 0; u < kTile; ++u) acc[u] = 0;
  const int ilo = k0 - (r - 1) > 0 ? k0 - (r - 1) : 0;
  const int ib0 = ilo & ~(kTile - 1);
  const int span = ((k0 - 1) >> 1) - ib0 + 1;  // terms ib0 .. (k0 - 1) / 2
  const int ib_stop = ib0 + (span >= kTile ? span / kTile * kTile : 0);
  for (int ib = ib0 + kTile * l; ib < ib_stop; ib += 4 * kTile) {
    uint32_t a[kTile], x[2 * kTile - 1];
    load_block(Pp, ib, k0, a, x);
#pragma unroll
    for (int q = 0; q < kTile; ++q)
#pragma unroll
      for (int u = 0; u < kTile; ++u) acc[u] = mac<W32>(a[q], x[u - q + kTile - 1], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < kTile; ++u) acc[u] = group4_sum(acc[u]);
  const u32x4* pa = (const u32x4*)(Pp + ib_stop);
  const u32x4 w0 = pa[0], w1 = pa[1];
  const uint32_t a[kTile] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t mine = acc[4 * h];
#pragma unroll
    for (int u = 1; u < 4; ++u) mine = l == u ? acc[4 * h + u] : mine;
    const int k = k0 + l + 4 * h;
    const int lim = k - 2 * ib_stop;  // term ib_stop + q belongs to output k when 2 q < lim
#pragma unroll
    for (int q = 0; q < kTile; ++q) {
      const uint32_t t = mac<W32>(a[q], Pp[k - ib_stop - q], mine);
      mine = 2 * q < lim ? t : mine;
    }
    if (k < 2 * r - 1) {
      uint32_t v = mine << 1;
      if (!(k & 1)) v = mac<W32>(Pp[k >> 1], Pp[k >> 1], v);
      Q[k] = v;
    }
  }
}

// Threads of the jump workgroup: 4 lanes per tile of kTile outputs in the
// square, up to 64 quads.  Quad g squares the tiles c NG + g (c even) and
// (c + 1) NG - 1 - g (c odd) of the T = ceil((2r - 1) / kTile) tiles, NG the
// number of quads: the sweep alternates direction, which balances the
// triangular work profile across quads.
uint32_t jump_threads(uint32_t r) {
  const uint32_t tiles = (2 * r - 1 + kTile - 1) / kTile;
  const uint32_t lanes = 4 * tiles;
  return lanes >= 256 ? 256u : (lanes + 63) / 64 * 64;
}

// LDS layout of the jump (words; every buffer starts on a multiple of kTile
// words, so the 16-byte tile reads are aligned): P padded with kTile words
// below and 3 kTile above r rounded up to kTile, then Q[2 r8 + 2 kTile] (the
// application's 16-word windows reach index 2r + 13; words past 2r - 2 only
// meet zero coefficients or outputs past r - 1).
uint32_t jump_q_offset(uint32_t r) { return (r + kTile - 1) / kTile * kTile + 4 * kTile; }
size_t jump_lds_words(uint32_t r) {
  return jump_q_offset(r) + 2 * (size_t)((r + kTile - 1) / kTile * kTile) + 2 * kTile;
}

// The state src jumped by J, written to dst (may alias src): the words by
// the polynomial P_J in LDS (padded view), the Hankel product
// x'_l = sum_i b_i X_{i+l} over the window extended by r - 1 steps (in Q), c by
// (c - (J mod m) d) mod m with jm = J mod m.  Called by the whole workgroup.
template <bool W32>
__device__ __forceinline__ void apply_state(const LfgDev& g, const uint32_t* P, uint32_t* Q, const uint32_t* src,
                                            uint32_t* dst, uint32_t jm) {
  const int r = (int)g.r, s = (int)g.s;
  const int tid = threadIdx.x, bs = blockDim.x, groups = bs / 8, grp = tid >> 3, gl = tid & 7;
  const uint32_t c0 = src[r];
  for (int i = tid; i < r; i += bs) Q[i] = src[i];
  __syncthreads();
  for (int lo = r; lo < 2 * r - 1; lo += s) {
    const int hi = lo + s - 1 < 2 * r - 2 ? lo + s - 1 : 2 * r - 2;
    for (int k = lo + tid; k <= hi; k += bs) Q[k] = Q[k - r] - Q[k - s];
    __syncthreads();
  }
  // Tiles of kTile outputs per lane group, lane gl taking the blocks
  // kTile (gl + 8 m) of i, then the group sum.
  const int otiles = (r + kTile - 1) / kTile;
  for (int c = 0; c * groups < otiles; ++c) {
    const int t = c * groups + grp;
    if (t >= otiles) continue;
    const int l0 = t * kTile;
    uint32_t acc[kTile];
#pragma unroll
    for (int u = 0; u < kTile; ++u) acc[u] = 0;
    for (int ib = kTile * gl; ib < r; ib += 8 * kTile) {
      const u32x4* pa = (const u32x4*)(P + ib);
      const u32x4* px = (const u32x4*)(Q + ib + l0);
      uint32_t a[kTile], xx[2 * kTile];
#pragma unroll
      for (int v = 0; v < kTile / 4; ++v) {
        const u32x4 w = pa[v];
        a[4 * v] = w.x, a[4 * v + 1] = w.y, a[4 * v + 2] = w.z, a[4 * v + 3] = w.w;
      }
#pragma unroll
      for (int v = 0; v < kTile / 2; ++v) {
        const u32x4 w = px[v];
        xx[4 * v] = w.x, xx[4 * v + 1] = w.y, xx[4 * v + 2] = w.z, xx[4 * v + 3] = w.w;
      }
#pragma unroll
      for (int q = 0; q < kTile; ++q)
#pragma unroll
        for (int u = 0; u < kTile; ++u) acc[u] = mac<W32>(a[q], xx[q + u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < kTile; ++u) acc[u] = group8_sum(acc[u]);
    uint32_t mine = acc[0];
#pragma unroll
    for (int u = 1; u < kTile; ++u) mine = gl == u ? acc[u] : mine;
    if (l0 + gl < r) dst[l0 + gl] = mine & g.mask;
  }
  if (tid == 0) {
    const uint64_t M = g.m;
    dst[r] = (uint32_t)(((uint64_t)c0 + M - ((uint64_t)jm * g.d) % M) % M);
  }
  __syncthreads();
}

// One workgroup per item.  Dynamic LDS: jump_lds_words(r).
// Items below n_state jump states s_in -> s_out (r + 1 words per record; may
// alias), the record of item q at s_in + q * in_stride (in_stride 0: one shared
// input).  Items from n_state on write P_J (r words each) to P_out and stop.
template <bool W32>
__global__ __launch_bounds__(256) void k_lfg_jump(LfgDev g, const ranmar_u128* __restrict__ Js, const uint32_t* s_in,
                                                  uint64_t in_stride, uint32_t* s_out, uint32_t* P_out, uint64_t n,
                                                  uint64_t n_state, uint32_t q_off) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const int r = (int)g.r, s = (int)g.s;
  const int tid = threadIdx.x, bs = blockDim.x;
  uint32_t* P = lds + kTile;  // P[-kTile .. r + 3 kTile - 1]; zero outside [0, r)
  uint32_t* Q = lds + q_off;
  const int tiles = (2 * r - 1 + kTile - 1) / kTile, groups = bs / 4, grp = tid >> 2, gl = tid & 3;
  for (uint64_t item = blockIdx.x; item < n; item += gridDim.x) {
    const ranmar_u128 J = Js[item];
    // Leading bits of J that form an exponent below r give a monomial start.
    int bit = J.hi ? 127 - __builtin_clzll(J.hi) : (J.lo ? 63 - __builtin_clzll(J.lo) : -1);
    uint32_t v = 0;
    while (bit >= 0) {
      const uint32_t b = bit >= 64 ? (uint32_t)(J.hi >> (bit - 64)) & 1u : (uint32_t)(J.lo >> bit) & 1u;
      if (2 * v + b >= (uint32_t)r) break;
      v = 2 * v + b;
      --bit;
    }
    for (int i = tid - kTile; i < r + 3 * kTile; i += bs) P[i] = (i == (int)v) ? 1u : 0u;
    __syncthreads();
    for (; bit >= 0; --bit) {
      for (int c = 0; c * groups < tiles; ++c) {
        const int t = (c & 1) ? (c + 1) * groups - 1 - grp : c * groups + grp;
        if (t < tiles) square_tile<W32>(P, Q, r, t * kTile, gl);
      }
      __syncthreads();
      fold_phi(Q, r, s, 2 * r - 2, tid, bs);
      const uint32_t b = bit >= 64 ? (uint32_t)(J.hi >> (bit - 64)) & 1u : (uint32_t)(J.lo >> bit) & 1u;
      // The new P: Q mod phi, times t if the bit is set (shift up one place;
      // t^r = 1 - t^{r-s}).
      const uint32_t topc = Q[r - 1];
      auto next = [&](int i) -> uint32_t {
        if (!b) return Q[i];
        uint32_t x = i ? Q[i - 1] : topc;
        if (i == r - s) x -= topc;
        return x;
      };
      for (int i = tid; i < r; i += bs) P[i] = next(i);
      __syncthreads();
    }
    if (item >= n_state) {
      for (int i = tid; i < r; i += bs) P_out[(item - n_state) * r + i] = P[i] & g.mask;
      __syncthreads();
      continue;
    }
    apply_state<W32>(g, P, Q, s_in + item * in_stride, s_out + item * (uint64_t)(r + 1), j_mod_m(J, g.m));
  }
}

// Generation.  Dynamic LDS: (waves per workgroup) x G rings of Z words, with
// G <= 64 / W streams per wave (fewer when the rings would not fit).
template <int FMT, int U>
__global__ __launch_bounds__(256) void k_lfg_gen(LfgDev g, uint32_t lw, uint32_t G, uint32_t Z, const uint32_t* s_in,
                                                 uint32_t* s_out, uint64_t n, uint64_t count, void* out,
                                                 uint64_t ld, float scale) {
  extern __shared__ uint32_t lds[];
  const uint32_t r = g.r, s = g.s, mask = g.mask, m = g.m;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t W = 1u << lw;
  const uint32_t grp = lane >> lw, j = lane & (W - 1u);
  const uint64_t stream = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * G + grp;
  const bool active = grp < G && stream < n;
  uint32_t* ring = lds + (wave * G + (grp < G ? grp : 0u)) * Z;  // idle lanes only read
  const uint32_t zm = Z - 1u;
  const uint32_t* src = s_in + (active ? stream : 0) * (uint64_t)(r + 1);
  const uint32_t c0 = active ? src[r] : 0u;
  // The state, 16 loads in flight per lane before their LDS writes.
  for (uint32_t base = 0; base < r; base += 16 * W) {
    uint32_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const uint32_t i = base + j + u * W;
      v[u] = (active && i < r) ? src[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const uint32_t i = base + j + u * W;
      if (active && i < r) ring[i] = v[u];
    }
  }
  lane_order();
  // c before draw q + j is c_q - (j + 1) d; c_q steps by W d per step.
  const uint32_t dj = (uint32_t)(((uint64_t)(j + 1) * g.d) % m);
  const uint32_t dW = (uint32_t)(((uint64_t)W * g.d) % m);
  uint32_t c = c0;
  uint32_t pos = r;  // sequence index of the next word, kept mod 2^32 (Z divides 2^32)
  const uint64_t row = (active ? stream : 0) * ld;
  uint64_t q = 0;
  if constexpr (U > 1) {
    // U steps at once (U W <= s): every operand of the U W new words is older
    // than the first of them, so all reads precede the writes.
    uint32_t du[U];  // (u W + j + 1) d mod m
#pragma unroll
    for (int u = 0; u < U; ++u) du[u] = (uint32_t)(((uint64_t)(u * W + j + 1) * g.d) % m);
    const uint32_t dUW = (uint32_t)(((uint64_t)U * W * g.d) % m);
    for (; q + (uint64_t)U * W <= count; q += (uint64_t)U * W) {
      uint32_t a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = ring[(pos + u * W + j - r) & zm];
        b[u] = ring[(pos + u * W + j - s) & zm];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t x = (a[u] - b[u]) & mask;
        const uint32_t cj = c >= du[u] ? c - du[u] : c - du[u] + m;
        const uint32_t k = (x - cj) & mask;
        if (active) {
          ring[(pos + u * W + j) & zm] = x;
          if constexpr (FMT == 0)
            __builtin_nontemporal_store(k, (uint32_t*)out + row + q + u * W + j);
          else
            __builtin_nontemporal_store((float)k * scale, (float*)out + row + q + u * W + j);
        }
      }
      c = c >= dUW ? c - dUW : c - dUW + m;
      pos += U * W;
      lane_order();
    }
  }
  for (; q < count; q += W) {
    const bool live = active && q + j < count;
    const uint32_t a = ring[(pos + j - r) & zm];
    const uint32_t b = ring[(pos + j - s) & zm];
    const uint32_t x = (a - b) & mask;
    const uint32_t cj = c >= dj ? c - dj : c - dj + m;
    const uint32_t k = (x - cj) & mask;
    if (live) {
      ring[(pos + j) & zm] = x;
      if constexpr (FMT == 0)
        __builtin_nontemporal_store(k, (uint32_t*)out + row + q + j);
      else
        __builtin_nontemporal_store((float)k * scale, (float*)out + row + q + j);
    }
    c = c >= dW ? c - dW : c - dW + m;
    pos += W;
    lane_order();
  }
  if (active && s_out) {
    uint32_t* dst = s_out + stream * (uint64_t)(r + 1);
    const uint32_t end = (uint32_t)count;  // sequence index of the oldest kept word, mod 2^32
    for (uint32_t base = 0; base < r; base += 16 * W) {
      uint32_t v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = ring[(end + base + j + u * W) & zm];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const uint32_t i = base + j + u * W;
        if (i < r) dst[i] = v[u];
      }
    }
    if (j == 0) {
      const uint64_t M = m;
      const uint64_t sub = ((count % M) * g.d) % M;
      dst[r] = (uint32_t)(((uint64_t)c0 + M - sub) % M);
    }
  }
}

LfgDev to_dev(const ranmar_lfg_params& p) {
  return LfgDev{p.r, p.s, p.e >= 32 ? 0xFFFFFFFFu : ((1u << p.e) - 1u), p.m, p.d};
}

}  // namespace

int lfg_params_ok(const ranmar_lfg_params* p) {
  if (!p) return 0;
  if (p->r < 2 || p->r > RANMAR_LFG_MAX_R || p->s < 1 || p->s >= p->r || p->e < 1 || p->e > 32) return 0;
  const uint32_t mask = p->e >= 32 ? 0xFFFFFFFFu : ((1u << p->e) - 1u);
  if (p->m < 1 || (p->e < 32 && p->m > mask) || p->d >= p->m) return 0;
  return 1;
}

uint32_t lfg_jump_threads(uint32_t r) { return jump_threads(r); }


static hipError_t lfg_jump_strided(const ranmar_lfg_params& p, const ranmar_u128* J, const uint32_t* s_in,
                                   uint64_t in_stride, uint32_t* s_out, uint32_t* P_out, uint64_t n, uint64_t n_state,
                                   hipStream_t st) {
  if (n == 0) return hipSuccess;
  const LfgDev g = to_dev(p);
  const uint32_t bs = lfg_jump_threads(p.r);
  const size_t lds = jump_lds_words(p.r) * sizeof(uint32_t);
  const uint32_t q_off = jump_q_offset(p.r);
  const uint64_t grid = n < (1u << 20) ? n : (1u << 20);
  if (p.e > 24)
    hipLaunchKernelGGL(k_lfg_jump<true>, dim3((uint32_t)grid), dim3(bs), lds, st, g, J, s_in, in_stride, s_out, P_out,
                       n, n_state, q_off);
  else
    hipLaunchKernelGGL(k_lfg_jump<false>, dim3((uint32_t)grid), dim3(bs), lds, st, g, J, s_in, in_stride, s_out, P_out,
                       n, n_state, q_off);
  return hipGetLastError();
}

hipError_t launch_lfg_jump(const ranmar_lfg_params& p, const ranmar_u128* J, const uint32_t* s_in, uint32_t* s_out,
                           uint32_t* P_out, uint64_t n, hipStream_t st) {
  return lfg_jump_strided(p, J, s_in, (uint64_t)p.r + 1, s_out, P_out, n, P_out ? 0 : n, st);
}

// Families (Sec. 1 block splitting for any generator): out[k] = f^{k delta}
// of one base state.  With A ~ sqrt(n) and B = ceil(n / A), the starts
// a < A are direct jumps by a delta, the B - 1 shared polynomials are
// P_{b A delta}, and every other start is out[a + b A] = P_{b A delta}
// applied to out[a]: one r^2 application instead of a jump of ~log2(J)
// squarings.
__global__ void k_lfg_multiples(ranmar_u128* J, uint64_t count, uint64_t first, uint64_t step_lo, uint64_t step_hi) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const unsigned __int128 v = (unsigned __int128)(first + i) * (((unsigned __int128)step_hi << 64) | step_lo);
  J[i] = ranmar_u128{(uint64_t)v, (uint64_t)(v >> 64)};
}

// Workgroup (x, y): polynomial b = y + 1 (LDS, padded view), starts
// a = x per_wg .. x per_wg + per_wg - 1 (a < A, a + b A < n).
template <bool W32>
__global__ __launch_bounds__(256) void k_lfg_family(LfgDev g, const uint32_t* polys, uint32_t* out, uint64_t n,
                                                    uint64_t A, uint32_t per_wg, uint32_t adm, uint32_t q_off) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  const int r = (int)g.r;
  const int tid = threadIdx.x, bs = blockDim.x;
  uint32_t* P = lds + kTile;
  uint32_t* Q = lds + q_off;
  const uint64_t b = (uint64_t)blockIdx.y + 1;
  const uint32_t* pb = polys + (b - 1) * (uint64_t)r;
  for (int i = tid - kTile; i < r + 3 * kTile; i += bs) P[i] = (i >= 0 && i < r) ? pb[i] : 0u;
  __syncthreads();
  const uint32_t jm = (uint32_t)(((b % g.m) * (uint64_t)adm) % g.m);  // b A delta mod m
  for (uint32_t t = 0; t < per_wg; ++t) {
    const uint64_t a = (uint64_t)blockIdx.x * per_wg + t;
    const uint64_t k = a + b * A;
    if (a >= A || k >= n) break;
    apply_state<W32>(g, P, Q, out + a * (uint64_t)(r + 1), out + k * (uint64_t)(r + 1), jm);
  }
}

hipError_t launch_lfg_family(const ranmar_lfg_params& p, const uint32_t* base, ranmar_u128 delta, uint64_t n,
                             uint32_t* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  if (n > 1 && D > ~(unsigned __int128)0 / (n - 1)) return hipErrorInvalidValue;
  if (n > (1ull << 32)) return hipErrorInvalidValue;
  uint64_t A = (uint64_t)std::ceil(std::sqrt((double)n));
  if (A < 1) A = 1;
  if (A > n) A = n;
  const uint64_t B = (n + A - 1) / A;
  if (B - 1 > 65535) return hipErrorInvalidValue;
  ranmar_u128* J = nullptr;
  uint32_t* polys = nullptr;
  hipError_t e = hipMallocAsync((void**)&J, sizeof(ranmar_u128) * (A + B), st);
  if (e != hipSuccess) return e;
  if (B > 1) e = hipMallocAsync((void**)&polys, sizeof(uint32_t) * p.r * (B - 1), st);
  if (e == hipSuccess) {
    // J[a] = a delta (a < A); J[A + b - 1] = b A delta (1 <= b < B).
    const unsigned __int128 AD = D * A;  // <= (n - 1) delta when B > 1
    hipLaunchKernelGGL(k_lfg_multiples, dim3((uint32_t)((A + 255) / 256)), dim3(256), 0, st, J, A, 0ull,
                       (uint64_t)D, (uint64_t)(D >> 64));
    if (B > 1)
      hipLaunchKernelGGL(k_lfg_multiples, dim3((uint32_t)((B - 1 + 255) / 256)), dim3(256), 0, st, J + A, B - 1, 1ull,
                         (uint64_t)AD, (uint64_t)(AD >> 64));
    e = hipGetLastError();
    // One launch: the direct starts from the one base record (stride 0) and
    // the polynomials, which are independent and run side by side.
    if (e == hipSuccess) e = lfg_jump_strided(p, J, base, 0, out, polys, A + (B - 1), A, st);
    if (e == hipSuccess && B > 1) {
      const LfgDev g = to_dev(p);
      int dev = 0, cus = 256;
      if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      // Enough workgroups to fill the device a few times over; each loads its
      // polynomial once for per_wg starts.
      const uint64_t target = 8ull * (uint64_t)(cus > 0 ? cus : 256);
      uint64_t per = (A * (B - 1) + target - 1) / target;
      if (per < 1) per = 1;
      if (per > A) per = A;
      const uint64_t gx = (A + per - 1) / per;
      const uint32_t adm = (uint32_t)(AD % p.m);
      const size_t lds = jump_lds_words(p.r) * sizeof(uint32_t);
      const uint32_t q_off = jump_q_offset(p.r);
      const uint32_t bs = jump_threads(p.r);
      if (p.e > 24)
        hipLaunchKernelGGL(k_lfg_family<true>, dim3((uint32_t)gx, (uint32_t)(B - 1)), dim3(bs), lds, st, g, polys, out,
                           n, A, (uint32_t)per, adm, q_off);
      else
        hipLaunchKernelGGL(k_lfg_family<false>, dim3((uint32_t)gx, (uint32_t)(B - 1)), dim3(bs), lds, st, g, polys,
                           out, n, A, (uint32_t)per, adm, q_off);
      e = hipGetLastError();
    }
  }
  const hipError_t f1 = polys ? hipFreeAsync(polys, st) : hipSuccess;
  const hipError_t f2 = hipFreeAsync(J, st);
  return e != hipSuccess ? e : (f1 != hipSuccess ? f1 : f2);
}

// Launch shape of the generator: log2 of the lanes per stream, streams per
// wave, ring words, waves per workgroup.  Every workgroup's rings fit in
// 64 KiB: Z <= 8192 for r <= RANMAR_LFG_MAX_R, and G is capped at 16384 / Z.
void lfg_gen_shape(uint32_t r, uint32_t s, uint32_t* lw, uint32_t* G, uint32_t* Z, uint32_t* waves) {
  uint32_t w = 0;
  while ((2u << w) <= s && (2u << w) <= 64u) ++w;
  uint32_t z = 64;
  while (z < r + (1u << w)) z <<= 1;
  uint32_t gr = 64u >> w;
  if (gr > 16384u / z) gr = 16384u / z;
  if (gr < 1) gr = 1;
  const uint32_t per_wave = gr * z * 4u;  // bytes of ring per wave, <= 64 KiB
  uint32_t wv = 65536u / per_wave;
  if (wv > 4) wv = 4;
  if (wv < 1) wv = 1;
  *lw = w;
  *G = gr;
  *Z = z;
  *waves = wv;
}

hipError_t launch_lfg_generate(const ranmar_lfg_params& p, const uint32_t* s_in, uint32_t* s_out, uint64_t n,
                               uint64_t count, int fmt, void* out, uint64_t ld, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const LfgDev g = to_dev(p);
  uint32_t lw, G, Z, waves;
  lfg_gen_shape(p.r, p.s, &lw, &G, &Z, &waves);
  const uint64_t per_wg = (uint64_t)waves * G;
  const uint64_t grid = (n + per_wg - 1) / per_wg;
  if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const size_t lds = (size_t)waves * G * Z * sizeof(uint32_t);
  const float scale = 1.0f / (float)(1u << (p.e < 24 ? p.e : 24));
  const uint32_t W = 1u << lw;
  const int U = 4 * W <= p.s ? 4 : 2 * W <= p.s ? 2 : 1;  // steps issued together
#define LFG_GEN_LAUNCH(F, UU)                                                                                  \
  hipLaunchKernelGGL((k_lfg_gen<F, UU>), dim3((uint32_t)grid), dim3(64 * waves), lds, st, g, lw, G, Z, s_in, s_out, \
                     n, count, out, ld, scale)
  if (fmt == RANMAR_F32) {
    if (U == 4) LFG_GEN_LAUNCH(1, 4);
    else if (U == 2) LFG_GEN_LAUNCH(1, 2);
    else LFG_GEN_LAUNCH(1, 1);
  } else {
    if (U == 4) LFG_GEN_LAUNCH(0, 4);
    else if (U == 2) LFG_GEN_LAUNCH(0, 2);
    else LFG_GEN_LAUNCH(0, 1);
  }
#undef LFG_GEN_LAUNCH
  return hipGetLastError();
}

}  // namespace ranmar
