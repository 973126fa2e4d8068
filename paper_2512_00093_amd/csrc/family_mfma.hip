// Stream families as a matrix product on the matrix cores (MFMA int8).
//
// Starts k * delta, k < n, from a base state.  Write n = A * B (A a multiple
// of 16, A ~ sqrt(n), B = ceil(n / A)) and start s = j A + i (i < A, j < B).
// Then
//     x_s = x_i  P_j(A_c)        with P_j = t^(j A delta) mod phi
// (Sec. 3.1: the jump is the matrix P(A_c) of the companion matrix A_c acting
// on the row vector x), and c_s is c_i jumped by j A delta (Sec. 3.2).  So the
// x-parts of all starts with the same j are one product
//     Y_j [A x 97] = W [A x 97] * Q_j [97 x 97],   Q_j = P_j(A_c) mod 2^24,
// a dense contraction: every factor is shared by A starts, unlike a jump of
// one state by its own polynomial.
//
// Row r of Q_j is the unit window e_r jumped by J = j A delta, i.e. terms
// J .. J+96 of the sequence g_r that starts from e_r.  The recurrence
// x_n = x_(n-97) - x_(n-33) gives g_r(n) = g_(r+1)(n+1) for r != 63 and
// g_63(n) = g_64(n+1) + g_96(n), so with h = terms J .. J+192 of g_96 (e_96
// jumped by J, then extended by 96 steps):
//     Q_j[r][l] = h[l + 96 - r] + (r <= 63 ? h[l + 63 - r] : 0)   (mod 2^24).
// One jump per factor instead of 97.
//
// Launch 1 (VALU, 32 lanes per job, the windowed jump of coop_dev.hpp):
//   jobs [0, A):          x_i = base jumped by i delta (with c), into out;
//   jobs [A, A + B - 1):  h of factor j = job - A + 1, 193 words.
// Launch 2 (MFMA): a workgroup per (j, 4 x tpw tiles of 16 sources) turns h
// into the limb sequences from which every B operand is read (Q_j is two
// Toeplitz bands, see below); each wave loads its tiles' 16 x 97 blocks of W
// into registers, splits them into limbs, and for each of seven 16-column
// tiles computes
//     Y = W0 Q0 + 2^8 (W0 Q1 + W1 Q0) + 2^16 (W0 Q2 + W1 Q1 + W2 Q0)  (mod 2^24)
// with v_mfma_i32_16x16x64_i8 (K = 97 padded to 128: two steps), 12 MFMAs
// per column tile.  Exactness: a 24-bit word is w0 + 2^8 w1 + 2^16 w2 (mod 2^24)
// with signed limbs in [-128, 127]; limb products with weight >= 2^24 vanish
// mod 2^24; each of the six accumulators (one per limb product) sums at most
// 97 products of magnitude <= 2^14, far inside int32, and the final
// combination wraps mod 2^32, then is masked.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "coop_dev.hpp"
#include "internal.hpp"

namespace ranmar {

namespace {

constexpr int kQN = 112;  // output columns, padded to 7 tiles of 16
constexpr int kHWords = 196;  // one factor's h (193 words), rows 16-byte aligned
constexpr int kL1Words = 193 + 97;  // LDS per half-wave: extended window + polynomial

typedef int v4i __attribute__((ext_vector_type(4)));

// v (< 2^24) as w0 + 2^8 w1 + 2^16 w2 (mod 2^24), signed 8-bit limbs.
__device__ __forceinline__ void limbs3(uint32_t v, int& w0, int& w1, int& w2) {
  int t = (int)v;
  w0 = (int)(int8_t)(t & 0xFF);
  t = (t - w0) >> 8;  // exact: t - w0 is a multiple of 256 and >= 0
  w1 = (int)(int8_t)(t & 0xFF);
  t = (t - w1) >> 8;
  w2 = (int)(int8_t)(t & 0xFF);  // the top carry (2^24) is dropped: mod 2^24
}

// Start jobs begin from the base record, or (seed > 0) from the seeded state
// of `seed` (Algorithm 3, by the half-wave); start t is then jumped by
// E0 + t delta.
__global__ __launch_bounds__(256) void k_family_l1(const uint32_t* base, uint32_t* out, uint32_t* __restrict__ H,
                                                   const uint32_t* __restrict__ T, uint64_t A, uint64_t njobs,
                                                   uint64_t d_lo, uint64_t d_hi, uint64_t ad_lo, uint64_t ad_hi,
                                                   uint32_t in_place, int32_t seed, uint64_t e0_lo, uint64_t e0_hi) {
  __shared__ uint32_t lds[8 * kL1Words];
  __shared__ uint32_t seeded[97];
  const uint32_t hw = threadIdx.x >> 5, l = threadIdx.x & 31u;
  const uint64_t t = (uint64_t)blockIdx.x * 8u + hw;
  const bool active = t < njobs;
  const bool is_start = t < A;
  // Workgroups of start jobs only (A is a multiple of 8) seed together: one
  // word per thread instead of three per lane.
  const bool wg_seeds = seed > 0 && ((uint64_t)blockIdx.x + 1) * 8u <= A;
  if (wg_seeds) {
    uint32_t a0, b0, c0, l0;
    seed_start(seed, a0, b0, c0, l0);
    if (threadIdx.x < 97) seeded[96 - threadIdx.x] = seed_word_at((int)threadIdx.x, a0, b0, c0, l0);
    __syncthreads();  // uniform over the workgroup
  }
  uint32_t* X = lds + hw * kL1Words;
  uint32_t* Bp = X + 193;
  unsigned __int128 E = 0;
  uint32_t c = 0;
  if (is_start) {
    if (wg_seeds) {
      X[l] = seeded[l];
      X[l + 32] = seeded[l + 32];
      X[l + 64] = seeded[l + 64];
      if (l == 0) X[96] = seeded[96];
      c = kC0;
    } else if (seed > 0) {
      seed_half(seed, X, l);  // the host checked the seed
      wave_sync();
      c = X[97];
    } else {
      X[l] = base[l];
      X[l + 32] = base[l + 32];
      X[l + 64] = base[l + 64];
      if (l == 0) X[96] = base[96];
      c = base[97];
    }
    // E0 + t delta <= E0 + (n - 1) delta < 2^128: checked on the host.
    E = (((unsigned __int128)e0_hi << 64) | e0_lo) + (unsigned __int128)t * (((unsigned __int128)d_hi << 64) | d_lo);
  } else {
    X[l] = X[l + 32] = X[l + 64] = 0;  // e_96
    if (l == 0) X[96] = 1u;
    if (active) E = (unsigned __int128)(t - A + 1) * (((unsigned __int128)ad_hi << 64) | ad_lo);
  }
  wave_sync();
  const uint32_t j0 = (uint32_t)E, j1 = (uint32_t)(E >> 32), j2 = (uint32_t)(E >> 64), j3 = (uint32_t)(E >> 96);
  jump_half(X, Bp, T, j0, j1, j2, j3, wave_windows(j0, j1, j2, j3), l);
  if (!active) return;  // a whole half-wave leaves together, after the last wave-wide step
  if (is_start) {
    if (in_place && t == 0) return;  // start 0 is the base record itself
    uint32_t* dst = out + t * kWords;
    dst[l] = X[l];
    dst[l + 32] = X[l + 32];
    dst[l + 64] = X[l + 64];
    if (l == 0) {
      dst[96] = X[96];
      dst[97] = c_jump(c, u128_mod_m(j0, j1, j2, j3));
    }
  } else {
    // h: the jumped window extended by 96 steps, X_(97+i) = X_i - X_(i+64).
#pragma unroll
    for (uint32_t s0 = 0; s0 < 96; s0 += 32) {
      X[97 + s0 + l] = X[s0 + l] - X[s0 + l + 64];
      wave_sync();
    }
    uint32_t* h = H + (t - A) * kHWords;
#pragma unroll
    for (uint32_t o = l; o < 193; o += 32) h[o] = X[o] & kMask;
  }
}

// Signed 8-bit digits of v < 2^24 in bytes 0..2: with e = v + 0x808080,
// digit k = byte k of e minus 128 lies in [-128, 127], and their weighted sum
// is v + 2^24 (byte 3 of e), i.e. v mod 2^24; byte k of e xor 0x80 is that
// digit in two's complement.
__device__ __forceinline__ uint32_t limb_bytes(uint32_t v) { return (v + 0x808080u) ^ 0x808080u; }

// Q_j in LDS without expanding it.  Q_j[r][o] depends only on d = o - r and
// on whether r <= 63 (two Toeplitz bands), and the MFMA B operand of column
// o, K-step kk and lane group kg is the 16 limbs of rows r = 64 kk + 16 kg
// .. +15: with m = 112 - o + r these are 16 consecutive entries of
//     L_kk,b[m] = limb b of (kk == 0 ? h[208 - m] + h[175 - m] : h[208 - m])
// (h index out of [0, 192]: 0), since K-step 0 holds exactly the rows
// r <= 63 and K-step 1 the rest.  The six sequences (kk, b) of 240 bytes are
// kept in 16 copies, copy c shifted left by c bytes, so that every operand
// is one aligned 16-byte read: entries m0 .. m0+15 sit at byte m0 - c of copy
// c = m0 mod 16.  Entries for o >= 97 or r >= 97 are never used: those output
// columns are not stored, and the A operand is zero for r >= 97.
constexpr int kSeqLen = 240;                   // m in [0, 240): m0 + 15 <= 112 + 64 + 48 + 15
constexpr int kCopyStride = 6 * kSeqLen + 16;  // 364 words = 4 x 91: copies start on distinct bank groups
constexpr int kBaseLen = 256;                  // unshifted sequences, zero-padded

typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));  // records are only 8-byte aligned

// One tile's sources in the A-operand layout: lane (mrow, kg) holds words
// kk*64 + kg*16 + e (e < 16) of record i0 + mrow, zero for words >= 97, and
// lanes 0..15 (kg = 0) the record's c.
struct SrcTile {
  uint32_t w[2][16];
  uint32_t c;
};

// Reads stay inside the output buffer: the last source record is A - 1 and
// the furthest word read is 127 of it, inside row A < n.  Words >= 97 are
// loaded but replaced by zero before use (they are c or the start of the
// next record, which another workgroup may be writing: the value is unused).
__device__ __forceinline__ void load_tile(const uint32_t* rec, uint32_t kg, SrcTile& s) {
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const u32x4a* p = (const u32x4a*)(rec + kk * 64 + kg * 16);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const u32x4a v = p[d];
      s.w[kk][4 * d] = v.x;
      s.w[kk][4 * d + 1] = v.y;
      s.w[kk][4 * d + 2] = v.z;
      s.w[kk][4 * d + 3] = v.w;
    }
  }
  s.c = rec[97];
}

// The product kernel.  Workgroup (x, jq): factor j = jq + 1, source tiles
// (4 x + wave) tpw + tt.  Every wave first loads its first tile, then the
// workgroup turns h_j into the shifted limb sequences in LDS; tiles are
// multiplied from registers and written straight from the accumulators (16
// consecutive words of 4 records per store; the L2 merges a tile's 6272
// bytes).  At most 168 VGPRs (three waves per SIMD).
__global__ __launch_bounds__(256, 3) void k_family_gemm(uint32_t* out, const uint32_t* __restrict__ H, uint64_t A,
                                                     uint64_t n, uint32_t ad_mod, uint32_t tpw) {
  __shared__ __attribute__((aligned(16))) uint8_t tq[16 * kCopyStride];
  __shared__ __attribute__((aligned(16))) uint8_t tb[6 * kBaseLen];
  __shared__ uint32_t hl[196];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t mrow = lane & 15u, kg = lane >> 4;
  const uint64_t jq = blockIdx.y, j = jq + 1;
  const uint64_t tiles = A / 16;
  const uint64_t tile0 = ((uint64_t)blockIdx.x * 4 + wave) * tpw;
  auto tile_ok = [&](uint64_t tile) {
    return tile < tiles && j * A + tile * 16 < n;  // blocks of the last factor may lie beyond n
  };
  SrcTile cur;
  if (tile_ok(tile0)) load_tile(out + (tile0 * 16 + mrow) * kWords, kg, cur);
  if (threadIdx.x < 193) hl[threadIdx.x] = H[jq * kHWords + threadIdx.x];
  __syncthreads();
  {  // the six limb sequences, entry m = threadIdx.x
    const int m = (int)threadIdx.x, i1 = 208 - m, i2 = 175 - m;
    const uint32_t va = (i1 >= 0 && i1 <= 192) ? hl[i1] : 0u;
    const uint32_t vb = (va + ((i2 >= 0 && i2 <= 192) ? hl[i2] : 0u)) & kMask;
    int a0, a1, a2, b0, b1, b2;
    limbs3(vb, b0, b1, b2);  // K-step 0: rows r <= 63
    limbs3(va, a0, a1, a2);  // K-step 1
    tb[0 * kBaseLen + m] = (uint8_t)b0;
    tb[1 * kBaseLen + m] = (uint8_t)b1;
    tb[2 * kBaseLen + m] = (uint8_t)b2;
    tb[3 * kBaseLen + m] = (uint8_t)a0;
    tb[4 * kBaseLen + m] = (uint8_t)a1;
    tb[5 * kBaseLen + m] = (uint8_t)a2;
  }
  __syncthreads();
  // Shifted copies: wave w fills rows it = w, w + 4, ... of the 96 (copy c,
  // sequence cb) rows, lane p < 60 the word at bytes 4 p .. 4 p + 3, which
  // are base bytes 4 p + c .. 4 p + c + 3 (<= cb * 256 + 254).
  {
    const uint32_t* tb32 = (const uint32_t*)tb;
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(wave);  // uniform: scalar loop control
#pragma unroll
    for (uint32_t k = 0; k < 24; ++k) {
      const uint32_t it = w0 + 4 * k, c = it / 6, cb = it % 6;
      if (lane < kSeqLen / 4) {
        const uint32_t wi = cb * (kBaseLen / 4) + (c >> 2) + lane;
        const uint32_t w = __builtin_amdgcn_alignbyte(tb32[wi + 1], tb32[wi], c & 3u);
        *(uint32_t*)(tq + c * kCopyStride + cb * kSeqLen + 4 * lane) = w;
      }
    }
  }
  __syncthreads();  // every wave reaches the three barriers
  const uint32_t jm = (uint32_t)(j * ad_mod % kMod);
  // B operands: column o = nt*16 + mrow, K-step kk, lane group kg reads
  // entries m0 = 112 - o + 64 kk + 16 kg of copy c = m0 mod 16 = (16 - mrow)
  // mod 16, at byte m0 - c = (mrow == 0 ? 16 : 0) + 16 kg + 16 (6 - nt) + 64 kk
  // of that copy's sequence (kk, b): one base per lane, constant offsets.
  const uint32_t cq = (16u - mrow) & 15u;
  const uint8_t* qb = tq + cq * kCopyStride + (mrow == 0 ? 16u : 0u) + kg * 16;
  for (uint32_t tt = 0; tt < tpw; ++tt) {
    const uint64_t tile = tile0 + tt;
    if (!tile_ok(tile)) break;  // and so are the later tiles
    const uint64_t s0 = j * A + tile * 16;
    // A operand from the registers: limbs of words k = kk*64 + kg*16 + e.
    v4i a[3][2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t x[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t k = kk * 64 + kg * 16 + 4 * d + e;
          x[e] = limb_bytes(k < 97 ? cur.w[kk][4 * d + e] : 0u);
        }
        // Byte transpose: plane b takes byte b of the four words, in order.
        const uint32_t lo01 = __builtin_amdgcn_perm(x[1], x[0], 0x05010400u);  // x0.0 x1.0 x0.1 x1.1
        const uint32_t lo23 = __builtin_amdgcn_perm(x[3], x[2], 0x05010400u);
        const uint32_t hi01 = __builtin_amdgcn_perm(x[1], x[0], 0x0C0C0602u);  // x0.2 x1.2 0 0
        const uint32_t hi23 = __builtin_amdgcn_perm(x[3], x[2], 0x0C0C0602u);
        a[0][kk][d] = (int)__builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
        a[1][kk][d] = (int)__builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
        a[2][kk][d] = (int)__builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
      }
    const uint32_t c_src = cur.c;
    if (tt + 1 < tpw && tile_ok(tile + 1)) load_tile(out + ((tile + 1) * 16 + mrow) * kWords, kg, cur);
    const uint32_t rows = (uint32_t)(n - s0 < 16 ? n - s0 : 16);  // s0 < n: checked above
    uint32_t* dst = out + s0 * kWords;
    uint32_t* lp = dst + kg * 4 * kWords + mrow;  // row kg*4, column mrow; the rest are constant offsets
#pragma unroll
    for (int nt = 0; nt < kQN / 16; ++nt) {
      v4i q[3][2];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          q[b][kk] = *(const v4i*)(qb + (6 - nt) * 16 + kk * (3 * kSeqLen + 64) + b * kSeqLen);
      // Six accumulators, one per limb product, so that no MFMA waits for
      // more than the one of the previous K-step.
      v4i acc0 = {0, 0, 0, 0}, acc1a = acc0, acc1b = acc0, acc2a = acc0, acc2b = acc0, acc2c = acc0;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        acc0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0][kk], q[0][kk], acc0, 0, 0, 0);
        acc1a = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0][kk], q[1][kk], acc1a, 0, 0, 0);
        acc2a = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0][kk], q[2][kk], acc2a, 0, 0, 0);
        acc1b = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1][kk], q[0][kk], acc1b, 0, 0, 0);
        acc2b = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1][kk], q[1][kk], acc2b, 0, 0, 0);
        acc2c = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[2][kk], q[0][kk], acc2c, 0, 0, 0);
      }
      const v4i acc1 = acc1a + acc1b, acc2 = acc2a + acc2b + acc2c;
      // D layout: lane holds rows kg*4 + i, column nt*16 + mrow (< 97 unless
      // nt = 6 and mrow > 0).
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t y = ((uint32_t)acc0[i] + ((uint32_t)acc1[i] << 8) + ((uint32_t)acc2[i] << 16)) & kMask;
        if ((nt < 6 || mrow == 0) && kg * 4 + i < rows) lp[i * kWords + nt * 16] = y;
      }
    }
    // c of the block's starts (Sec. 3.2): c_i jumped by j A delta.
    if (lane < rows) dst[lane * kWords + 97] = c_jump(c_src, jm);
  }
}

typedef int v16i __attribute__((ext_vector_type(16)));

// One 32-row tile's sources for v_mfma_i32_32x32x32_i8: lane (mrow = l mod 32,
// kg = l / 32) holds words 32 kk + 16 kg + e (kk < 3, e < 16) of record
// i0 + mrow, all below 96, and the record's word 96 and c.  Every read is
// inside the record.
struct SrcTile32 {
  uint32_t w[3][16];
  uint32_t w96, c;
};

__device__ __forceinline__ void load_tile32(const uint32_t* rec, uint32_t kg, SrcTile32& s) {
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const u32x4a* p = (const u32x4a*)(rec + kk * 32 + kg * 16);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const u32x4a v = p[d];
      s.w[kk][4 * d] = v.x;
      s.w[kk][4 * d + 1] = v.y;
      s.w[kk][4 * d + 2] = v.z;
      s.w[kk][4 * d + 3] = v.w;
    }
  }
  s.w96 = rec[96];
  s.c = rec[97];
}

// The product kernel with 32 x 32 x 32 int8 MFMAs (lane layouts checked on
// the device with a probe: A and B by row / column l mod 32 and
// k = 16 (l / 32) + 0..15; accumulator i of lane l is row
// 8 (i / 4) + 4 (l / 32) + i mod 4, column l mod 32).  The matrix cores take
// rows and columns 0..95 of Q_j (three K-steps of 32, the first two in the
// band r <= 63, the third in r >= 64; three column tiles of 32); the VALU
// adds row 96 (W[s][96] Q_j[96][o] with Q_j[96][o] = h[o]) and computes column
// 96 (a dot product of length 97 with Q_j[r][96] = h[192 - r] + [r <= 63]
// h[159 - r]).  Tiles of 32 starts; B operands from the same shifted limb
// sequences as k_family_gemm.
__global__ __launch_bounds__(256, 2) void k_family_gemm32(uint32_t* out, const uint32_t* __restrict__ H, uint64_t A,
                                                       uint64_t n, uint32_t ad_mod, uint32_t tpw) {
  __shared__ __attribute__((aligned(16))) uint8_t tq[16 * kCopyStride];
  __shared__ __attribute__((aligned(16))) uint8_t tb[6 * kBaseLen];
  __shared__ __attribute__((aligned(16))) uint32_t hl[196];
  __shared__ __attribute__((aligned(16))) uint32_t qcol[128];  // Q_j[r][96], r < 97 (rest 0)
  __shared__ __attribute__((aligned(16))) uint32_t w96s[4][32];  // per wave: word 96 of the tile's rows
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t mrow = lane & 31u, kg = lane >> 5;
  const uint64_t jq = blockIdx.y, j = jq + 1;
  const uint64_t tiles = A / 32;
  const uint64_t tile0 = ((uint64_t)blockIdx.x * 4 + wave) * tpw;
  auto tile_ok = [&](uint64_t tile) { return tile < tiles && j * A + tile * 32 < n; };
  SrcTile32 cur;
  if (tile_ok(tile0)) load_tile32(out + (tile0 * 32 + mrow) * kWords, kg, cur);
  if (threadIdx.x < 193) hl[threadIdx.x] = H[jq * kHWords + threadIdx.x];
  __syncthreads();
  {  // the six limb sequences (entry m = threadIdx.x) and Q_j's column 96
    const int m = (int)threadIdx.x, i1 = 208 - m, i2 = 175 - m;
    const uint32_t va = (i1 >= 0 && i1 <= 192) ? hl[i1] : 0u;
    const uint32_t vb = (va + ((i2 >= 0 && i2 <= 192) ? hl[i2] : 0u)) & kMask;
    int a0, a1, a2, b0, b1, b2;
    limbs3(vb, b0, b1, b2);  // rows r <= 63
    limbs3(va, a0, a1, a2);  // rows r >= 64
    tb[0 * kBaseLen + m] = (uint8_t)b0;
    tb[1 * kBaseLen + m] = (uint8_t)b1;
    tb[2 * kBaseLen + m] = (uint8_t)b2;
    tb[3 * kBaseLen + m] = (uint8_t)a0;
    tb[4 * kBaseLen + m] = (uint8_t)a1;
    tb[5 * kBaseLen + m] = (uint8_t)a2;
    if (m < 128) qcol[m] = m < 97 ? (hl[192 - m] + (m <= 63 ? hl[159 - m] : 0u)) & kMask : 0u;
  }
  __syncthreads();
  {
    const uint32_t* tb32 = (const uint32_t*)tb;
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
    for (uint32_t k = 0; k < 24; ++k) {
      const uint32_t it = w0 + 4 * k, c = it / 6, cb = it % 6;
      if (lane < kSeqLen / 4) {
        const uint32_t wi = cb * (kBaseLen / 4) + (c >> 2) + lane;
        const uint32_t w = __builtin_amdgcn_alignbyte(tb32[wi + 1], tb32[wi], c & 3u);
        *(uint32_t*)(tq + c * kCopyStride + cb * kSeqLen + 4 * lane) = w;
      }
    }
  }
  __syncthreads();  // every wave reaches the three barriers
  const uint32_t jm = (uint32_t)(j * ad_mod % kMod);
  // B operands: column o = 32 nt + mrow, K-step kk, lane group kg: entries
  // m0 = 112 - o + 32 kk + 16 kg of copy c = (16 - mrow mod 16) mod 16, at
  // byte m0 - c = qbase + 32 (2 - nt) + 32 kk of sequence (band, b).
  const uint32_t cq = (16u - (mrow & 15u)) & 15u;
  const uint32_t qbase = ((mrow & 15u) == 0 ? 112u : 96u) - 16u * ((mrow >> 4) & 1u) + 16u * kg - 64u;
  const uint8_t* qb = tq + cq * kCopyStride + qbase;
  uint32_t* w96w = w96s[wave];
  for (uint32_t tt = 0; tt < tpw; ++tt) {
    const uint64_t tile = tile0 + tt;
    if (!tile_ok(tile)) break;  // and so are the later tiles
    const uint64_t s0 = j * A + tile * 32;
    v4i a[3][3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t x[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = limb_bytes(cur.w[kk][4 * d + e]);
        const uint32_t lo01 = __builtin_amdgcn_perm(x[1], x[0], 0x05010400u);
        const uint32_t lo23 = __builtin_amdgcn_perm(x[3], x[2], 0x05010400u);
        const uint32_t hi01 = __builtin_amdgcn_perm(x[1], x[0], 0x0C0C0602u);
        const uint32_t hi23 = __builtin_amdgcn_perm(x[3], x[2], 0x0C0C0602u);
        a[0][kk][d] = (int)__builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
        a[1][kk][d] = (int)__builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
        a[2][kk][d] = (int)__builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
      }
    // Column 96 of this lane's row (two lanes per row: halves of the sum).
    uint32_t col96 = 0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int e = 0; e < 16; ++e) col96 = mad24(cur.w[kk][e], qcol[kk * 32 + kg * 16 + e], col96);
    if (kg == 0) col96 = mad24(cur.w96, qcol[96], col96);
    col96 += (uint32_t)__shfl_xor((int)col96, 32, 64);
    const uint32_t c_src = cur.c;
    if (kg == 0) w96w[mrow] = cur.w96;
    wave_sync();
    uint32_t w96r[16];  // word 96 of the accumulator rows 8 (i / 4) + 4 kg + i mod 4
#pragma unroll
    for (int i = 0; i < 16; ++i) w96r[i] = w96w[8 * (i / 4) + 4 * kg + (i % 4)];
    if (tt + 1 < tpw && tile_ok(tile + 1)) load_tile32(out + ((tile + 1) * 32 + mrow) * kWords, kg, cur);
    const uint32_t rows = (uint32_t)(n - s0 < 32 ? n - s0 : 32);  // s0 < n: checked above
    uint32_t* dst = out + s0 * kWords;
    uint32_t* lp = dst + 4 * kg * kWords + mrow;  // row 4 kg, column mrow; the rest are constant offsets
#pragma unroll
    for (int nt = 0; nt < 3; ++nt) {
      v4i q[3][3];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          q[b][kk] = *(const v4i*)(qb + (kk < 2 ? 0 : 3 * kSeqLen) + b * kSeqLen + (2 - nt) * 32 + kk * 32);
      v16i acc0 = {}, acc1 = {}, acc2a = {}, acc2b = {};
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0][kk], q[0][kk], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0][kk], q[1][kk], acc1, 0, 0, 0);
        acc2a = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0][kk], q[2][kk], acc2a, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1][kk], q[0][kk], acc1, 0, 0, 0);
        acc2b = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1][kk], q[1][kk], acc2b, 0, 0, 0);
        acc2a = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[2][kk], q[0][kk], acc2a, 0, 0, 0);
      }
      const uint32_t q96 = hl[32 * nt + mrow];  // Q_j[96][o] = h[o]
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        uint32_t y = (uint32_t)acc0[i] + ((uint32_t)acc1[i] << 8) + ((uint32_t)(acc2a[i] + acc2b[i]) << 16);
        y = mad24(w96r[i], q96, y) & kMask;
        const uint32_t row = 8 * (i / 4) + 4 * kg + (i % 4);
        if (row < rows) lp[(8 * (i / 4) + (i % 4)) * kWords + 32 * nt] = y;
      }
    }
    // Column 96 and c (Sec. 3.2: c_i jumped by j A delta) of the tile's rows.
    if (kg == 0 && mrow < rows) {
      dst[mrow * kWords + 96] = col96 & kMask;
      dst[mrow * kWords + 97] = c_jump(c_src, jm);
    }
    wave_sync();  // w96w is rewritten by the next tile
  }
}

}  // namespace

// Returns hipErrorInvalidValue (nothing launched) when the family is too small
// for the product form (n < 2 A), or E0 + (n - 1) delta needs more than 128
// bits.  Starts from `base` (seed == 0, E0 == 0) or from the state of `seed`
// at offset E0.
// H_fixed, if not null, holds the factor sequences instead of stream-ordered
// memory (room for h_cap factors; hipErrorInvalidValue if B - 1 exceeds it).
static hipError_t family_gemm(const uint32_t* base, int32_t seed, ranmar_u128 e0, ranmar_u128 delta, uint64_t n,
                              uint32_t* out, hipStream_t st, uint32_t tr, uint32_t* H_fixed = nullptr,
                              uint64_t h_cap = 0) {
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  const unsigned __int128 E0 = ((unsigned __int128)e0.hi << 64) | e0.lo;
  const unsigned __int128 kMax = ~(unsigned __int128)0;
  if (n < 2 || D > (kMax - E0) / (n - 1)) return hipErrorInvalidValue;
  // A ~ sqrt(n) (a multiple of the tile height tr): A direct jumps plus B - 1
  // factor jumps.
  uint64_t A = (uint64_t)std::ceil(std::sqrt((double)n) / (double)tr) * tr;
  if (A < tr) A = tr;
  if (2 * A > n) return hipErrorInvalidValue;
  const uint64_t B = (n + A - 1) / A;
  const uint64_t njobs = A + (B - 1);
  // Tiles per wave: enough that the workgroups fit on the device at once,
  // at most eight (a workgroup builds its factor's sequences once).
  int dev = 0, cus = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* kern = tr == 32 ? (const void*)k_family_gemm32 : (const void*)k_family_gemm;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu <= 0) per_cu = 2;
  const uint64_t slots = (uint64_t)(cus > 0 ? cus : 256) * (uint64_t)per_cu;  // resident workgroups
  const uint64_t all_tiles = (B - 1) * (A / tr);
  const uint64_t want = (all_tiles + 4 * slots - 1) / (4 * slots);
  const uint32_t tpw = (uint32_t)(want < 1 ? 1 : (want > 8 ? 8 : want));
  const uint64_t wg_tiles = 4 * (uint64_t)tpw;  // source tiles per workgroup
  const uint64_t gx = (A / tr + wg_tiles - 1) / wg_tiles;
  if ((njobs + 7) / 8 > 0x7FFFFFFFull || gx > 0x7FFFFFFFull || B - 1 > 65535) return hipErrorInvalidValue;
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  if (H_fixed && B - 1 > h_cap) return hipErrorInvalidValue;
  const unsigned __int128 AD = D * A;  // < n delta, and A <= n - 1
  uint32_t* H = H_fixed;
  hipError_t e = hipSuccess;
  if (!H_fixed) e = hipMallocAsync((void**)&H, sizeof(uint32_t) * kHWords * (B - 1), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_family_l1, dim3((unsigned)((njobs + 7) / 8)), dim3(256), 0, st, base, out, H, T, A, njobs,
                     (uint64_t)D, (uint64_t)(D >> 64), (uint64_t)AD, (uint64_t)(AD >> 64),
                     (uint32_t)(seed == 0 && base == out ? 1 : 0), seed, e0.lo, e0.hi);
  e = hipGetLastError();
  if (e == hipSuccess) {
    if (tr == 32)
      hipLaunchKernelGGL(k_family_gemm32, dim3((unsigned)gx, (unsigned)(B - 1)), dim3(256), 0, st, out, H, A, n,
                         (uint32_t)(AD % kMod), tpw);
    else
      hipLaunchKernelGGL(k_family_gemm, dim3((unsigned)gx, (unsigned)(B - 1)), dim3(256), 0, st, out, H, A, n,
                         (uint32_t)(AD % kMod), tpw);
    e = hipGetLastError();
  }
  const hipError_t f = H_fixed ? hipSuccess : hipFreeAsync(H, st);
  return e != hipSuccess ? e : f;
}

hipError_t launch_family_gemm(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st,
                              uint32_t tile_rows) {
  return family_gemm(base, 0, ranmar_u128{0, 0}, delta, n, out, st, tile_rows == 32 ? 32u : 16u);
}

// ---------------------------------------------------------------------------
// No-allocation form, for callers that cannot allocate device memory.  The
// factor sequences go to a fixed array instead of stream-ordered memory:
// kHWords words per factor, room for kNoAllocFactors factors (3.2 MB), which
// covers every family of up to 2^24 starts (A = B = 4096 at most).  The array
// is held by each device the library runs on until the process ends; host
// code uses only the address taken from it at set-up, never its name (which
// on the host is a stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr uint64_t kNoAllocFactors = 4096;
static __device__ __align__(256) uint32_t scratch[kHWords * kNoAllocFactors];
static_assert(sizeof(uint32_t) * kHWords * kNoAllocFactors == RANMAR_NOALLOC_FAMILY_BYTES,
              "the public size of the no-allocation scratch array");

static std::mutex g_scratch_mu;
static std::atomic<uint32_t*> g_scratch_ptr[64];  // per device, set once by noalloc_setup

int noalloc_setup() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RANMAR_ENODEV;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev].load(std::memory_order_acquire)) return RANMAR_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return RANMAR_EHIP;
  }
  // The family's first launch reads the 8-bit window table: build it now, so
  // that the no-allocation calls never have to.
  if (!window_table()) return RANMAR_ENOMEM;
  g_scratch_ptr[dev].store((uint32_t*)ptr, std::memory_order_release);
  return RANMAR_OK;
}

uint32_t* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  return g_scratch_ptr[dev].load(std::memory_order_acquire);
}

hipError_t launch_family_gemm_fixed(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out,
                                    hipStream_t st, uint32_t tile_rows, uint32_t* H) {
  return family_gemm(base, 0, ranmar_u128{0, 0}, delta, n, out, st, tile_rows == 32 ? 32u : 16u, H,
                     kNoAllocFactors);
}

hipError_t launch_family_gemm_seeded(int32_t seed, ranmar_u128 e0, ranmar_u128 delta, uint64_t n, uint32_t* out,
                                     hipStream_t st, uint32_t tile_rows) {
  return family_gemm(nullptr, seed, e0, delta, n, out, st, tile_rows == 32 ? 32u : 16u);
}

}  // namespace ranmar
