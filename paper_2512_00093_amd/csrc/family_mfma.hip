// Stream families as a matrix product on the matrix cores (MFMA int8).
//
// Starts k * delta, k < n, from a base state.  Write n = A * B (A a multiple
// of 16, B = ceil(n / A)) and start s = j A + i (i < A, j < B).  Then
//     x_s = x_i  P_j(A_c)        with P_j = t^(j A delta) mod phi
// (Sec. 3.1: the jump is the matrix P(A_c) of the companion matrix A_c acting
// on the row vector x), and c_s is c_i jumped by j A delta (Sec. 3.2).  So the
// x-parts of all starts with the same j are one product
//     Y_j [A x 97] = W [A x 97] * Q_j [97 x 97],   Q_j = P_j(A_c) mod 2^24,
// where row r of Q_j is the unit window e_r jumped by j A delta.  Every
// factor is shared by A starts: a dense contraction, unlike a jump of one
// state by its own polynomial.
//
// Launch 1 (VALU, 32 lanes per job, the windowed jump of coop_dev.hpp):
//   jobs [0, A):          x_i = base jumped by i delta (with c), into out;
//   jobs [A, A + 128(B-1)): job (j, r): row r of Q_j (e_r jumped by j A delta),
//                         written as three signed 8-bit limbs, transposed
//                         (k = r contiguous) and zero-padded to 112 x 128,
//                         the layout the MFMA B operand reads.
// Launch 2 (MFMA): a workgroup per (j, 8 tiles of 16 sources) stages Q_j in
// LDS once; each wave takes two tiles: the 16 x 97 block of W is split into
// limbs in registers, and for each of seven 16-column tiles
//     Y = W0 Q0 + 2^8 (W0 Q1 + W1 Q0) + 2^16 (W0 Q2 + W1 Q1 + W2 Q0)  (mod 2^24)
// with v_mfma_i32_16x16x64_i8 (K = 97 padded to 128: two steps), 12 MFMAs
// per tile.  Exactness: a 24-bit word is w0 + 2^8 w1 + 2^16 w2 (mod 2^24)
// with signed limbs in [-128, 127]; limb products with weight >= 2^24 vanish
// mod 2^24; each accumulator sums at most 3 x 97 products of magnitude <= 2^14,
// far inside int32, and the final combination wraps mod 2^32, then is masked.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "coop_dev.hpp"
#include "internal.hpp"

namespace ranmar {

namespace {

constexpr int kQN = 112;  // output columns, padded to 7 tiles of 16
constexpr int kQK = 128;  // source words, padded to 2 K-steps of 64
constexpr uint64_t kQBytes = 3ull * kQN * kQK;  // one Q_j: three limb planes of [kQN][kQK] int8
constexpr int kL1Words = 193 + 97;             // LDS per half-wave: extended window + polynomial

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

__global__ __launch_bounds__(256) void k_family_l1(const uint32_t* base, uint32_t* out, int8_t* __restrict__ Qg,
                                                   const uint32_t* __restrict__ T, uint64_t A, uint64_t njobs,
                                                   uint64_t d_lo, uint64_t d_hi, uint64_t ad_lo, uint64_t ad_hi,
                                                   uint32_t in_place) {
  __shared__ uint32_t lds[8 * kL1Words];
  const uint32_t hw = threadIdx.x >> 5, l = threadIdx.x & 31u;
  const uint64_t t = (uint64_t)blockIdx.x * 8u + hw;
  const bool active = t < njobs;
  const bool is_start = t < A;
  uint32_t* X = lds + hw * kL1Words;
  uint32_t* Bp = X + 193;
  unsigned __int128 E = 0;
  uint32_t c = 0;
  uint64_t jq = 0, r = 0;
  if (is_start) {
    X[l] = base[l];
    X[l + 32] = base[l + 32];
    X[l + 64] = base[l + 64];
    if (l == 0) X[96] = base[96];
    c = base[97];
    E = (unsigned __int128)t * (((unsigned __int128)d_hi << 64) | d_lo);  // t delta <= (n - 1) delta
  } else {
    const uint64_t u = active ? t - A : 0;
    jq = u / kQK;  // j - 1
    r = u % kQK;
    X[l] = X[l + 32] = X[l + 64] = 0;
    if (l == 0) X[96] = 0;
    wave_sync();
    if (l == 0 && r < 97) X[r] = 1u;
    if (active && r < 97) E = (unsigned __int128)(jq + 1) * (((unsigned __int128)ad_hi << 64) | ad_lo);
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
    // Column r of the transposed limb planes: Qg[jq][b][o][r], o < kQN.
    int8_t* q = Qg + jq * kQBytes + r;
#pragma unroll
    for (uint32_t o = l; o < (uint32_t)kQN; o += 32) {
      int w0 = 0, w1 = 0, w2 = 0;
      if (o < 97 && r < 97) limbs3(X[o], w0, w1, w2);
      q[(0 * kQN + o) * kQK] = (int8_t)w0;
      q[(1 * kQN + o) * kQK] = (int8_t)w1;
      q[(2 * kQN + o) * kQK] = (int8_t)w2;
    }
  }
}

// 16 int8 limbs (plane b) of words w[0..15] packed for an MFMA operand.
__device__ __forceinline__ v4i pack_limbs(const int (&w)[16]) {
  v4i v;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    v[d] = (w[4 * d] & 0xFF) | ((w[4 * d + 1] & 0xFF) << 8) | ((w[4 * d + 2] & 0xFF) << 16) |
           ((uint32_t)(w[4 * d + 3] & 0xFF) << 24);
  return v;
}

// LDS layout of Q_j: 336 rows (3 limb planes x 112 columns) of 128 bytes,
// padded to 144 so that the 16 lanes reading one 16-byte piece of 16
// consecutive rows fall on different banks.
constexpr int kQRow = 144;
constexpr int kTilesPerWave = 2;

__global__ __launch_bounds__(256) void k_family_gemm(uint32_t* out, const int8_t* __restrict__ Qg, uint64_t A,
                                                     uint64_t n, uint32_t ad_mod) {
  __shared__ __attribute__((aligned(16))) int8_t q_lds[3 * kQN * kQRow];
  // Per wave: the 16 source records of a tile, then its 16 output records
  // (both contiguous in memory, so they are read and written whole).
  __shared__ uint32_t blk_all[4][16 * kWords];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint64_t jq = blockIdx.y, j = jq + 1;
  const uint64_t tiles = A / 16;
  // Q_j, staged once for the workgroup's tiles: every load is issued before
  // the first LDS write, so the round trips overlap.
  {
    constexpr uint32_t kChunks = kQBytes / 16, kIt = (kChunks + 255) / 256;
    const v4i* src = (const v4i*)(Qg + jq * kQBytes);
    v4i tmp[kIt];
#pragma unroll
    for (uint32_t it = 0; it < kIt; ++it) {
      const uint32_t x = threadIdx.x + 256 * it;
      if (x < kChunks) tmp[it] = src[x];
    }
#pragma unroll
    for (uint32_t it = 0; it < kIt; ++it) {
      const uint32_t x = threadIdx.x + 256 * it;
      if (x < kChunks) *(v4i*)(q_lds + (x >> 3) * kQRow + (x & 7) * 16) = tmp[it];
    }
  }
  __syncthreads();  // the only workgroup barrier: every wave reaches it
  uint32_t* blk = blk_all[wave];
  const uint32_t mrow = lane & 15u, kg = lane >> 4;
  // Source records of a tile: 16 contiguous records, loaded into registers
  // (all loads in flight together); the next tile's are loaded while the
  // current tile is multiplied.
  constexpr uint32_t kIt = (16 * kWords + 63) / 64;
  auto tile_ok = [&](int tt) {
    const uint64_t tile = ((uint64_t)blockIdx.x * 4 + wave) * kTilesPerWave + tt;
    return tile < tiles && j * A + tile * 16 < n;  // blocks of the last factor may lie beyond n
  };
  auto load_src = [&](int tt, uint32_t (&tmp)[kIt]) {
    const uint64_t i0 = (((uint64_t)blockIdx.x * 4 + wave) * kTilesPerWave + tt) * 16;
    const uint32_t* wsrc = out + i0 * kWords;
#pragma unroll
    for (uint32_t it = 0; it < kIt; ++it) {
      const uint32_t w = lane + 64 * it;
      if (w < 16 * kWords) tmp[it] = wsrc[w];
    }
  };
  uint32_t nxt[kIt];
  if (tile_ok(0)) load_src(0, nxt);
  for (int tt = 0; tt < kTilesPerWave; ++tt) {
    if (!tile_ok(tt)) break;  // and so are the later tiles
    const uint64_t tile = ((uint64_t)blockIdx.x * 4 + wave) * kTilesPerWave + tt;
    const uint64_t i0 = tile * 16, s0 = j * A + i0;
#pragma unroll
    for (uint32_t it = 0; it < kIt; ++it) {
      const uint32_t w = lane + 64 * it;
      if (w < 16 * kWords) blk[w] = nxt[it];
    }
    if (tt + 1 < kTilesPerWave && tile_ok(tt + 1)) load_src(tt + 1, nxt);
    wave_sync();
    // A operand: rows mrow, words k = kk*64 + kg*16 + 0..15 (k >= 97: zero).
    v4i a[3][2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      int l0[16], l1[16], l2[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t k = kk * 64 + kg * 16 + e;
        const uint32_t v = k < 97 ? blk[mrow * kWords + k] : 0u;
        limbs3(v, l0[e], l1[e], l2[e]);
      }
      a[0][kk] = pack_limbs(l0);
      a[1][kk] = pack_limbs(l1);
      a[2][kk] = pack_limbs(l2);
    }
    const uint32_t c_src = lane < 16 ? blk[lane * kWords + 97] : 0u;
    wave_sync();  // blk now takes the outputs
#pragma unroll
    for (int nt = 0; nt < kQN / 16; ++nt) {
      const uint32_t o = nt * 16 + mrow;
      v4i q[3][2];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) q[b][kk] = *(const v4i*)(q_lds + (b * kQN + o) * kQRow + kk * 64 + kg * 16);
      v4i acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        acc0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0][kk], q[0][kk], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0][kk], q[1][kk], acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0][kk], q[2][kk], acc2, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1][kk], q[0][kk], acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1][kk], q[1][kk], acc2, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[2][kk], q[0][kk], acc2, 0, 0, 0);
      }
      // D layout: lane holds rows kg*4 + i, column mrow of the tile.
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t y = ((uint32_t)acc0[i] + ((uint32_t)acc1[i] << 8) + ((uint32_t)acc2[i] << 16)) & kMask;
        if (o < 97) blk[(kg * 4 + i) * kWords + o] = y;
      }
    }
    // c of the block's starts (Sec. 3.2): c_i jumped by j A delta.
    if (lane < 16) blk[lane * kWords + 97] = c_jump(c_src, (uint32_t)(j * ad_mod % kMod));
    wave_sync();
    const uint64_t rows = n - s0 < 16 ? n - s0 : 16;  // s0 < n: checked above
    uint32_t* dst = out + s0 * kWords;
#pragma unroll
    for (uint32_t it = 0; it < (16 * kWords + 63) / 64; ++it) {
      const uint32_t w = lane + 64 * it;
      if (w < rows * kWords) dst[w] = blk[w];
    }
    wave_sync();  // blk is reused by the next tile
  }
}

}  // namespace

// Returns hipErrorInvalidValue (nothing launched) when the family is too small
// for the product form (n < 2 A), or (n - 1) delta needs more than 128 bits.
hipError_t launch_family_gemm(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st) {
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  const unsigned __int128 kMax = ~(unsigned __int128)0;
  if (n < 2 || D > kMax / (n - 1)) return hipErrorInvalidValue;
  // A ~ sqrt(97 n): A direct jumps plus 97 (B - 1) factor rows.
  uint64_t A = (uint64_t)std::ceil(std::sqrt(97.0 * (double)n) / 16.0) * 16;
  if (A < 16) A = 16;
  if (2 * A > n) return hipErrorInvalidValue;
  const uint64_t B = (n + A - 1) / A;
  const uint64_t njobs = A + kQK * (B - 1);
  const uint64_t wg_tiles = 4 * kTilesPerWave;  // source tiles per workgroup
  const uint64_t gx = (A / 16 + wg_tiles - 1) / wg_tiles;
  if ((njobs + 7) / 8 > 0x7FFFFFFFull || gx > 0x7FFFFFFFull || B - 1 > 65535) return hipErrorInvalidValue;
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  const unsigned __int128 AD = D * A;  // < n delta, and A <= n - 1
  int8_t* Qg = nullptr;
  hipError_t e = hipMallocAsync((void**)&Qg, kQBytes * (B - 1), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_family_l1, dim3((unsigned)((njobs + 7) / 8)), dim3(256), 0, st, base, out, Qg, T, A, njobs,
                     (uint64_t)D, (uint64_t)(D >> 64), (uint64_t)AD, (uint64_t)(AD >> 64),
                     (uint32_t)(base == out ? 1 : 0));
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_family_gemm, dim3((unsigned)gx, (unsigned)(B - 1)), dim3(256), 0, st, out, Qg, A, n,
                       (uint32_t)(AD % kMod));
    e = hipGetLastError();
  }
  const hipError_t f = hipFreeAsync(Qg, st);
  return e != hipSuccess ? e : f;
}

}  // namespace ranmar
