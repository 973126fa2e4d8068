// Half-wave cooperative seeding and windowed jump-ahead (see coop_dev.hpp):
// eight requests per 256-thread workgroup, state and polynomial in LDS.
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "coop_dev.hpp"
#include "internal.hpp"
#include "jump_dev.hpp"

namespace ranmar {

constexpr int kHalfWords = 193 + 97;  // extended window + polynomial

template <bool SEED, int WB>
__global__ __launch_bounds__(256) void k_jump_coop(uint32_t* __restrict__ states, const int32_t* __restrict__ seeds,
                                                   const ranmar_u128* __restrict__ J, uint64_t n,
                                                   const uint32_t* __restrict__ T) {
  __shared__ uint32_t lds[8 * kHalfWords];
  const uint32_t hw = threadIdx.x >> 5, l = threadIdx.x & 31u;
  const uint64_t r = (uint64_t)blockIdx.x * 8u + hw;
  const bool active = r < n;
  uint32_t* X = lds + hw * kHalfWords;
  uint32_t* B = X + 193;
  uint32_t* slot = states + (active ? r : 0) * kWords;
  bool valid = active;
  uint32_t c = 0;
  if (SEED) {
    if (active) valid = seed_half(seeds[r], X, l);
    wave_sync();
    c = X[97];
  } else if (active) {
    X[l] = slot[l];
    X[l + 32] = slot[l + 32];
    X[l + 64] = slot[l + 64];
    if (l == 0) X[96] = slot[96];
    c = slot[97];
  }
  uint32_t j0 = 0, j1 = 0, j2 = 0, j3 = 0;
  if (valid && J) {
    const uint64_t lo = J[r].lo, hi = J[r].hi;
    j0 = (uint32_t)lo;
    j1 = (uint32_t)(lo >> 32);
    j2 = (uint32_t)hi;
    j3 = (uint32_t)(hi >> 32);
  }
  if (!valid) X[l] = X[l + 32] = X[l + 64] = 0;  // keep the idle half's arithmetic defined
  wave_sync();
  jump_half<WB>(X, B, T, j0, j1, j2, j3, wave_windows<WB>(j0, j1, j2, j3), l);
  if (valid) {
    slot[l] = X[l];
    slot[l + 32] = X[l + 32];
    slot[l + 64] = X[l + 64];
    if (l == 0) {
      slot[96] = X[96];
      slot[97] = c_jump(c, u128_mod_m(j0, j1, j2, j3));
    }
  } else if (SEED && active) {
    slot[l] = slot[l + 32] = slot[l + 64] = 0;
    if (l == 0) {
      slot[96] = 0;
      slot[97] = kInvalidC;
    }
  }
}

// The same with G lanes per request (G = 8 or 16), 256 / G requests per
// workgroup.  The per-request LDS stride is 1 mod 4, so the requests that
// share one 32-lane LDS pass fall on disjoint bank residues (a group's lanes
// are K = 96 / G words apart, K a multiple of 2 or 4).
constexpr int kGroupStride = 193 + 97 + 3;

template <int G, int WB, bool SEED>
__global__ __launch_bounds__(256) void k_jump_grp(uint32_t* __restrict__ states, const int32_t* __restrict__ seeds,
                                                  const ranmar_u128* __restrict__ J, uint64_t n,
                                                  const uint32_t* __restrict__ T) {
  constexpr uint32_t kPerWg = 256 / G;
  __shared__ uint32_t lds[kPerWg * kGroupStride];
  __shared__ SeedLds<true> seed_tab;
  const uint32_t q = threadIdx.x / G, l = threadIdx.x % G;
  const uint64_t r = (uint64_t)blockIdx.x * kPerWg + q;
  const bool active = r < n;
  uint32_t* X = lds + q * kGroupStride;
  uint32_t* B = X + 193;
  uint32_t* slot = states + (active ? r : 0) * kWords;
  bool valid = active;
  uint32_t c = 0;
  if (SEED) {
    seed_lds_fill(seed_tab, threadIdx.x, 256);
    __syncthreads();  // every thread of the workgroup reaches it
    if (active) valid = seed_group_tab<G, 7, true>(seeds[r], X, l, seed_tab);
    wave_sync();
    c = X[97];
  } else if (active) {
#pragma unroll
    for (int k = 0; k < 96; k += G) X[l + k] = slot[l + k];
    if (l == 0) X[96] = slot[96];
    c = slot[97];
  }
  uint32_t j0 = 0, j1 = 0, j2 = 0, j3 = 0;
  if (valid && J) {
    const uint64_t lo = J[r].lo, hi = J[r].hi;
    j0 = (uint32_t)lo;
    j1 = (uint32_t)(lo >> 32);
    j2 = (uint32_t)hi;
    j3 = (uint32_t)(hi >> 32);
  }
  if (!valid) {  // keep the idle group's arithmetic defined
#pragma unroll
    for (int k = 0; k < 96; k += G) X[l + k] = 0;
    if (l == 0) X[96] = 0;
  }
  wave_sync();
  jump_group<G, WB>(X, B, T, j0, j1, j2, j3, wave_windows<WB>(j0, j1, j2, j3), l);
  if (valid) {
#pragma unroll
    for (int k = 0; k < 96; k += G) slot[l + k] = X[l + k];
    if (l == 0) {
      slot[96] = X[96];
      slot[97] = c_jump(c, u128_mod_m(j0, j1, j2, j3));
    }
  } else if (SEED && active) {
#pragma unroll
    for (int k = 0; k < 96; k += G) slot[l + k] = 0;
    if (l == 0) {
      slot[96] = 0;
      slot[97] = kInvalidC;
    }
  }
}

// Seeding only, 32 lanes per seed (for few seeds: a lane-per-seed launch would
// run Algorithm 3's 2328 dependent steps on one lane).
__global__ __launch_bounds__(256) void k_seed_coop(const int32_t* __restrict__ seeds, uint64_t n,
                                                   uint32_t* __restrict__ out) {
  __shared__ uint32_t lds[8 * 98];
  const uint32_t hw = threadIdx.x >> 5, l = threadIdx.x & 31u;
  const uint64_t r = (uint64_t)blockIdx.x * 8u + hw;
  if (r >= n) return;  // a whole half-wave leaves together
  uint32_t* X = lds + hw * 98;
  const bool valid = seed_half(seeds[r], X, l);
  wave_sync();
  uint32_t* slot = out + r * kWords;
  slot[l] = valid ? X[l] : 0u;
  slot[l + 32] = valid ? X[l + 32] : 0u;
  slot[l + 64] = valid ? X[l + 64] : 0u;
  if (l == 0) {
    slot[96] = valid ? X[96] : 0u;
    slot[97] = valid ? X[97] : kInvalidC;
  }
}

// One radix-256 round of a stream family: with the first M starts in place,
// start s in [first, min(n, 256 M)) is start s mod M jumped by (s div M) M
// delta, the sources read from src (the family itself, or the base record in
// the first round, where M = 1 and start 0 is the base jumped by 0).
// MD = M delta (< 2^128), MDmod = MD mod m.  The factors are the table rows
// of the exponent's nonzero 8-bit digits; for delta = 2^40 and M = 256^i the
// exponent has one digit, so every start costs one application.
__global__ __launch_bounds__(256) void k_family_radix(uint32_t* __restrict__ out, const uint32_t* src_tab,
                                                      const uint32_t* __restrict__ T, uint64_t M, uint64_t first,
                                                      uint64_t cnt, uint64_t md_lo, uint64_t md_hi, uint32_t md_mod) {
  __shared__ uint32_t lds[8 * kHalfWords];
  const uint32_t hw = threadIdx.x >> 5, l = threadIdx.x & 31u;
  const uint64_t g = (uint64_t)blockIdx.x * 8u + hw;
  const bool active = g < cnt;
  const uint64_t s = first + (active ? g : 0);
  const uint64_t jdig = s / M, src_i = s - jdig * M;
  uint32_t* X = lds + hw * kHalfWords;
  uint32_t* B = X + 193;
  const uint32_t* src = src_tab + src_i * kWords;
  X[l] = src[l];
  X[l + 32] = src[l + 32];
  X[l + 64] = src[l + 64];
  if (l == 0) X[96] = src[96];
  const uint32_t c = src[97];
  // E = jdig * MD, exact: jdig < 256 and E <= (n - 1) delta < 2^128.
  const unsigned __int128 E = (unsigned __int128)jdig * (((unsigned __int128)md_hi << 64) | md_lo);
  const uint64_t elo = active ? (uint64_t)E : 0, ehi = active ? (uint64_t)(E >> 64) : 0;
  const uint32_t j0 = (uint32_t)elo, j1 = (uint32_t)(elo >> 32), j2 = (uint32_t)ehi, j3 = (uint32_t)(ehi >> 32);
  wave_sync();
  jump_half(X, B, T, j0, j1, j2, j3, wave_windows(j0, j1, j2, j3), l);
  if (active) {
    uint32_t* dst = out + s * kWords;
    dst[l] = X[l];
    dst[l + 32] = X[l + 32];
    dst[l + 64] = X[l + 64];
    if (l == 0) {
      dst[96] = X[96];
      dst[97] = c_jump(c, (uint32_t)(jdig * md_mod % kMod));
    }
  }
}

// The same round with G lanes per start (the grouped jump of k_jump_grp), for
// rounds with many starts.
template <int G>
__global__ __launch_bounds__(256) void k_family_radix_grp(uint32_t* __restrict__ out, const uint32_t* src_tab,
                                                          const uint32_t* __restrict__ T, uint64_t M, uint64_t first,
                                                          uint64_t cnt, uint64_t md_lo, uint64_t md_hi,
                                                          uint32_t md_mod) {
  constexpr uint32_t kPerWg = 256 / G;
  __shared__ uint32_t lds[kPerWg * kGroupStride];
  const uint32_t q = threadIdx.x / G, l = threadIdx.x % G;
  const uint64_t g = (uint64_t)blockIdx.x * kPerWg + q;
  const bool active = g < cnt;
  const uint64_t s = first + (active ? g : 0);
  const uint64_t jdig = s / M, src_i = s - jdig * M;
  uint32_t* X = lds + q * kGroupStride;
  uint32_t* B = X + 193;
  const uint32_t* src = src_tab + src_i * kWords;
#pragma unroll
  for (int k = 0; k < 96; k += G) X[l + k] = src[l + k];
  if (l == 0) X[96] = src[96];
  const uint32_t c = src[97];
  const unsigned __int128 E = (unsigned __int128)jdig * (((unsigned __int128)md_hi << 64) | md_lo);
  const uint64_t elo = active ? (uint64_t)E : 0, ehi = active ? (uint64_t)(E >> 64) : 0;
  const uint32_t j0 = (uint32_t)elo, j1 = (uint32_t)(elo >> 32), j2 = (uint32_t)ehi, j3 = (uint32_t)(ehi >> 32);
  wave_sync();
  jump_group<G, 8>(X, B, T, j0, j1, j2, j3, wave_windows<8>(j0, j1, j2, j3), l);
  if (active) {
    uint32_t* dst = out + s * kWords;
#pragma unroll
    for (int k = 0; k < 96; k += G) dst[l + k] = X[l + k];
    if (l == 0) {
      dst[96] = X[96];
      dst[97] = c_jump(c, (uint32_t)(jdig * md_mod % kMod));
    }
  }
}

// One request with its values passed by argument: the state of `seed` at
// offset E (Algorithm 3, then the windowed jump with c by its closed form).
// One half-wave; the caller has checked the seed.
__global__ __launch_bounds__(32) void k_seed_jump_one(uint32_t* __restrict__ out, int32_t seed, uint64_t e_lo,
                                                      uint64_t e_hi, const uint32_t* __restrict__ T) {
  __shared__ uint32_t lds[kHalfWords];
  const uint32_t l = threadIdx.x & 31u;
  uint32_t* X = lds;
  uint32_t* B = X + 193;
  seed_half(seed, X, l);
  wave_sync();
  const uint32_t c = X[97];
  const uint32_t j0 = (uint32_t)e_lo, j1 = (uint32_t)(e_lo >> 32), j2 = (uint32_t)e_hi, j3 = (uint32_t)(e_hi >> 32);
  jump_half(X, B, T, j0, j1, j2, j3, wave_windows(j0, j1, j2, j3), l);
  out[l] = X[l];
  out[l + 32] = X[l + 32];
  out[l + 64] = X[l + 64];
  if (l == 0) {
    out[96] = X[96];
    out[97] = c_jump(c, u128_mod_m(j0, j1, j2, j3));
  }
}

hipError_t launch_seed_jump_one(uint32_t* out, int32_t seed, ranmar_u128 E, hipStream_t st) {
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(k_seed_jump_one, dim3(1), dim3(32), 0, st, out, seed, E.lo, E.hi, T);
  return hipGetLastError();
}

hipError_t launch_seed_coop(const int32_t* seeds, uint64_t n, uint32_t* out, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_seed_coop, dim3((unsigned)((n + 7) / 8)), dim3(256), 0, st, seeds, n, out);
  return hipGetLastError();
}

// Family by radix-256 rounds (each one launch).  Returns hipErrorInvalidValue
// (nothing launched) when (n - 1) delta does not fit in 128 bits; the caller
// then uses the polynomial path.
hipError_t launch_family_window(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st) {
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  const unsigned __int128 kMax = ~(unsigned __int128)0;
  if (n > 1 && D > kMax / (n - 1)) return hipErrorInvalidValue;
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  // The first radix round reads the base record and also writes start 0 (the base itself)
  // unless the family is built in place.
  for (uint64_t M = 1, first = (base != out) ? 0 : 1; M < n || first < M; first = M) {
    const uint64_t top = (M <= n / 256) ? 256 * M : n;  // starts [first, top) this round
    const uint64_t cnt = top - first;
    if ((cnt + 7) / 8 > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const unsigned __int128 MD = D * M;  // <= (n - 1) delta
    const uint32_t md_mod = (uint32_t)(MD % kMod);
    const uint32_t* src = M == 1 ? base : (const uint32_t*)out;
    if (cnt >= 16384)  // many starts: 8 lanes each (more useful multiply-adds per issue)
      hipLaunchKernelGGL((k_family_radix_grp<8>), dim3((unsigned)((cnt + 31) / 32)), dim3(256), 0, st, out, src, T,
                         M, first, cnt, (uint64_t)MD, (uint64_t)(MD >> 64), md_mod);
    else  // few: 32 lanes each (lower latency)
      hipLaunchKernelGGL(k_family_radix, dim3((unsigned)((cnt + 7) / 8)), dim3(256), 0, st, out, src, T, M, first,
                         cnt, (uint64_t)MD, (uint64_t)(MD >> 64), md_mod);
    M = top;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window tables, one per device and width, built by the square-and-multiply
// kernel: T[w][d] = t^(d 2^(WB w)) mod phi.  WB = 8: 16 x 256 rows (1.6 MB,
// L2-resident).  WB = 16: 8 x 65536 rows (203 MB), for bulk jumps, where it
// halves the number of applications; WB = 20 (2.4 GB) and WB = 24 (32.5 GB of
// the device's 288 GB) take 6 and 5 factors for a 120-bit J instead of 15.
// ---------------------------------------------------------------------------

// J[i] = d 2^(wb w) for row r0 + i = w 2^wb + d.
__global__ __launch_bounds__(256) void k_window_exponents(ranmar_u128* __restrict__ J, uint64_t r0, uint64_t n,
                                                          int wb) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint64_t r = r0 + i;
  const uint64_t w = r >> wb, d = r & ((1ull << wb) - 1ull);
  const unsigned __int128 v = (unsigned __int128)d << (wb * w);
  J[i].lo = (uint64_t)v;
  J[i].hi = (uint64_t)(v >> 64);
}

template <int WB>
__global__ __launch_bounds__(256) void k_jump_poly_tab(const ranmar_u128* __restrict__ J, uint64_t n,
                                                       uint32_t* __restrict__ P, const uint32_t* __restrict__ T);

// T8: the 8-bit table when wb > 8 (the wider tables are products of its
// factors), else nullptr.
static const uint32_t* build_window_table(int wb, const uint32_t* T8) {
  const int windows = (128 + wb - 1) / wb;
  const uint64_t digits = 1ull << wb;
  const int last_bits = 128 - wb * (windows - 1);  // the last window may be narrower (8 bits for wb = 20 or 24)
  const uint64_t n = (uint64_t)(windows - 1) * digits + (1ull << last_bits);
  // The exponents are made on the device, a slice of rows at a time.
  constexpr uint64_t kSlice = 1ull << 22;
  const uint64_t slice = n < kSlice ? n : kSlice;
  uint32_t* T = nullptr;
  ranmar_u128* dJ = nullptr;
  hipStream_t st = nullptr;
  bool ok = hipMalloc(&T, 4 * 97 * n) == hipSuccess && hipMalloc(&dJ, sizeof(ranmar_u128) * slice) == hipSuccess &&
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  // The 8-bit table is built by square-and-multiply; the wider ones as
  // products of its factors (a 24-bit digit spans three 8-bit ones: at most
  // two products per row, where square-and-multiply takes up to 122 squarings).
  for (uint64_t r0 = 0; ok && r0 < n; r0 += slice) {
    const uint64_t cnt = n - r0 < slice ? n - r0 : slice;
    hipLaunchKernelGGL(k_window_exponents, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, dJ, r0, cnt, wb);
    ok = hipGetLastError() == hipSuccess;
    if (ok && T8)
      hipLaunchKernelGGL(k_jump_poly_tab<8>, dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, st, dJ, cnt, T + r0 * 97,
                         T8);
    else if (ok)
      ok = launch_jump_poly(dJ, cnt, T + r0 * 97, st) == hipSuccess;
    ok = ok && hipGetLastError() == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (st) hipStreamDestroy(st);
  hipFree(dJ);
  if (!ok) {
    hipFree(T);
    (void)hipGetLastError();  // a failed allocation is reported by the nullptr, not left for the next call
    return nullptr;
  }
  return T;
}

// Built 20-bit tables, published for readers that must not wait for a build
// (devices 0..63).
static std::atomic<const uint32_t*> g_t20_ready[64];

static const uint32_t* cached_window_table(int wb) {
  // A wider table is built from the 8-bit one, which is taken first (its
  // own call holds the lock below only while it builds).
  const uint32_t* T8 = wb > 8 ? cached_window_table(8) : nullptr;
  if (wb > 8 && !T8) return nullptr;
  static std::mutex mu;
  static std::map<std::pair<int, int>, const uint32_t*> tabs;  // (device, width) -> table; failures cached too
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  auto it = tabs.find({dev, wb});
  if (it != tabs.end()) return it->second;
  const uint32_t* T = build_window_table(wb, T8);
  tabs[{dev, wb}] = T;
  if (wb == 20 && dev >= 0 && dev < 64) g_t20_ready[dev].store(T, std::memory_order_release);
  return T;
}

const uint32_t* window_table() { return cached_window_table(8); }
const uint32_t* window16_table() { return cached_window_table(16); }
const uint32_t* window20_table() { return cached_window_table(20); }
const uint32_t* window24_table() { return cached_window_table(24); }

const uint32_t* window20_table_ready() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  return g_t20_ready[dev].load(std::memory_order_acquire);
}

// t^J mod phi (Sec. 3.1), one J per wave, as the product of the window
// table's factors t^(d_w 2^(WB w)) over J's nonzero digits: with the 8-bit
// table at most 15 products of two 97-coefficient polynomials, each reduced
// mod phi, where square-and-multiply takes up to 122 squarings.  Lane l makes
// coefficients 3l .. 3l + 2 of each product with a register window over the
// running product a, which slides by one coefficient per term.
template <int WB>
__global__ __launch_bounds__(256) void k_jump_poly_tab(const ranmar_u128* __restrict__ J, uint64_t n,
                                                       uint32_t* __restrict__ P, const uint32_t* __restrict__ T) {
  constexpr int kPad = 96 + 97 + 96;  // a with 96 zeros on each side
  __shared__ uint32_t lds[4][kPad + 97 + 193];
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63u;
  const uint64_t r = (uint64_t)blockIdx.x * 4u + wv;
  if (r >= n) return;  // whole waves leave; no barrier follows
  uint32_t* pad = lds[wv];
  uint32_t* b = pad + kPad;   // the factor
  uint32_t* prod = b + 97;    // the unreduced product
  const uint64_t lo = J[r].lo, hi = J[r].hi;
  const uint32_t j0 = (uint32_t)lo, j1 = (uint32_t)(lo >> 32), j2 = (uint32_t)hi, j3 = (uint32_t)(hi >> 32);
  for (uint32_t i = l; i < (uint32_t)kPad; i += 64) pad[i] = i == 96 ? 1u : 0u;
  constexpr int kWin = (128 + WB - 1) / WB;
  // The next factor's row is fetched while the current product runs.
  int w = next_window<WB>(j0, j1, j2, j3, 0, kWin);
  uint32_t r0 = 0, r1 = 0;
  if (w < kWin) {
    const uint32_t* row = window_row<WB>(T, j0, j1, j2, j3, w);
    r0 = row[l];
    r1 = l < 33 ? row[64 + l] : 0u;
  }
  while (w < kWin) {
    b[l] = r0;
    if (l < 33) b[64 + l] = r1;
    wave_sync();
    w = next_window<WB>(j0, j1, j2, j3, w + 1, kWin);
    if (w < kWin) {
      const uint32_t* row = window_row<WB>(T, j0, j1, j2, j3, w);
      r0 = row[l];
      r1 = l < 33 ? row[64 + l] : 0u;
    }
    // w0, w1, w2 = a_(3l-i), a_(3l+1-i), a_(3l+2-i) at term i.
    const uint32_t* al = pad + 96 + 3 * l;
    uint32_t w0 = al[0], w1 = al[1], w2 = al[2], c0 = 0, c1 = 0, c2 = 0;
#pragma unroll 8
    for (int i = 0; i < 96; ++i) {
      const uint32_t bi = b[i];
      c0 = mad24(bi, w0, c0);
      c1 = mad24(bi, w1, c1);
      c2 = mad24(bi, w2, c2);
      w2 = w1;
      w1 = w0;
      w0 = al[-(i + 1)];
    }
    c0 = mad24(b[96], w0, c0);
    c1 = mad24(b[96], w1, c1);
    c2 = mad24(b[96], w2, c2);
    const uint32_t c192 = mad24(b[96], pad[96 + 96], 0u);  // the top coefficient, a_96 b_96
    prod[3 * l] = c0;
    prod[3 * l + 1] = c1;
    prod[3 * l + 2] = c2;
    if (l == 0) prod[192] = c192;
    wave_sync();
    const uint32_t v0 = fold_phi(prod, (int)l);
    const uint32_t v1 = l < 33 ? fold_phi(prod, (int)l + 64) : 0u;
    wave_sync();
    pad[96 + l] = v0 & kMask;
    if (l < 33) pad[160 + l] = v1 & kMask;
    wave_sync();
  }
  uint32_t* dst = P + r * 97u;
  dst[l] = pad[96 + l];
  if (l < 33) dst[64 + l] = pad[160 + l];
}

hipError_t launch_jump_poly_tab(const ranmar_u128* J, uint64_t n, uint32_t* P, hipStream_t st) {
  if (!n) return hipSuccess;
  if ((n + 3) / 4 > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 3) / 4));
  // The 20-bit table (6 factors for 120 bits instead of 15) where it exists,
  // and built for bulk calls, as the jump kernels do.
  if (const uint32_t* T20 = n >= 16384 ? window20_table() : window20_table_ready()) {
    hipLaunchKernelGGL(k_jump_poly_tab<20>, grid, dim3(256), 0, st, J, n, P, T20);
  } else {
    const uint32_t* T = window_table();
    if (!T) return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_jump_poly_tab<8>, grid, dim3(256), 0, st, J, n, P, T);
  }
  return hipGetLastError();
}

hipError_t launch_jump_coop(uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n,
                            hipStream_t st) {
  if (!n) return hipSuccess;
  const dim3 grid((unsigned)((n + 7) / 8));
  // Few requests: the 20-bit table's 6 factors where the table already
  // exists (it is not built for them), else the 8-bit table's.
  if (const uint32_t* T20 = window20_table_ready()) {
    if (seeds)
      hipLaunchKernelGGL((k_jump_coop<true, 20>), grid, dim3(256), 0, st, states, seeds, J, n, T20);
    else
      hipLaunchKernelGGL((k_jump_coop<false, 20>), grid, dim3(256), 0, st, states, seeds, J, n, T20);
    return hipGetLastError();
  }
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  if (seeds)
    hipLaunchKernelGGL((k_jump_coop<true, 8>), grid, dim3(256), 0, st, states, seeds, J, n, T);
  else
    hipLaunchKernelGGL((k_jump_coop<false, 8>), grid, dim3(256), 0, st, states, seeds, J, n, T);
  return hipGetLastError();
}

template <int G, int WB>
static hipError_t launch_jump_grp(uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n,
                                  hipStream_t st) {
  constexpr uint64_t kPerWg = 256 / G;
  if (!n) return hipSuccess;
  if ((n + kPerWg - 1) / kPerWg > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const uint32_t* T = WB == 24   ? window24_table()
                      : WB == 20 ? window20_table()
                      : WB == 16 ? window16_table()
                                 : window_table();
  if (!T) return hipErrorOutOfMemory;
  const dim3 grid((unsigned)((n + kPerWg - 1) / kPerWg));
  if (seeds)
    hipLaunchKernelGGL((k_jump_grp<G, WB, true>), grid, dim3(256), 0, st, states, seeds, J, n, T);
  else
    hipLaunchKernelGGL((k_jump_grp<G, WB, false>), grid, dim3(256), 0, st, states, seeds, J, n, T);
  return hipGetLastError();
}

hipError_t launch_jump_variant(int v, uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n,
                               hipStream_t st) {
  if (v == JUMP_QUARTER_WINDOW) return launch_jump_grp<16, 8>(states, seeds, J, n, st);
  if (v == JUMP_EIGHTH_WINDOW) return launch_jump_grp<8, 8>(states, seeds, J, n, st);
  // The 24-, 20- and 16-bit tables are large; without them narrower windows
  // do the same job.
  if (v == JUMP_EIGHTH_WINDOW24 && window24_table()) return launch_jump_grp<8, 24>(states, seeds, J, n, st);
  if ((v == JUMP_EIGHTH_WINDOW24 || v == JUMP_EIGHTH_WINDOW20) && window20_table())
    return launch_jump_grp<8, 20>(states, seeds, J, n, st);
  if (v == JUMP_EIGHTH_WINDOW24 || v == JUMP_EIGHTH_WINDOW20 || v == JUMP_EIGHTH_WINDOW16) {
    if (window16_table()) return launch_jump_grp<8, 16>(states, seeds, J, n, st);
    return launch_jump_grp<8, 8>(states, seeds, J, n, st);
  }
  if (v == JUMP_HALF_WINDOW) return launch_jump_coop(states, seeds, J, n, st);
  return launch_jump(states, seeds, J, n, st);
}

}  // namespace ranmar
