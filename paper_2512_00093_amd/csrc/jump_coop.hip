// Half-wave cooperative seeding and windowed jump-ahead (see coop_dev.hpp):
// eight requests per 256-thread workgroup, state and polynomial in LDS.
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "coop_dev.hpp"
#include "internal.hpp"

namespace ranmar {

constexpr int kHalfWords = 193 + 97;  // extended window + polynomial

template <bool SEED>
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
  const int nwin = wave_windows(j0, j1, j2, j3);
  jump_half(X, B, T, j0, j1, j2, j3, nwin, l);
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

// One doubling round of a stream family: for k < cnt,
// out[dst0 + k] = out[k] jumped by the exponent whose nonzero 8-bit digits
// are given (window w_i, digit d_i): one table factor per digit.
struct FamilyDigits {
  uint32_t n;
  uint32_t jmod;           // exponent mod m
  uint16_t w[16], d[16];
};

__global__ __launch_bounds__(256) void k_family_round_coop(uint32_t* __restrict__ out,
                                                           const uint32_t* __restrict__ T, uint64_t cnt,
                                                           uint64_t dst0, FamilyDigits dg) {
  __shared__ uint32_t lds[8 * kHalfWords];
  const uint32_t hw = threadIdx.x >> 5, l = threadIdx.x & 31u;
  const uint64_t k = (uint64_t)blockIdx.x * 8u + hw;
  if (k >= cnt) return;  // a whole half-wave leaves together
  uint32_t* X = lds + hw * kHalfWords;
  uint32_t* B = X + 193;
  const uint32_t* src = out + k * kWords;
  X[l] = src[l];
  X[l + 32] = src[l + 32];
  X[l + 64] = src[l + 64];
  if (l == 0) X[96] = src[96];
  const uint32_t c = src[97];
  for (uint32_t i = 0; i < dg.n; ++i) {
    const uint32_t* row = T + ((uint64_t)dg.w[i] * kWinDigits + dg.d[i]) * 97u;
    B[l] = row[l];
    B[l + 32] = row[l + 32];
    B[l + 64] = row[l + 64];
    if (l == 0) B[96] = row[96];
    wave_sync();
    apply_half(X, B, l);
  }
  uint32_t* dst = out + (dst0 + k) * kWords;
  dst[l] = X[l];
  dst[l + 32] = X[l + 32];
  dst[l + 64] = X[l + 64];
  if (l == 0) {
    dst[96] = X[96];
    dst[97] = c_jump(c, dg.jmod);
  }
}

hipError_t launch_seed_coop(const int32_t* seeds, uint64_t n, uint32_t* out, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_seed_coop, dim3((unsigned)((n + 7) / 8)), dim3(256), 0, st, seeds, n, out);
  return hipGetLastError();
}

// Family by doubling rounds that each apply the table factors of 2^b delta.
// Returns hipErrorInvalidValue (nothing launched) when some 2^b delta needs
// more than 128 bits; the caller then uses the polynomial path.
hipError_t launch_family_window(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st) {
  int nb = 0;
  while (nb < 64 && (1ull << nb) < n) ++nb;
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  int dbits = 0;
  for (unsigned __int128 t = D; t; t >>= 1) ++dbits;
  if (nb > 0 && dbits + nb - 1 > 128) return hipErrorInvalidValue;
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  if (base != out) {
    hipError_t e = hipMemcpyAsync(out, base, 4 * kWords, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  const uint64_t dmod = (uint64_t)(D % kMod);
  uint64_t pow2 = 1;
  for (int b = 0; b < nb; ++b) {
    const unsigned __int128 E = D << b;  // < 2^128 by the check above
    FamilyDigits dg{};
    for (int w = 0; w < kWindows; ++w) {
      const uint32_t d = (uint32_t)(E >> (kWinBits * w)) & 0xFFu;
      if (d) {
        dg.w[dg.n] = (uint16_t)w;
        dg.d[dg.n] = (uint16_t)d;
        ++dg.n;
      }
    }
    dg.jmod = (uint32_t)((dmod * pow2) % kMod);
    pow2 = pow2 * 2 % kMod;
    const uint64_t half = 1ull << b;
    const uint64_t cnt = (n - half < half) ? n - half : half;
    hipLaunchKernelGGL(k_family_round_coop, dim3((unsigned)((cnt + 7) / 8)), dim3(256), 0, st, out, T, cnt, half, dg);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window table, one per device, built by the square-and-multiply kernel.
// ---------------------------------------------------------------------------
const uint32_t* window_table() {
  static std::mutex mu;
  static std::map<int, uint32_t*> tabs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  auto it = tabs.find(dev);
  if (it != tabs.end()) return it->second;
  const uint64_t n = (uint64_t)kWindows * kWinDigits;
  std::vector<ranmar_u128> Jh(n);
  for (int w = 0; w < kWindows; ++w)
    for (int d = 0; d < kWinDigits; ++d) {
      const unsigned __int128 v = (unsigned __int128)d << (kWinBits * w);
      Jh[w * kWinDigits + d].lo = (uint64_t)v;
      Jh[w * kWinDigits + d].hi = (uint64_t)(v >> 64);
    }
  uint32_t* T = nullptr;
  ranmar_u128* dJ = nullptr;
  hipStream_t st = nullptr;
  bool ok = hipMalloc(&T, 4 * 97 * n) == hipSuccess && hipMalloc(&dJ, sizeof(ranmar_u128) * n) == hipSuccess &&
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipMemcpyAsync(dJ, Jh.data(), sizeof(ranmar_u128) * n, hipMemcpyHostToDevice, st) == hipSuccess &&
            launch_jump_poly(dJ, n, T, st) == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
  if (st) hipStreamDestroy(st);
  hipFree(dJ);
  if (!ok) {
    hipFree(T);
    return nullptr;
  }
  tabs[dev] = T;
  return T;
}

hipError_t launch_jump_coop(uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n,
                            hipStream_t st) {
  if (!n) return hipSuccess;
  const uint32_t* T = window_table();
  if (!T) return hipErrorOutOfMemory;
  const dim3 grid((unsigned)((n + 7) / 8));
  if (seeds)
    hipLaunchKernelGGL(k_jump_coop<true>, grid, dim3(256), 0, st, states, seeds, J, n, T);
  else
    hipLaunchKernelGGL(k_jump_coop<false>, grid, dim3(256), 0, st, states, seeds, J, n, T);
  return hipGetLastError();
}

}  // namespace ranmar
