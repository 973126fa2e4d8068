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
