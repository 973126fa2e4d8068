// Stream families (Haramoto & Suzuki, arXiv 2512.00093, Sec. 1: unit k starts
// at state s_{kJ}) computed by prefix doubling with the exact jump of Sec. 3:
//
//   out[0] = base;  for b = 0, 1, ...:  out[2^b + k] = f^(2^b delta)(out[k]),
//                                        k < min(2^b, n - 2^b),
//
// with f^(2^b delta) applied as x P_b(A), P_b = t^(2^b delta) mod phi, and
// c stepped by the closed form.  Bit-identical to n independent jumps (the
// jumps form a group: f^a o f^b = f^(a+b)), at one 97x97 application per
// stream instead of one polynomial power per stream.
//
// The polynomials P_b form one dependent chain (P_{b+1} = P_b^2), so they
// are computed by one workgroup cooperatively in LDS; small rounds apply
// them with one workgroup per stream (latency), large rounds with one lane per
// stream (throughput) and the coefficients read as wave-uniform scalars.
#include <map>
#include <mutex>
#include <utility>

#include "common.hpp"
#include "internal.hpp"
#include "jump_dev.hpp"

namespace ranmar {

constexpr int kPolyThreads = 256;
constexpr int kMaxRounds = 64;

// a (97 coefficients, padded with 96 zeros on each side in `pad`) is squared
// or multiplied by t in place, cooperatively by kPolyThreads threads.
__device__ void wg_square(uint32_t* pad, uint32_t* prod) {
  const int k = threadIdx.x;
  const uint32_t* a = pad + 96;
  if (k < 193) {
    // c_k = sum_i a_i a_{k-i}; pad supplies the zeros for k-i outside [0,96].
    uint32_t s0 = 0, s1 = 0;
    for (int i = 0; i < 96; i += 2) {
      s0 = mad24(a[i], pad[96 + k - i], s0);
      s1 = mad24(a[i + 1], pad[95 + k - i], s1);
    }
    s0 = mad24(a[96], pad[k], s0);
    prod[k] = s0 + s1;
  }
  __syncthreads();
  const uint32_t v = k < 97 ? fold_phi(prod, k) : 0u;
  __syncthreads();
  if (k < 97) pad[96 + k] = v & kMask;
  __syncthreads();
}

__device__ void wg_mul_t(uint32_t* pad) {
  const int k = threadIdx.x;
  const uint32_t top = pad[96 + 96];
  uint32_t v = 0;
  if (k < 97) v = (k == 0) ? top : pad[96 + k - 1];
  if (k == 64) v -= top;
  __syncthreads();
  if (k < 97) pad[96 + k] = v & kMask;
  __syncthreads();
}

// Ptab[b] = t^(2^b * delta) mod phi for b < nb (one workgroup).
__global__ __launch_bounds__(kPolyThreads) void k_family_polys(uint64_t dlo, uint64_t dhi, int nb,
                                                              uint32_t* __restrict__ Ptab) {
  __shared__ uint32_t pad[96 + 97 + 96];
  __shared__ uint32_t prod[193];
  for (int i = threadIdx.x; i < 96 + 97 + 96; i += blockDim.x) pad[i] = (i == 96) ? 1u : 0u;
  __syncthreads();
  int top = 127;
  while (top >= 0 && !((top >= 64 ? (dhi >> (top - 64)) : (dlo >> top)) & 1)) --top;
  for (int b = top; b >= 0; --b) {
    wg_square(pad, prod);
    if ((b >= 64 ? (dhi >> (b - 64)) : (dlo >> b)) & 1) wg_mul_t(pad);
  }
  for (int r = 0; r < nb; ++r) {
    if (r > 0) wg_square(pad, prod);
    for (int i = threadIdx.x; i < 97; i += blockDim.x) Ptab[r * 97 + i] = pad[96 + i];
    __syncthreads();
  }
}

// Round with one lane per destination stream: out[dst0 + k] = out[k] jumped.
__global__ __launch_bounds__(64, 2) void k_family_apply_lane(uint32_t* __restrict__ out,
                                                            const uint32_t* __restrict__ P, uint64_t cnt,
                                                            uint64_t dst0, uint32_t jmod) {
  const uint64_t k = (uint64_t)blockIdx.x * 64u + threadIdx.x;
  if (k >= cnt) return;
  const uint32_t* src = out + k * kWords;
  uint32_t u[97], v[97];
#pragma unroll
  for (int i = 0; i < 97; ++i) u[i] = src[i];
  const uint32_t c = src[97];
  horner_apply(u, P, 1, v);
  uint32_t* dst = out + (dst0 + k) * kWords;
#pragma unroll
  for (int i = 0; i < 97; ++i) dst[i] = v[i] & kMask;
  dst[97] = c_jump(c, jmod);
}

// Round with one workgroup per destination stream (small rounds): the new
// window is the Hankel product W'[l] = sum_i b_i X[i+l] with X the window
// extended by 96 steps of the recurrence.
__global__ __launch_bounds__(128) void k_family_apply_wg(uint32_t* __restrict__ out,
                                                        const uint32_t* __restrict__ P, uint64_t dst0,
                                                        uint32_t jmod) {
  __shared__ uint32_t X[193];
  __shared__ uint32_t B[97];
  const uint64_t k = blockIdx.x;
  const int t = threadIdx.x;
  const uint32_t* src = out + k * kWords;
  if (t < 97) {
    X[t] = src[t];
    B[t] = P[t];
  }
  __syncthreads();
  // x_{97+j} = x_j - x_{j+64}: 33 independent terms per step.
  for (int j0 = 0; j0 < 96; j0 += 33) {
    const int j = j0 + t;
    if (t < 33 && j < 96) X[97 + j] = X[j] - X[j + 64];
    __syncthreads();
  }
  if (t < 97) {
    uint32_t s0 = 0, s1 = 0;
    for (int i = 0; i < 96; i += 2) {
      s0 = mad24(B[i], X[i + t], s0);
      s1 = mad24(B[i + 1], X[i + 1 + t], s1);
    }
    s0 = mad24(B[96], X[96 + t], s0);
    uint32_t* dst = out + (dst0 + k) * kWords;
    dst[t] = (s0 + s1) & kMask;
    if (t == 0) dst[97] = c_jump(src[97], jmod);
  }
}

__global__ void k_copy_state(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  const int t = threadIdx.x;
  if (t < 97) dst[t] = src[t] & kMask;
  if (t == 97) dst[97] = src[97];
}

// Library-owned tables of the doubling polynomials, one per (device, stream):
// calls on one stream are ordered, so a table is never shared by two calls
// that may run at the same time.
static uint32_t* family_table(hipStream_t st) {
  static std::mutex mu;
  static std::map<std::pair<int, uintptr_t>, uint32_t*> tabs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  uint32_t*& t = tabs[{dev, (uintptr_t)st}];
  if (!t) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(uint32_t) * 97 * kMaxRounds) != hipSuccess) return nullptr;
    t = (uint32_t*)p;
  }
  return t;
}

hipError_t launch_family(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st) {
  if (!n) return hipSuccess;
  if (base != out) {
    hipLaunchKernelGGL(k_copy_state, dim3(1), dim3(128), 0, st, base, out);
  }
  int nb = 0;
  while (nb < 64 && (1ull << nb) < n) ++nb;
  if (nb == 0) return hipGetLastError();
  uint32_t* tab = family_table(st);
  if (!tab) return hipErrorOutOfMemory;
  hipLaunchKernelGGL(k_family_polys, dim3(1), dim3(kPolyThreads), 0, st, delta.lo, delta.hi, nb, tab);
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  const uint64_t dmod = (uint64_t)(D % kMod);
  uint64_t pow2 = 1;  // 2^b mod m
  for (int b = 0; b < nb; ++b) {
    const uint64_t half = 1ull << b;
    const uint64_t cnt = (n - half < half) ? n - half : half;
    const uint32_t jmod = (uint32_t)((dmod * pow2) % kMod);  // (2^b delta) mod m, exact
    pow2 = (pow2 * 2) % kMod;
    const uint32_t* P = tab + 97 * b;
    if (cnt <= 2048)
      hipLaunchKernelGGL(k_family_apply_wg, dim3((unsigned)cnt), dim3(128), 0, st, out, P, half, jmod);
    else
      hipLaunchKernelGGL(k_family_apply_lane, dim3((unsigned)((cnt + 63) / 64)), dim3(64), 0, st, out, P, cnt,
                         half, jmod);
  }
  return hipGetLastError();
}

}  // namespace ranmar
