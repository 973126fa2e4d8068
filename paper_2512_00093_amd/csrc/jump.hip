// Jump-ahead kernels: seeding (Appendix A), t^J mod phi (Sec. 3.1), Horner
// application (Sec. 3.1) and the closed-form jump of c (Sec. 3.2).
//
// One request per lane, 64 requests per workgroup (one wave): the polynomial
// lives in 97 VGPRs, the squaring scratch in 96 more, so the kernels run at
// two waves per SIMD with no spills.  During the Horner step the jump
// polynomial is parked in the request's own 392-byte state record (the state
// words having been loaded into registers first), so no workspace is needed.
#include "common.hpp"
#include "internal.hpp"
#include "jump_dev.hpp"
#include "seed_dev.hpp"

namespace ranmar {

// Seeds only: d_out[r] = state of seeds[r] at offset 0.
__global__ __launch_bounds__(64) void k_seed(const int32_t* __restrict__ seeds, uint64_t n,
                                             uint32_t* __restrict__ out) {
  const uint64_t r = (uint64_t)blockIdx.x * 64u + threadIdx.x;
  if (r >= n) return;
  uint32_t* slot = out + r * kWords;
  if (!seed_state(seeds[r], slot)) {
    for (int k = 0; k < 97; ++k) slot[k] = 0;
    slot[97] = kInvalidC;
  }
}

__device__ __forceinline__ void load_j(const ranmar_u128* J, uint64_t r, bool active, uint32_t& j0, uint32_t& j1,
                                       uint32_t& j2, uint32_t& j3) {
  j0 = j1 = j2 = j3 = 0;
  if (active && J) {
    const uint64_t lo = J[r].lo, hi = J[r].hi;
    j0 = (uint32_t)lo;
    j1 = (uint32_t)(lo >> 32);
    j2 = (uint32_t)hi;
    j3 = (uint32_t)(hi >> 32);
  }
}

// P_J only (the quantity of the paper's Table 2).
__global__ __launch_bounds__(64, 2) void k_jump_poly(const ranmar_u128* __restrict__ J, uint64_t n,
                                                    uint32_t* __restrict__ P) {
  const uint64_t r = (uint64_t)blockIdx.x * 64u + threadIdx.x;
  const bool active = r < n;
  uint32_t j0, j1, j2, j3;
  load_j(J, r, active, j0, j1, j2, j3);
  uint32_t a[97];
  xpow_lane(j0, j1, j2, j3, a);
  if (active) {
    uint32_t* dst = P + r * 97;
#pragma unroll
    for (int k = 0; k < 97; ++k) dst[k] = a[k] & kMask;
  }
}

// x <- x P(A) with P given; c untouched.
__global__ __launch_bounds__(64, 2) void k_apply_poly(uint32_t* __restrict__ states,
                                                     const uint32_t* __restrict__ P, uint64_t n) {
  const uint64_t r = (uint64_t)blockIdx.x * 64u + threadIdx.x;
  if (r >= n) return;
  uint32_t* slot = states + r * kWords;
  uint32_t u[97], v[97];
#pragma unroll
  for (int k = 0; k < 97; ++k) u[k] = slot[k];
  horner_apply(u, P + r * 97, 1, v);
#pragma unroll
  for (int k = 0; k < 97; ++k) slot[k] = v[k] & kMask;
}

// In-place f^J on state records; with SEED the record is first initialised
// from seeds[r].
template <bool SEED>
__global__ __launch_bounds__(64, 2) void k_jump(uint32_t* __restrict__ states, const int32_t* __restrict__ seeds,
                                               const ranmar_u128* __restrict__ J, uint64_t n) {
  const uint64_t r = (uint64_t)blockIdx.x * 64u + threadIdx.x;
  const bool active = r < n;
  uint32_t* slot = states + (active ? r : 0) * kWords;
  bool valid = active;
  if (SEED && active) {
    valid = seed_state(seeds[r], slot);
    if (!valid) {
      for (int k = 0; k < 97; ++k) slot[k] = 0;
      slot[97] = kInvalidC;
    }
  }
  uint32_t j0, j1, j2, j3;
  load_j(J, r, valid, j0, j1, j2, j3);
  jump_record_lane(slot, valid, j0, j1, j2, j3);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned grid64(uint64_t n) { return (unsigned)((n + 63) / 64); }

hipError_t launch_seed(const int32_t* seeds, uint64_t n, uint32_t* out, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_seed, dim3(grid64(n)), dim3(64), 0, st, seeds, n, out);
  return hipGetLastError();
}

hipError_t launch_jump_poly(const ranmar_u128* J, uint64_t n, uint32_t* P, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_jump_poly, dim3(grid64(n)), dim3(64), 0, st, J, n, P);
  return hipGetLastError();
}

hipError_t launch_apply_poly(uint32_t* states, const uint32_t* P, uint64_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_apply_poly, dim3(grid64(n)), dim3(64), 0, st, states, P, n);
  return hipGetLastError();
}

hipError_t launch_jump(uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  if (seeds)
    hipLaunchKernelGGL(k_jump<true>, dim3(grid64(n)), dim3(64), 0, st, states, seeds, J, n);
  else
    hipLaunchKernelGGL(k_jump<false>, dim3(grid64(n)), dim3(64), 0, st, states, seeds, J, n);
  return hipGetLastError();
}

}  // namespace ranmar
