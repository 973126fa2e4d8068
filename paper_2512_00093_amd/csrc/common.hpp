// Shared definitions of the RANMAR library (device and host side).
//
// Parameters of the generator (Haramoto & Suzuki, arXiv 2512.00093, Sec. 2):
// lags (r, s) = (97, 33), precision e = 24, M = 2^24, m = 2^24 - 3,
// d = 7654321 / 2^24, c = 362436 / 2^24.  In integer form (Sec. 3) every
// word of the lagged Fibonacci part lives in Z/2^24 and the arithmetic part is
// the numerator c' in [0, m).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ranmar.h"

namespace ranmar {

constexpr int kR = 97;                 // long lag, degree of phi
constexpr int kS = 33;                 // short lag
constexpr int kRS = kR - kS;           // 64: phi = t^97 + t^64 - 1
constexpr uint32_t kMask = 0xFFFFFFu;  // Z/2^24
constexpr uint32_t kMod = 16777213u;   // m
constexpr uint32_t kD = 7654321u;      // d'
constexpr uint32_t kC0 = 362436u;      // c'_0
constexpr uint32_t kWords = 98;        // words per ranmar_state record
constexpr uint32_t kInvalidC = 0xFFFFFFFFu;  // c of a record made from a bad seed

// Device memory seen through the global address space.  A pointer rebuilt
// from a 64-bit integer (the batch descriptors) is generic to the compiler,
// and generic ("flat") stores also count against the LDS wait counter: a loop
// that waits for an LDS permute would then wait for its own stores as well.
// Only for pointers into device memory (never LDS).
typedef __attribute__((address_space(1))) uint32_t gu32;
__device__ __forceinline__ gu32* gptr(void* p) { return (gu32*)p; }

// (m - (k d' mod m)): adding this mod m steps c forward by k draws.
constexpr uint32_t c_step(uint64_t k) { return (uint32_t)(kMod - (k * kD) % kMod) % kMod; }

static_assert(sizeof(ranmar_state) == 392, "state record is 98 packed words");
static_assert(sizeof(ranmar_u128) == 16, "u128 is two 64-bit limbs");

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// a*b + c with 24-bit operands (the low 24 bits of a and b are used), mod 2^32.
// Emitted as a single full-rate v_mad_u32_u24: the compiler's own lowering
// drops the operand masks (only the low 24 bits of the sums are demanded) and
// then falls back to the quarter-rate 32-bit multiply.
#if defined(__HIP_DEVICE_COMPILE__)
extern "C" __device__ uint32_t ranmar_llvm_mul_u24(uint32_t, uint32_t) __asm("llvm.amdgcn.mul.u24");
extern "C" __device__ uint32_t ranmar_llvm_mulhi_u24(uint32_t, uint32_t) __asm("llvm.amdgcn.mulhi.u24");
#endif

__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
#else
  return (a & kMask) * (b & kMask) + c;
#endif
}

__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ranmar_llvm_mul_u24(a, b);
#else
  return (a & kMask) * (b & kMask);
#endif
}

__device__ __forceinline__ uint32_t mulhi24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ranmar_llvm_mulhi_u24(a, b);
#else
  return (uint32_t)(((uint64_t)(a & kMask) * (b & kMask)) >> 32);
#endif
}

// c + step mod m for c < m, step < m: the smaller of (c+step) and (c+step-m)
// taken as unsigned is the reduced value.
__device__ __forceinline__ uint32_t c_add(uint32_t c, uint32_t step) {
  uint32_t t = c + step;
  uint32_t u = t - kMod;
  return t < u ? t : u;
}

// J mod m for J = (j3:j2:j1:j0); 2^32 = 768 (mod m).
__device__ __forceinline__ uint32_t u128_mod_m(uint32_t j0, uint32_t j1, uint32_t j2, uint32_t j3) {
  uint64_t r = j3 % kMod;
  r = (r * 768u + j2) % kMod;
  r = (r * 768u + j1) % kMod;
  r = (r * 768u + j0) % kMod;
  return (uint32_t)r;
}

// c'_J = (c' - (J mod m) d') mod m   (closed form of the arithmetic part)
__device__ __forceinline__ uint32_t c_jump(uint32_t c, uint32_t jmod) {
  uint64_t sub = ((uint64_t)jmod * kD) % kMod;
  return (uint32_t)(((uint64_t)c + kMod - sub) % kMod);
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    int w = __shfl_xor(v, o, 64);
    v = v > w ? v : w;
  }
  return v;
}

}  // namespace ranmar
