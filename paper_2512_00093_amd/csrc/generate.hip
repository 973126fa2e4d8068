// Bulk generation (Haramoto & Suzuki, arXiv 2512.00093, Algorithm 2) over many
// independent streams.
//
// Mapping: 32 lanes per stream, two streams per wave64.  With the window of
// the newest 97 words, the next 33 words x_{n+1..n+33} are independent
// (x_{t} = x_{t-97} - x_{t-33}), so a block of 32 is computed in one step,
// lane l producing draw 32q + l + 1 of block q.  Both lags are 1 mod 32
// (97 = 3*32 + 1, 33 = 32 + 1), so with blocks aligned at T = 98 + 32q the
// operands of lane l are lane l-1 of earlier blocks.  Each lane therefore
// keeps the "shifted" blocks
//     s97 = x_{T+l-97},  s65 = x_{T+l-65},  s33 = x_{T+l-33}
// and a block step is: v = s97 - s33 (the new word x_{T+l}); then s97 <- s65,
// s65 <- s33, s33 <- v shifted up one lane, lane 0 taking the previous
// block's last word (kept in `rprev`).  The shift is one ds_bpermute.
//
// The arithmetic part: lane l keeps c_{32q+l+1} and steps it by 32 draws
// per block ((c - 32 d') mod m).  Output k = (x - c) mod 2^24 (Algorithm 2),
// as uint32 or as the float k * 2^-24 (exact).  Each half-wave stores one
// 128-byte row segment per block: fully coalesced, no staging.
#include "common.hpp"
#include "internal.hpp"

namespace ranmar {

template <int FMT, bool NT>
__device__ __forceinline__ void emit(void* row, uint64_t idx, uint32_t k) {
  if (FMT == RANMAR_F32) {
    float* p = (float*)row + idx;
    const float f = (float)k * 0x1p-24f;
    if (NT)
      __builtin_nontemporal_store(f, p);
    else
      *p = f;
  } else {
    uint32_t* p = (uint32_t*)row + idx;
    if (NT)
      __builtin_nontemporal_store(k, p);
    else
      *p = k;
  }
}

template <int FMT, bool NT>
__global__ __launch_bounds__(256) void k_gen32(const uint32_t* __restrict__ sin, uint32_t* sout, uint64_t n,
                                               uint64_t count, void* __restrict__ out, uint64_t ld) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t l = lane & 31u;
  const uint64_t s = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 2u + (lane >> 5);
  if (s >= n) return;  // a whole half-wave leaves together; shifts stay inside a half

  const uint32_t* W = sin + s * kWords;
  uint32_t s97 = W[l], s65 = W[32 + l], s33 = W[64 + l];
  uint32_t rprev = W[96];  // x_{T-1} for lane 0 of the first block
  const uint32_t c0 = W[97];

  if (count == 0) {
    if (sout && sout != sin) {
      uint32_t* dst = sout + s * kWords;
      dst[l] = s97 & kMask;
      dst[32 + l] = s65 & kMask;
      dst[64 + l] = s33 & kMask;
      if (l == 0) {
        dst[96] = rprev & kMask;
        dst[97] = c0;
      }
    }
    return;
  }

  uint32_t c = (uint32_t)(((uint64_t)c0 + (uint64_t)(l + 1) * (kMod - kD)) % kMod);  // c_{l+1}
  constexpr uint32_t kStep = c_step(32);
  const int src = (int)(((lane & 32u) | ((l - 1u) & 31u)) << 2);
  const bool lead = (l == 0);
  const uint64_t nblk = (count + 31) / 32;
  char* row = (char*)out + (s * ld + l) * 4u;

  uint64_t q = 0;
#pragma unroll 6
  for (; q + 1 < nblk; ++q) {
    const uint32_t v = s97 - s33;
    emit<FMT, NT>(row, q * 32u, (v - c) & kMask);
    c = c_add(c, kStep);
    const uint32_t rot = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)v);
    const uint32_t nx = lead ? rprev : rot;
    rprev = rot;
    s97 = s65;
    s65 = s33;
    s33 = nx;
  }

  // Last (possibly partial) block: rr = count - 32q draws in 1..32.
  const uint32_t v = s97 - s33;
  const uint32_t rr = (uint32_t)(count - 32u * q);
  if (l < rr) emit<FMT, NT>(row, q * 32u, (v - c) & kMask);

  if (sout) {
    // The new window x_{count+1..count+97} is covered by what the lanes hold:
    // s97 -> slot l-rr (l >= rr), s65 -> 32+l-rr, s33 -> 64+l-rr,
    // lane 0's rprev -> 96-rr, v -> 97+l-rr (l < rr); c_count sits in lane rr-1.
    uint32_t* dst = sout + s * kWords;
    if (l >= rr) dst[l - rr] = s97 & kMask;
    dst[32 + l - rr] = s65 & kMask;
    dst[64 + l - rr] = s33 & kMask;
    if (lead) dst[96 - rr] = rprev & kMask;
    if (l < rr) dst[97 + l - rr] = v & kMask;
    if (l == rr - 1) dst[97] = c;
  }
}

const char* gen_variant_name(int v) {
  switch (v) {
    case GEN_LANES32: return "lanes32";
    case GEN_LANES32_NT: return "lanes32_nt";
    default: return "?";
  }
}

template <int FMT>
static hipError_t launch_fmt(int variant, const uint32_t* sin, uint32_t* sout, uint64_t n, uint64_t count, void* out,
                             uint64_t ld, hipStream_t st) {
  const unsigned wg = 256;
  const uint64_t per_wg = wg / 32;
  const dim3 grid((unsigned)((n + per_wg - 1) / per_wg));
  switch (variant) {
    case GEN_LANES32_NT:
      hipLaunchKernelGGL((k_gen32<FMT, true>), grid, dim3(wg), 0, st, sin, sout, n, count, out, ld);
      break;
    default:
      hipLaunchKernelGGL((k_gen32<FMT, false>), grid, dim3(wg), 0, st, sin, sout, n, count, out, ld);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_generate(int variant, const uint32_t* sin, uint32_t* sout, uint64_t n, uint64_t count, int fmt,
                           void* out, uint64_t ld, hipStream_t st) {
  if (!n) return hipSuccess;
  if (fmt == RANMAR_F32) return launch_fmt<RANMAR_F32>(variant, sin, sout, n, count, out, ld, st);
  return launch_fmt<RANMAR_U24>(variant, sin, sout, n, count, out, ld, st);
}

}  // namespace ranmar
