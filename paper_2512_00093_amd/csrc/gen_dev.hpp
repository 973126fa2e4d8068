// Device-side generation (Haramoto & Suzuki, arXiv 2512.00093, Algorithm 2)
// by the 32 lanes of a half-wave; shared by the bulk generator and the
// persistent batch kernel.
//
// With the window of the newest 97 words, the next 33 words x_{n+1..n+33} are
// independent (x_t = x_{t-97} - x_{t-33}), so a block of 32 is computed in
// one step, lane l producing draw 32q + l + 1 of block q.  Both lags are
// 1 mod 32 (97 = 3*32 + 1, 33 = 32 + 1), so with blocks aligned at
// T = 98 + 32q the operands of lane l are lane l-1 of earlier blocks.  Each
// lane therefore keeps the "shifted" blocks
//     s97 = x_{T+l-97},  s65 = x_{T+l-65},  s33 = x_{T+l-33}
// and a block step is: v = s97 - s33 (the new word x_{T+l}); then s97 <- s65,
// s65 <- s33, s33 <- v shifted up one lane, lane 0 taking the previous
// block's last word (kept in `rprev`).  The shift is one ds_bpermute.
//
// The arithmetic part: lane l keeps c_{32q+l+1} and steps it by 32 draws per
// block ((c - 32 d') mod m).  Output k = (x - c) mod 2^24 (Algorithm 2), as
// uint32 or as the float k * 2^-24 (exact).  Each half-wave stores one
// 128-byte row segment per block: fully coalesced, no staging.
#pragma once

#include "common.hpp"

namespace ranmar {

// Runtime-format variant of the output stage (FMT_RUNTIME): both encodings
// are formed and the word for the stream's format is stored, so two half-waves
// of one wave may write different formats without diverging.
constexpr int FMT_RUNTIME = 2;

template <int FMT, bool NT>
__device__ __forceinline__ void emit(void* row, uint64_t idx, uint32_t k, bool is_f32) {
  uint32_t w;
  if (FMT == RANMAR_F32) {
    w = __float_as_uint((float)k * 0x1p-24f);
  } else if (FMT == RANMAR_U24) {
    w = k;
  } else {
    const uint32_t fw = __float_as_uint((float)k * 0x1p-24f);
    w = is_f32 ? fw : k;
  }
  uint32_t* p = (uint32_t*)row + idx;
  if (NT)
    __builtin_nontemporal_store(w, p);
  else
    *p = w;
}

// `count` draws of one stream by the 32 lanes of a half-wave (l = lane within
// the half, lane = lane within the wave).  W: the stream's state record;
// dst: where the state after the draws goes (may equal W; nullptr: nowhere);
// row: the stream's first output element.  All lanes of the half must call it
// with the same arguments; the other half may run a different stream.
template <int FMT, bool NT>
__device__ __forceinline__ void gen_stream32(uint32_t l, uint32_t lane, const uint32_t* W, uint32_t* dst,
                                             uint64_t count, bool is_f32, void* out_row) {
  uint32_t s97 = W[l], s65 = W[32 + l], s33 = W[64 + l];
  uint32_t rprev = W[96];  // x_{T-1} for lane 0 of the first block
  const uint32_t c0 = W[97];

  if (count == 0) {
    if (dst && dst != W) {
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
  char* row = (char*)out_row + (uint64_t)l * 4u;

  uint64_t q = 0;
#pragma unroll 6
  for (; q + 1 < nblk; ++q) {
    const uint32_t v = s97 - s33;
    emit<FMT, NT>(row, q * 32u, (v - c) & kMask, is_f32);
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
  if (l < rr) emit<FMT, NT>(row, q * 32u, (v - c) & kMask, is_f32);

  if (dst) {
    // The new window x_{count+1..count+97} is covered by what the lanes hold:
    // s97 -> slot l-rr (l >= rr), s65 -> 32+l-rr, s33 -> 64+l-rr,
    // lane 0's rprev -> 96-rr, v -> 97+l-rr (l < rr); c_count sits in lane rr-1.
    if (l >= rr) dst[l - rr] = s97 & kMask;
    dst[32 + l - rr] = s65 & kMask;
    dst[64 + l - rr] = s33 & kMask;
    if (lead) dst[96 - rr] = rprev & kMask;
    if (l < rr) dst[97 + l - rr] = v & kMask;
    if (l == rr - 1) dst[97] = c;
  }
}

}  // namespace ranmar
