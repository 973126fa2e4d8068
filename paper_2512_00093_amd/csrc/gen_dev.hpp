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

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;

// Output stage.  FMT is RANMAR_U24, RANMAR_F32, RANMAR_U24_F32 (both: k to
// plane 0, the float to plane 1, `plane` elements further on) or FMT_RUNTIME:
// both encodings are formed and the one for the stream's format is stored, so
// two half-waves of one wave may write different formats without diverging.
constexpr int FMT_RUNTIME = 16;

template <int FMT, bool NT>
__device__ __forceinline__ void emit(void* row, uint64_t idx, uint32_t k, bool is_f32, uint64_t plane = 0) {
  gu32* p = gptr(row) + idx;
  const uint32_t fw = __float_as_uint((float)k * 0x1p-24f);
  if (FMT == RANMAR_U24_F32) {
    if (NT) {
      __builtin_nontemporal_store(k, p);
      __builtin_nontemporal_store(fw, p + plane);
    } else {
      p[0] = k;
      p[plane] = fw;
    }
    return;
  }
  const uint32_t w = FMT == RANMAR_F32 ? fw : FMT == RANMAR_U24 ? k : (is_f32 ? fw : k);
  if (NT)
    __builtin_nontemporal_store(w, p);
  else
    *p = w;
}

// A stream's state as the 32 lanes of a half-wave hold it: lane l has words
// l, 32+l, 64+l of the window; every lane has word 96 and c.
struct StreamRegs {
  uint32_t s97, s65, s33, rprev, c0;
};

__device__ __forceinline__ StreamRegs load_stream(const uint32_t* W, uint32_t l) {
  return StreamRegs{W[l], W[32 + l], W[64 + l], W[96], W[97]};
}

// `count` draws of one stream by the 32 lanes of a half-wave (l = lane within
// the half, lane = lane within the wave).  W: the stream's state record;
// dst: where the state after the draws goes (may equal W; nullptr: nowhere);
// row: the stream's first output element.  All lanes of the half must call it
// with the same arguments; the other half may run a different stream.
template <int FMT, bool NT>
__device__ __forceinline__ void gen_regs32(uint32_t l, uint32_t lane, StreamRegs st, const uint32_t* W,
                                           uint32_t* dst, uint64_t count, bool is_f32, void* out_row,
                                           uint64_t plane = 0);

template <int FMT, bool NT>
__device__ __forceinline__ void gen_stream32(uint32_t l, uint32_t lane, const uint32_t* W, uint32_t* dst,
                                             uint64_t count, bool is_f32, void* out_row, uint64_t plane = 0) {
  gen_regs32<FMT, NT>(l, lane, load_stream(W, l), W, dst, count, is_f32, out_row, plane);
}

// The same from a state already in registers (W: its record, compared with
// dst only).
template <int FMT, bool NT>
__device__ __forceinline__ void gen_regs32(uint32_t l, uint32_t lane, StreamRegs st, const uint32_t* W,
                                           uint32_t* dst, uint64_t count, bool is_f32, void* out_row,
                                           uint64_t plane) {
  uint32_t s97 = st.s97, s65 = st.s65, s33 = st.s33;
  uint32_t rprev = st.rprev;  // x_{T-1} for lane 0 of the first block
  const uint32_t c0 = st.c0;

  if (count == 0) {
    if (dst && dst != W) {
      gu32* d = gptr(dst);
      d[l] = s97 & kMask;
      d[32 + l] = s65 & kMask;
      d[64 + l] = s33 & kMask;
      if (l == 0) {
        d[96] = rprev & kMask;
        d[97] = c0;
      }
    }
    return;
  }

  // c_{l+1} = (c_0 - (l+1) d') mod m; (l+1)(m - d') + c_0 < 2^32 for l < 32.
  uint32_t c = (c0 + (l + 1u) * (kMod - kD)) % kMod;
  constexpr uint32_t kStep = c_step(32);
  const int src = (int)(((lane & 32u) | ((l - 1u) & 31u)) << 2);
  const bool lead = (l == 0);
  const uint64_t nblk = (count + 31) / 32;
  char* row = (char*)out_row + (uint64_t)l * 4u;

  // One block step: the new words v = s97 - s33, their draws, and the shifted
  // block that becomes s33 written into s97's register (s97 is dead after v).
  // Three steps with rotated names bring the roles back, so the unrolled loop
  // needs no register moves.
#define RANMAR_GEN_STEP(S97, S33, Q)                                       \
  {                                                                        \
    const uint32_t v_ = S97 - S33;                                         \
    emit<FMT, NT>(row, (Q) * 32u, (v_ - c) & kMask, is_f32, plane);        \
    c = c_add(c, kStep);                                                   \
    const uint32_t rot_ = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)v_); \
    S97 = lead ? rprev : rot_;                                             \
    rprev = rot_;                                                          \
  }
  uint64_t q = 0;
  for (; q + 7 <= nblk; q += 6) {  // six full blocks, none of them the last
    RANMAR_GEN_STEP(s97, s33, q);
    RANMAR_GEN_STEP(s65, s97, q + 1);
    RANMAR_GEN_STEP(s33, s65, q + 2);
    RANMAR_GEN_STEP(s97, s33, q + 3);
    RANMAR_GEN_STEP(s65, s97, q + 4);
    RANMAR_GEN_STEP(s33, s65, q + 5);
  }
  for (; q + 1 < nblk; ++q) {
    RANMAR_GEN_STEP(s97, s33, q);
    const uint32_t t_ = s97;  // restore the (s97, s65, s33) roles
    s97 = s65;
    s65 = s33;
    s33 = t_;
  }
#undef RANMAR_GEN_STEP

  // Last (possibly partial) block: rr = count - 32q draws in 1..32.
  const uint32_t v = s97 - s33;
  const uint32_t rr = (uint32_t)(count - 32u * q);
  if (l < rr) emit<FMT, NT>(row, q * 32u, (v - c) & kMask, is_f32, plane);

  if (dst) {
    // The new window x_{count+1..count+97} is covered by what the lanes hold:
    // s97 -> slot l-rr (l >= rr), s65 -> 32+l-rr, s33 -> 64+l-rr,
    // lane 0's rprev -> 96-rr, v -> 97+l-rr (l < rr); c_count sits in lane rr-1.
    gu32* d = gptr(dst);
    if (l >= rr) d[l - rr] = s97 & kMask;
    d[32 + l - rr] = s65 & kMask;
    d[64 + l - rr] = s33 & kMask;
    if (lead) d[96 - rr] = rprev & kMask;
    if (l < rr) d[97 + l - rr] = v & kMask;
    if (l == rr - 1) d[97] = c;
  }
}

// Same draws as gen_stream32, written four blocks at a time: the 128 outputs of
// four consecutive blocks are transposed through `buf` (128 words of LDS owned
// by this half-wave) so that every lane stores 16 consecutive bytes and the
// half-wave writes 512 contiguous bytes per store.  Requires a 16-byte aligned
// row start.
template <int FMT, bool NT>
__device__ __forceinline__ void gen_stream32_wide(uint32_t l, uint32_t lane, const uint32_t* W, uint32_t* dst,
                                                  uint64_t count, bool is_f32, void* out_row, uint32_t* buf) {
  if (count == 0) {
    gen_stream32<FMT, NT>(l, lane, W, dst, count, is_f32, out_row);
    return;
  }
  uint32_t s97 = W[l], s65 = W[32 + l], s33 = W[64 + l];
  uint32_t rprev = W[96];
  const uint32_t c0 = W[97];
  uint32_t c = (c0 + (l + 1u) * (kMod - kD)) % kMod;
  constexpr uint32_t kStep = c_step(32);
  const int src = (int)(((lane & 32u) | ((l - 1u) & 31u)) << 2);
  const bool lead = (l == 0);
  const uint64_t nblk = (count + 31) / 32;
  const uint64_t nmacro = (nblk - 1) / 4;  // groups of four full blocks before the last block

  auto encode = [&](uint32_t k) -> uint32_t {
    if (FMT == RANMAR_F32) return __float_as_uint((float)k * 0x1p-24f);
    if (FMT == RANMAR_U24) return k;
    return is_f32 ? __float_as_uint((float)k * 0x1p-24f) : k;
  };
  // One block step on roles (s97 = A, s33 = C): returns the encoded draws and
  // leaves the shifted block in A (see gen_stream32).
  auto step = [&](uint32_t& A, uint32_t C) -> uint32_t {
    const uint32_t v = A - C;
    const uint32_t y = encode((v - c) & kMask);
    c = c_add(c, kStep);
    const uint32_t rot = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)v);
    A = lead ? rprev : rot;
    rprev = rot;
    return y;
  };
  gu32x4* row4 = (gu32x4*)out_row;
  // Four blocks (roles (A, B, C) -> (B, C, A)), transposed through LDS and
  // stored as 16 bytes per lane.
  auto macro = [&](uint32_t& A, uint32_t& B, uint32_t& C, uint64_t m) {
    const uint32_t y0 = step(A, C);
    const uint32_t y1 = step(B, A);
    const uint32_t y2 = step(C, B);
    const uint32_t y3 = step(A, C);
    buf[l] = y0;
    buf[32 + l] = y1;
    buf[64 + l] = y2;
    buf[96 + l] = y3;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const u32x4 w4 = ((const u32x4*)buf)[l];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (NT)
      __builtin_nontemporal_store(w4, row4 + m * 32u + l);
    else
      row4[m * 32u + l] = w4;
  };
  uint64_t m = 0;
  for (; m + 3 <= nmacro; m += 3) {  // three macros bring the roles back
    macro(s97, s65, s33, m);
    macro(s65, s33, s97, m + 1);
    macro(s33, s97, s65, m + 2);
  }
  for (; m < nmacro; ++m) {
    macro(s97, s65, s33, m);
    const uint32_t t = s97;
    s97 = s65;
    s65 = s33;
    s33 = t;
  }
  // Remaining full blocks one at a time, then the last block.
  gu32* row = gptr(out_row) + l;
  uint64_t q = nmacro * 4;
  for (; q + 1 < nblk; ++q) {
    const uint32_t y = step(s97, s33);
    if (NT)
      __builtin_nontemporal_store(y, row + q * 32u);
    else
      row[q * 32u] = y;
    const uint32_t t = s97;
    s97 = s65;
    s65 = s33;
    s33 = t;
  }
  const uint32_t v = s97 - s33;
  const uint32_t rr = (uint32_t)(count - 32u * q);
  if (l < rr) {
    const uint32_t y = encode((v - c) & kMask);
    if (NT)
      __builtin_nontemporal_store(y, row + q * 32u);
    else
      row[q * 32u] = y;
  }
  if (dst) {
    gu32* d = gptr(dst);
    if (l >= rr) d[l - rr] = s97 & kMask;
    d[32 + l - rr] = s65 & kMask;
    d[64 + l - rr] = s33 & kMask;
    if (lead) d[96 - rr] = rprev & kMask;
    if (l < rr) d[97 + l - rr] = v & kMask;
    if (l == rr - 1) d[97] = c;
  }
}

}  // namespace ranmar
