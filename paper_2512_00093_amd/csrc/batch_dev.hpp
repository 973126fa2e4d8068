// Device side of the batched executor: one persistent kernel runs requests of
// uneven size (seed, offset, count) through seeding (Appendix A), the exact
// jump (Sec. 3) and generation (Algorithm 2).
//
// A request is cut into chunks of L draws.  Chunk q starts at
// offset + q L, obtained from the request's start state by one application of
// the precomputed P_{qL} = t^(qL) mod phi (Sec. 3.1) and the closed-form c
// jump (Sec. 3.2): the jumps compose exactly (f^a o f^b = f^(a+b)), so every
// chunk's draws are exactly those of the request's single stream.
//
// Work items, taken in order from an atomic counter by one-wave workgroups:
//   [0, n_jg)           jump groups: 64 requests, one per lane (seed + jump);
//   [n_jg, n_jg + n_cg) chunk pairs: each half-wave places one chunk start
//                       (the Hankel product of P_{qL} with the request's
//                       window extended by 96 steps, in LDS) and generates the
//                       chunk's draws.
// A chunk group waits for the flag of each of its requests' jump groups
// (flag == run epoch, so flags never need clearing).  All jump groups precede
// all chunk groups in the queue, so the group a chunk waits for has already
// been taken by a running wave; the wait is still bounded, and a wait that
// runs out sets the host-visible error word instead of hanging.
#pragma once

#include "common.hpp"
#include "gen_dev.hpp"
#include "jump_dev.hpp"
#include "seed_dev.hpp"

namespace ranmar {

struct BHeader {        // 64 bytes
  uint32_t n_req, n_jg, n_chunks, n_cg;
  uint32_t epoch, L, pad0, pad1;
  uint64_t chunk_off;   // byte offset of the chunk table from the header
  uint64_t pad[3];
};
struct BReq {           // 48 bytes
  int32_t seed;
  uint32_t fmt;
  uint64_t off_lo, off_hi;
  uint64_t count;
  uint64_t out;
  uint64_t state;
};
struct BChunk {         // 16 bytes
  uint32_t req, q, draws, last;
};
static_assert(sizeof(BHeader) == 64 && sizeof(BReq) == 48 && sizeof(BChunk) == 16, "descriptor layout");

constexpr uint32_t kSpinLimit = 1u << 22;  // x ~100 cycles per sleep: about 0.2 s

// Descriptor access: either tables in device memory, or a single request
// passed by value (the one-launch-per-request path).
struct TableDesc {
  const uint8_t* desc;
  __device__ __forceinline__ BHeader header() const { return *(const BHeader*)desc; }
  __device__ __forceinline__ BReq req(uint32_t r) const { return ((const BReq*)(desc + 64))[r]; }
  __device__ __forceinline__ BChunk chunk(const BHeader& h, uint32_t j) const {
    return ((const BChunk*)(desc + h.chunk_off))[j];
  }
};
struct SingleDesc {
  BReq r0;
  uint32_t L, epoch;
  __device__ __forceinline__ BHeader header() const {
    BHeader h{};
    const uint64_t nq = (r0.count + L - 1) / L;
    h.n_req = 1;
    h.n_jg = 1;
    h.n_chunks = (uint32_t)nq;
    h.n_cg = (uint32_t)((nq + 1) / 2);
    h.epoch = epoch;
    h.L = L;
    return h;
  }
  __device__ __forceinline__ BReq req(uint32_t) const { return r0; }
  __device__ __forceinline__ BChunk chunk(const BHeader& h, uint32_t j) const {
    BChunk c;
    c.req = 0;
    c.q = j;
    const uint64_t first = (uint64_t)j * h.L;
    c.draws = (uint32_t)((r0.count - first) < h.L ? (r0.count - first) : h.L);
    c.last = (j + 1 == h.n_chunks) ? 1u : 0u;
    return c;
  }
};

struct BatchBuffers {
  uint32_t* req_states;    // 98 words per request
  uint32_t* done;          // one flag per jump group
  const uint32_t* ptab;    // 97 words per q: P_{qL}
  uint32_t* queue;         // [0] next item, [1] finished workgroups
  int* err;                // host-visible error word
};

template <class Desc>
__device__ __forceinline__ void batch_jump_group(const Desc& D, const BHeader& h, const BatchBuffers& B, uint32_t g) {
  const uint32_t lane = threadIdx.x;
  const uint32_t r = g * 64u + lane;
  const bool active = r < h.n_req;
  BReq q{};
  if (active) q = D.req(r);
  // A request with no draws but a state output is jumped directly in the
  // caller's state record.
  uint32_t* slot = (active && q.count == 0 && q.state) ? (uint32_t*)q.state : B.req_states + (uint64_t)r * kWords;
  bool valid = false;
  if (active) {
    valid = seed_state(q.seed, slot);
    if (!valid) {
      for (int k = 0; k < 97; ++k) slot[k] = 0;
      slot[97] = kInvalidC;
    }
  }
  const uint32_t j0 = valid ? (uint32_t)q.off_lo : 0u, j1 = valid ? (uint32_t)(q.off_lo >> 32) : 0u;
  const uint32_t j2 = valid ? (uint32_t)q.off_hi : 0u, j3 = valid ? (uint32_t)(q.off_hi >> 32) : 0u;
  jump_record_lane(slot, valid, j0, j1, j2, j3);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  // Every lane stores the same value: no lane-conditional branch here (see
  // batch_persistent).
  __hip_atomic_store(&B.done[g], h.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS per half-wave: the extended window X (193 words), the coefficients of
// P_{qL} (97) and the chunk's start state (98).
constexpr int kHalfLds = 193 + 97 + 98;

template <class Desc>
__device__ __forceinline__ void batch_chunk_pair(const Desc& D, const BHeader& h, const BatchBuffers& B, uint32_t cp,
                                                 uint32_t* lds) {
  const uint32_t lane = threadIdx.x;
  const uint32_t half = lane >> 5, l = lane & 31u;
  const uint32_t j = 2u * cp + half;
  const bool active = j < h.n_chunks;
  uint32_t* X = lds + half * kHalfLds;
  uint32_t* Bc = X + 193;
  uint32_t* Wn = Bc + 97;
  BChunk ch{};
  BReq rq{};
  if (active) {
    ch = D.chunk(h, j);
    rq = D.req(ch.req);
    uint32_t it = 0;
    while (__hip_atomic_load(&B.done[ch.req >> 6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != h.epoch) {
      __builtin_amdgcn_s_sleep(2);
      if (++it > kSpinLimit) {
        __hip_atomic_store(B.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        break;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  uint32_t c0 = 0;
  if (active) {
    const uint32_t* src = B.req_states + (uint64_t)ch.req * kWords;
    const uint32_t* P = B.ptab + (uint64_t)ch.q * 97u;
    for (uint32_t k = l; k < 97; k += 32) {
      X[k] = src[k];
      Bc[k] = P[k];
    }
    c0 = src[97];
  }
  __syncthreads();
  // Extend the window: x_{97+i} = x_i - x_{i+64}, 32 terms per step.
  for (uint32_t s0 = 0; s0 < 96; s0 += 32) {
    if (active) X[97 + s0 + l] = X[s0 + l] - X[s0 + l + 64];
    __syncthreads();
  }
  // New window W'[o] = sum_i b_i X[i + o] for o = l, l+32, l+64 (+96 on lane 0).
  if (active) {
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 4
    for (int i = 0; i < 97; ++i) {
      const uint32_t b = Bc[i];
      a0 = mad24(b, X[i + l], a0);
      a1 = mad24(b, X[i + l + 32], a1);
      a2 = mad24(b, X[i + l + 64], a2);
      if (l == 0) a3 = mad24(b, X[i + 96], a3);
    }
    Wn[l] = a0 & kMask;
    Wn[l + 32] = a1 & kMask;
    Wn[l + 64] = a2 & kMask;
    if (l == 0) {
      Wn[96] = a3 & kMask;
      Wn[97] = c_jump(c0, (uint32_t)(((uint64_t)ch.q * h.L) % kMod));
    }
  }
  __syncthreads();
  if (active) {
    uint32_t* dst = (ch.last && rq.state) ? (uint32_t*)rq.state : nullptr;
    gen_stream32<FMT_RUNTIME, true>(l, lane, Wn, dst, ch.draws, rq.fmt == RANMAR_F32,
                                    (char*)rq.out + (uint64_t)ch.q * h.L * 4u);
  }
  __syncthreads();
}

template <class Desc>
__device__ __forceinline__ void batch_persistent(const Desc& D, const BatchBuffers& B) {
  const BHeader h = D.header();
  const uint32_t lane = threadIdx.x;
  __shared__ uint32_t lds[2 * kHalfLds];
  for (;;) {
    // Dequeue without a lane-conditional branch: every lane executes the
    // atomic, lane 0 adding 1 and the others 0, and lane 0's result is taken.
    // (With `if (lane == 0) item = atomicAdd(...)` only lane 0 holds the item,
    // and the compiler may merge that branch with other lane-0 branches of
    // the loop body so that lanes 1..63 re-enter the body on a stale item.)
    const uint32_t got = atomicAdd(&B.queue[0], lane == 0 ? 1u : 0u);
    const uint32_t item = __builtin_amdgcn_readfirstlane(got);
    if (item < h.n_jg)
      batch_jump_group(D, h, B, item);
    else if (item < h.n_jg + h.n_cg)
      batch_chunk_pair(D, h, B, item - h.n_jg, lds);
    else
      break;
  }
  // The last workgroup out resets the counters for the next launch.
  if (lane == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t f = atomicAdd(&B.queue[1], 1u);
    if (f == gridDim.x - 1) {
      atomicExch(&B.queue[0], 0u);
      atomicExch(&B.queue[1], 0u);
    }
  }
}

}  // namespace ranmar
