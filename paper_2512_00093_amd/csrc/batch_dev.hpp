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
// Work items, taken in order from an atomic counter by one-wave workgroups
// (jump pairs g at a time when there are many):
//   [0, n_jg)           jump pairs: each half-wave seeds one request and jumps
//                       it to its offset (parallel seeding and the windowed
//                       jump of coop_dev.hpp), then raises the request's flag;
//   [n_jg, n_jg + n_cg) chunk pairs: each half-wave places one chunk start
//                       (P_{qL} applied to the request's start state, in LDS)
//                       and generates the chunk's draws.
// A chunk waits for its request's flag (flag == run epoch, so flags never
// need clearing).  All jump pairs precede all chunk pairs in the queue, so the
// request a chunk waits for has already been taken by a running wave; the wait
// is still bounded, and a wait that runs out sets the host-visible error word
// instead of hanging.
#pragma once

#include "common.hpp"
#include "coop_dev.hpp"
#include "gen_dev.hpp"

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
    h.n_jg = 1;  // one jump pair, its second half idle
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
  uint32_t* done;          // one flag per request, plus one spare written by idle halves
  const uint32_t* ptab;    // 97 words per q: P_{qL}
  const uint32_t* wtab;    // window table T[w][d]
  uint32_t* queue;         // [0] next item, [1] finished workgroups
  int* err;                // host-visible error word
  uint32_t spare;          // index of the spare flag
};

// LDS per half-wave: the extended window X (193 words) and a polynomial (97).
constexpr int kHalfLds = 193 + 97;

template <class Desc>
__device__ __forceinline__ void batch_jump_pair(const Desc& D, const BHeader& h, const BatchBuffers& B, uint32_t p,
                                                uint32_t* lds) {
  const uint32_t lane = threadIdx.x;
  const uint32_t half = lane >> 5, l = lane & 31u;
  const uint32_t r = 2u * p + half;
  const bool active = r < h.n_req;
  uint32_t* X = lds + half * kHalfLds;
  uint32_t* Bp = X + 193;
  BReq q{};
  if (active) q = D.req(r);
  const bool valid = active && seed_half(q.seed, X, l);
  if (!valid) X[l] = X[l + 32] = X[l + 64] = X[97] = 0;
  wave_sync();
  const uint32_t c = X[97];
  const uint32_t j0 = valid ? (uint32_t)q.off_lo : 0u, j1 = valid ? (uint32_t)(q.off_lo >> 32) : 0u;
  const uint32_t j2 = valid ? (uint32_t)q.off_hi : 0u, j3 = valid ? (uint32_t)(q.off_hi >> 32) : 0u;
  jump_half(X, Bp, B.wtab, j0, j1, j2, j3, wave_windows(j0, j1, j2, j3), l);
  // A request with no draws but a state output is written straight to the
  // caller's record.
  uint32_t* slot = (active && q.count == 0 && q.state) ? (uint32_t*)q.state : B.req_states + (uint64_t)r * kWords;
  if (active) {
    slot[l] = valid ? X[l] : 0u;
    slot[l + 32] = valid ? X[l + 32] : 0u;
    slot[l + 64] = valid ? X[l + 64] : 0u;
    if (l == 0) {
      slot[96] = valid ? X[96] : 0u;
      slot[97] = valid ? c_jump(c, u128_mod_m(j0, j1, j2, j3)) : kInvalidC;
    }
  }
  // Only requests with draws have chunks waiting for them.  The release fence
  // writes back this XCD's L2, so it is skipped when no request of the pair
  // has consumers (jump-only batches); the test is wave-uniform.
  if (__any(active && q.count > 0)) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // Every lane of the half stores the same value (idle halves to the spare).
    __hip_atomic_store(&B.done[active ? r : B.spare], h.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  wave_sync();
}

template <class Desc>
__device__ __forceinline__ void batch_chunk_pair(const Desc& D, const BHeader& h, const BatchBuffers& B, uint32_t cp,
                                                 uint32_t* lds) {
  const uint32_t lane = threadIdx.x;
  const uint32_t half = lane >> 5, l = lane & 31u;
  const uint32_t j = 2u * cp + half;
  const bool active = j < h.n_chunks;
  uint32_t* X = lds + half * kHalfLds;
  uint32_t* Bp = X + 193;
  BChunk ch{};
  BReq rq{};
  if (active) {
    ch = D.chunk(h, j);
    rq = D.req(ch.req);
    uint32_t it = 0;
    while (__hip_atomic_load(&B.done[ch.req], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != h.epoch) {
      __builtin_amdgcn_s_sleep(2);
      if (++it > kSpinLimit) {
        __hip_atomic_store(B.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        break;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  // Chunk start: the request's start state times P_{qL}(A), c by qL steps.
  const uint32_t* src = B.req_states + (uint64_t)ch.req * kWords;
  const uint32_t* P = B.ptab + (uint64_t)ch.q * 97u;
  X[l] = active ? src[l] : 0u;
  X[l + 32] = active ? src[l + 32] : 0u;
  X[l + 64] = active ? src[l + 64] : 0u;
  Bp[l] = P[l];
  Bp[l + 32] = P[l + 32];
  Bp[l + 64] = P[l + 64];
  if (l == 0) {
    X[96] = active ? src[96] : 0u;
    Bp[96] = P[96];
  }
  const uint32_t c0 = active ? src[97] : 0u;
  wave_sync();
  apply_half(X, Bp, l);
  if (l == 0) X[97] = c_jump(c0, (uint32_t)(((uint64_t)ch.q * h.L) % kMod));
  wave_sync();
  if (active) {
    uint32_t* dst = (ch.last && rq.state) ? (uint32_t*)rq.state : nullptr;
    gen_stream32<FMT_RUNTIME, true>(l, lane, X, dst, ch.draws, rq.fmt == RANMAR_F32,
                                    (char*)rq.out + (uint64_t)ch.q * h.L * 4u);
  }
  wave_sync();
}

template <class Desc>
__device__ __forceinline__ void batch_persistent(const Desc& D, const BatchBuffers& B) {
  const BHeader h = D.header();
  const uint32_t lane = threadIdx.x;
  __shared__ uint32_t lds[2 * kHalfLds];
  // Jump pairs are taken g at a time when there are many (one queue atomic per
  // g pairs instead of per pair); small batches keep g = 1 for latency.
  uint32_t g = h.n_jg / (2u * gridDim.x);
  g = g < 1u ? 1u : (g > 8u ? 8u : g);
  const uint32_t n_ju = (h.n_jg + g - 1) / g;
  for (;;) {
    // Dequeue without a lane-conditional branch: every lane executes the
    // atomic, lane 0 adding 1 and the others 0, and lane 0's result is taken.
    // (With `if (lane == 0) item = atomicAdd(...)` only lane 0 holds the item,
    // and the compiler may merge that branch with other lane-0 branches of
    // the loop body so that lanes 1..63 re-enter the body on a stale item.)
    const uint32_t got = atomicAdd(&B.queue[0], lane == 0 ? 1u : 0u);
    const uint32_t item = __builtin_amdgcn_readfirstlane(got);
    if (item < n_ju) {
      const uint32_t p1 = (item + 1) * g < h.n_jg ? (item + 1) * g : h.n_jg;
      for (uint32_t p = item * g; p < p1; ++p) batch_jump_pair(D, h, B, p, lds);
    } else if (item < n_ju + h.n_cg) {
      batch_chunk_pair(D, h, B, item - n_ju, lds);
    } else {
      break;
    }
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
