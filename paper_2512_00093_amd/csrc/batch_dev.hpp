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
// The work is split into bins (up to 64).  A bin is a contiguous range of
// slices (a slice is a request or an exact part of one: offset + first draw,
// its own seed + jump) and of their chunks, and has its own queue counter on
// its own 256-byte line: one counter shared by the whole grid serialises
// every dequeue at one memory channel.  Workgroup w serves bin w mod n_bins.
// A bin's slices with draws come first, then its slices without (jumps
// only).  Items of a bin, taken in order from its counter by one-wave
// workgroups:
//   [0, n_ju)                   pair items: g jump pairs; each half-wave seeds
//                               one slice with draws and jumps it to its
//                               offset (parallel seeding and the windowed jump
//                               of coop_dev.hpp), then raises its flag;
//   [n_ju, n_ju + n_cg)         chunk pairs: each half-wave places one chunk
//                               start (P_{qL} applied to the slice's start
//                               state, in LDS) and generates the chunk's draws;
//   [.., .. + n_qi)             octet items: gq jump octets; each 8-lane group
//                               seeds and jumps one slice without draws
//                               (nothing waits for these, so they come last).
// A chunk waits for its slice's flag (flag == run epoch, so flags never need
// clearing).  A chunk's slice is in the chunk's own bin and every jump item of
// a bin precedes its chunk items, so the jump a chunk waits for has already
// been taken by a running wave; the wait is still bounded, and a wait that
// runs out sets the host-visible error word instead of hanging.
#pragma once

#include "common.hpp"
#include "coop_dev.hpp"
#include "gen_dev.hpp"

namespace ranmar {

struct BHeader {        // 64 bytes
  uint32_t n_bins, n_workers, epoch, L;  // n_workers: one-wave workgroups launched
  uint64_t req_off;     // byte offset of the table of slices with draws (copied to the device)
  uint64_t chunk_off;   // byte offset of the chunk table (copied to the device)
  uint64_t jo_off;      // byte offset of the table of slices without draws (BJump, read from host memory)
  uint64_t pad[3];
};
struct BBin {           // 256 bytes: the counter alone on its line
  uint32_t ctr;         // next item (0 at launch: the descriptor copy resets it)
  uint32_t s0, ns, nsc; // slices [s0, s0 + ns): the first nsc by pair items, the rest (no draws) by octet items
  uint32_t k0, nk;      // chunks [k0, k0 + nk)
  uint32_t g, n_ju;     // jump pairs (slices with draws) per pair item, pair items
  uint32_t n_cg;        // chunk pairs
  uint32_t gq, n_qi;    // jump octets (slices without draws) per octet item, octet items
  uint32_t a0, na;      // the bin's slices with draws: entries [a0, a0 + na) of their table
  uint32_t b0;          // the bin's slices without draws: entries b0 .. of theirs
  uint32_t pad[50];
};
struct BReq {           // 48 bytes
  int32_t seed;
  uint32_t fmt;
  uint64_t off_lo, off_hi;
  uint64_t count;
  uint64_t out;
  uint64_t state;
};
struct BJump {          // 32 bytes: a slice without draws (no format, count or output)
  int32_t seed;
  uint32_t pad;
  uint64_t off_lo, off_hi;
  uint64_t state;
};
// The nv (<= 8) consecutive BJump records at `recs` as the whole wave reads
// them at once: lane 2i holds bytes 0..15 of record i and lane 2i + 1 bytes
// 16..31 (zeros past nv).  One coalesced read of host memory per octet
// instead of one per field and lane.
__device__ __forceinline__ uint4 octet_load(const uint8_t* recs, uint32_t nv, uint32_t lane) {
  return lane < 2u * nv ? ((const uint4*)recs)[lane] : make_uint4(0u, 0u, 0u, 0u);
}
// A batch of jumps only under the direct mapping (n = 0 otherwise): worker w
// takes requests 8w .. 8w + 7, with no bins and no queue.
struct DirectJumps {
  const uint8_t* recs;  // its BJump records, as the device addresses them
  uint32_t n;           // requests
  uint32_t pad;
};
struct BChunk {         // 16 bytes
  uint32_t req, q, draws, last;  // slice (index within its bin), chunk index in the slice, draws, last of the slice
};
static_assert(sizeof(BHeader) == 64 && sizeof(BBin) == 256 && sizeof(BReq) == 48 && sizeof(BJump) == 32 &&
                  sizeof(BChunk) == 16,
              "descriptor layout");
constexpr uint32_t kMaxBins = 64;

// A bin's ranges, as held in registers (the counter is only touched atomically).
struct BinInfo {
  uint32_t s0, ns, nsc, k0, nk, g, n_ju, n_cg, gq, n_qi, a0, na, b0;
};

constexpr uint32_t kSpinLimit = 1u << 22;  // x ~100 cycles per sleep: about 0.2 s

// Descriptor access: either tables in device memory, or a single request
// passed by value (the one-launch-per-request path).
struct TableDesc {
  uint8_t* desc;          // device copy: header, bins, chunks, slices with draws
  const uint8_t* hdesc;   // the host staging buffer as the device sees it (slices without draws)
  __device__ __forceinline__ BHeader header() const { return *(const BHeader*)desc; }
  __device__ __forceinline__ BinInfo bin(uint32_t x) const {
    const BBin* b = (const BBin*)(desc + 64) + x;
    return BinInfo{b->s0, b->ns, b->nsc, b->k0, b->nk, b->g, b->n_ju, b->n_cg, b->gq, b->n_qi, b->a0, b->na, b->b0};
  }
  __device__ __forceinline__ uint32_t* counter(uint32_t x, uint32_t*) const { return &((BBin*)(desc + 64))[x].ctr; }
  // Slice rl of a bin: its slices with draws first (device table), then
  // those without (read from host memory, where the host wrote them: a
  // batch of jumps copies no slice table before its launch).
  __device__ __forceinline__ BReq req(const BHeader& h, const BinInfo& bn, uint32_t rl) const {
    if (rl < bn.na) return ((const BReq*)(desc + h.req_off))[bn.a0 + rl];
    const BJump j = ((const BJump*)(hdesc + h.jo_off))[bn.b0 + (rl - bn.na)];
    BReq q{};
    q.seed = j.seed;
    q.off_lo = j.off_lo;
    q.off_hi = j.off_hi;
    q.state = j.state;
    return q;
  }
  // The records of the slices rl0 .. rl0 + nv - 1 without draws (rl0 >= na).
  __device__ __forceinline__ uint4 octet_raw(const BHeader& h, const BinInfo& bn, uint32_t rl0, uint32_t nv,
                                             uint32_t lane) const {
    return octet_load(hdesc + h.jo_off + 32ull * (bn.b0 + (rl0 - bn.na)), nv, lane);
  }
  __device__ __forceinline__ BChunk chunk(const BHeader& h, uint32_t j) const {
    return ((const BChunk*)(desc + h.chunk_off))[j];
  }
  // The counters are reset by the next launch's descriptor copy.
  __device__ __forceinline__ void finish(uint32_t*) const {}
};
struct SingleDesc {
  BReq r0;
  uint32_t L, epoch;
  __device__ __forceinline__ BHeader header() const {
    BHeader h{};
    h.n_bins = 1;
    h.n_workers = gridDim.x;
    h.epoch = epoch;
    h.L = L;
    return h;
  }
  __device__ __forceinline__ BinInfo bin(uint32_t) const {
    BinInfo b;
    const uint64_t nq = (r0.count + L - 1) / L;
    b.s0 = 0;
    b.ns = 1;  // one jump pair, its second half idle
    b.nsc = 1;
    b.k0 = 0;
    b.nk = (uint32_t)nq;
    b.g = 1;
    b.n_ju = 1;
    b.n_cg = (uint32_t)((nq + 1) / 2);
    b.gq = 1;
    b.n_qi = 0;
    b.a0 = 0;
    b.na = 1;
    b.b0 = 0;
    return b;
  }
  __device__ __forceinline__ uint32_t* counter(uint32_t, uint32_t* queue) const { return queue; }
  __device__ __forceinline__ BReq req(const BHeader&, const BinInfo&, uint32_t) const { return r0; }
  // A single request has no octet items (n_qi = 0).
  __device__ __forceinline__ uint4 octet_raw(const BHeader&, const BinInfo&, uint32_t, uint32_t, uint32_t) const {
    return make_uint4(0u, 0u, 0u, 0u);
  }
  __device__ __forceinline__ BChunk chunk(const BHeader& h, uint32_t j) const {
    BChunk c;
    c.req = 0;
    c.q = j;
    const uint64_t first = (uint64_t)j * h.L;
    c.draws = (uint32_t)((r0.count - first) < h.L ? (r0.count - first) : h.L);
    c.last = (first + h.L >= r0.count) ? 1u : 0u;
    return c;
  }
  // The last workgroup out resets the counters for the next launch.
  __device__ __forceinline__ void finish(uint32_t* queue) const {
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const uint32_t f = atomicAdd(&queue[1], 1u);
      if (f == gridDim.x - 1) {
        atomicExch(&queue[0], 0u);
        atomicExch(&queue[1], 0u);
      }
    }
  }
};

struct BatchBuffers {
  uint32_t* req_states;    // 98 words per slice
  uint32_t* done;          // one flag per slice, plus one spare written by idle halves
  const uint32_t* ptab;    // 97 words per q: P_{qL}
  const uint32_t* wtab;    // window table T[w][d], 8-bit digits
  const uint32_t* wtab20;  // window table with 20-bit digits, or nullptr
  const uint32_t* wtab24;  // window table with 24-bit digits (octets take it when set), or nullptr
  uint32_t* queue;         // single-request launches: [0] next item, [1] finished workgroups
  int* err;                // host-visible error word
  uint32_t spare;          // index of the spare flag
};

// LDS per half-wave: the extended window X (193 words) and a polynomial (97).
constexpr int kHalfLds = 193 + 97;
// LDS per 8-lane group of a jump octet (stride 1 mod 4: see k_jump_grp).
constexpr int kOctStride = 193 + 97 + 3;
constexpr int kWaveLds = 8 * kOctStride > 2 * kHalfLds + 256 ? 8 * kOctStride : 2 * kHalfLds + 256;
static_assert(2 * kHalfLds + 256 <= kWaveLds, "chunk pairs: two half-wave windows and their transpose buffers");

// Hand-off of a slice's start state from the wave that jumped it to the waves
// that generate its chunks, which may run on other XCDs (each XCD has its own
// L2).  The producer writes the words with device-scope stores, which are
// written through to the device's coherence point and acknowledged from
// there; publish_wait waits for those acknowledgements (vmcnt = 0) before
// the flag is stored.  The consumers poll the flag and then read the words
// with device-scope loads, which are served from the coherence point rather
// than from a possibly stale L2 line.  This gives the same visibility as an
// agent-scope release/acquire pair without that pair's whole-L2 writeback
// and invalidate (one of each per slice and per chunk).
__device__ __forceinline__ void dev_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t dev_load(uint32_t* p) {
  return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish_wait() {
  __builtin_amdgcn_s_waitcnt(0);  // all counters zero: every store above has been acknowledged
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // keeps the flag store after it in program order
}

// The lane within the wave, opaque to the optimiser: the item functions run
// inside the persistent loop, and without this the compiler hoists every
// lane-derived address and constant-table read of the seeding out of the loop
// and keeps them in registers across items (135 VGPRs for the octet path
// against 97).
__device__ __forceinline__ uint32_t item_lane() {
  uint32_t lane = threadIdx.x & 63u;
  asm volatile("" : "+v"(lane));
  return lane;
}

template <class Desc>
__device__ __forceinline__ void batch_jump_pair(const Desc& D, const BHeader& h, const BatchBuffers& B,
                                                const BinInfo& bn, uint32_t p, uint32_t* lds, const SeedLds<true>& stab) {
  const uint32_t lane = item_lane();
  const uint32_t half = lane >> 5, l = lane & 31u;
  const uint32_t rl = 2u * p + half;
  const bool active = rl < bn.nsc;
  const uint32_t r = bn.s0 + rl;
  uint32_t* X = lds + half * kHalfLds;
  uint32_t* Bp = X + 193;
  BReq q{};
  if (active) q = D.req(h, bn, rl);
  const bool valid = active && seed_group_tab<32, 4, true>(q.seed, X, l, stab);
  if (!valid) X[l] = X[l + 32] = X[l + 64] = X[97] = 0;
  wave_sync();
  const uint32_t c = X[97];
  const uint32_t j0 = valid ? (uint32_t)q.off_lo : 0u, j1 = valid ? (uint32_t)(q.off_lo >> 32) : 0u;
  const uint32_t j2 = valid ? (uint32_t)q.off_hi : 0u, j3 = valid ? (uint32_t)(q.off_hi >> 32) : 0u;
  if (B.wtab24)  // uniform: 5 factors for a 120-bit offset instead of 15
    jump_half<24>(X, Bp, B.wtab24, j0, j1, j2, j3, wave_windows<24>(j0, j1, j2, j3), l);
  else if (B.wtab20)  // 6 factors
    jump_half<20>(X, Bp, B.wtab20, j0, j1, j2, j3, wave_windows<20>(j0, j1, j2, j3), l);
  else
    jump_half<8>(X, Bp, B.wtab, j0, j1, j2, j3, wave_windows<8>(j0, j1, j2, j3), l);
  // A request with no draws but a state output is written straight to the
  // caller's record.  The words go out as device-scope stores (written
  // through to the device's coherence point, see publish_wait), so chunks on
  // other XCDs can read them without an L2 writeback here or an L2
  // invalidate there.
  uint32_t* slot = (active && q.count == 0 && q.state) ? (uint32_t*)q.state : B.req_states + (uint64_t)r * kWords;
  if (active) {
    dev_store(slot + l, valid ? X[l] : 0u);
    dev_store(slot + l + 32, valid ? X[l + 32] : 0u);
    dev_store(slot + l + 64, valid ? X[l + 64] : 0u);
    if (l == 0) {
      dev_store(slot + 96, valid ? X[96] : 0u);
      dev_store(slot + 97, valid ? c_jump(c, u128_mod_m(j0, j1, j2, j3)) : kInvalidC);
    }
  }
  // Only slices with draws have chunks waiting for them (the test is
  // wave-uniform).
  if (__any(active && q.count > 0)) {
    publish_wait();
    // Every lane of the half stores the same value (idle halves to the spare).
    __hip_atomic_store(&B.done[active ? r : B.spare], h.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  wave_sync();
}

template <class Desc>
__device__ __forceinline__ void batch_chunk_pair(const Desc& D, const BHeader& h, const BatchBuffers& B,
                                                 const BinInfo& bn, uint32_t cp, uint32_t* lds) {
  const uint32_t lane = item_lane();
  const uint32_t half = lane >> 5, l = lane & 31u;
  const uint32_t jl = 2u * cp + half;
  const bool active = jl < bn.nk;
  const uint32_t j = bn.k0 + jl;
  uint32_t* X = lds + half * kHalfLds;
  uint32_t* Bp = X + 193;
  BChunk ch{};
  BReq rq{};
  if (active) ch = D.chunk(h, j);
  const uint32_t r = bn.s0 + ch.req;  // the chunk's slice
  // P_{qL} does not depend on the slice: fetch it before waiting.
  const uint32_t* P = B.ptab + (uint64_t)ch.q * 97u;
  const uint32_t p0 = P[l], p1 = P[l + 32], p2 = P[l + 64], p3 = P[96];
  if (active) {
    rq = D.req(h, bn, ch.req);
    uint32_t it = 0;
    while (__hip_atomic_load(&B.done[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != h.epoch) {
      __builtin_amdgcn_s_sleep(2);
      if (++it > kSpinLimit) {
        __hip_atomic_store(B.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        break;
      }
    }
  }
  // No loads below may be moved above the wait (the fence emits no code at
  // this scope; the words are read with device-scope loads).
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  // Chunk start: the slice's start state times P_{qL}(A), c by qL steps.
  uint32_t* src = B.req_states + (uint64_t)r * kWords;
  X[l] = active ? dev_load(src + l) : 0u;
  X[l + 32] = active ? dev_load(src + l + 32) : 0u;
  X[l + 64] = active ? dev_load(src + l + 64) : 0u;
  Bp[l] = p0;
  Bp[l + 32] = p1;
  Bp[l + 64] = p2;
  if (l == 0) {
    X[96] = active ? dev_load(src + 96) : 0u;
    Bp[96] = p3;
  }
  const uint32_t c0 = active ? dev_load(src + 97) : 0u;
  wave_sync();
  apply_half(X, Bp, l);
  if (l == 0) X[97] = c_jump(c0, (uint32_t)(((uint64_t)ch.q * h.L) % kMod));
  wave_sync();
  if (active) {
    uint32_t* dst = (ch.last && rq.state) ? (uint32_t*)rq.state : nullptr;
    char* row = (char*)rq.out + (uint64_t)ch.q * h.L * 4u;
    // A 16-byte aligned row (always, from a server's arena) is written four
    // blocks at a time, 16 bytes per lane, through 128 words of LDS per half.
    if (((uintptr_t)row & 15u) == 0)
      gen_stream32_wide<FMT_RUNTIME, true>(l, lane, X, dst, ch.draws, rq.fmt == RANMAR_F32, row,
                                           lds + 2 * kHalfLds + 128u * half);
    else
      gen_stream32<FMT_RUNTIME, true>(l, lane, X, dst, ch.draws, rq.fmt == RANMAR_F32, row);
  }
  wave_sync();
}

// Seeds and jumps the nv (<= 8) slices without draws of one octet, 8 lanes
// each (seed_group / jump_group of coop_dev.hpp, 20-bit windows; octets are
// made only when that table exists), from their records as octet_load reads
// them.  Nothing waits for them: the state goes straight to the caller's
// record, if it asked for one.  `issued` runs inside the jump, once its first
// factor is being fetched (see jump_group).
template <class Hook>
__device__ __forceinline__ void jump_octet(uint4 raw, uint32_t nv, uint32_t lane, uint32_t* lds,
                                           const SeedLds<true>& stab, const BatchBuffers& B, Hook issued) {
  const uint32_t grp = lane >> 3, l = lane & 7u;
  const bool active = grp < nv;
  uint32_t* X = lds + grp * kOctStride;
  uint32_t* Bp = X + 193;
  // The group's record from lanes 2 grp (seed, offset low) and 2 grp + 1
  // (offset high, state pointer).
  const int s0 = (int)(grp * 8u), s1 = s0 + 4;  // ds_bpermute byte addresses of lanes 2 grp, 2 grp + 1
  const int32_t seed = __builtin_amdgcn_ds_bpermute(s0, (int)raw.x);
  const uint32_t j0 = (uint32_t)__builtin_amdgcn_ds_bpermute(s0, (int)raw.z);
  const uint32_t j1 = (uint32_t)__builtin_amdgcn_ds_bpermute(s0, (int)raw.w);
  const uint32_t j2 = (uint32_t)__builtin_amdgcn_ds_bpermute(s1, (int)raw.x);
  const uint32_t j3 = (uint32_t)__builtin_amdgcn_ds_bpermute(s1, (int)raw.y);
  const uint64_t st = (uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(s1, (int)raw.z) |
                      (uint64_t)(uint32_t)__builtin_amdgcn_ds_bpermute(s1, (int)raw.w) << 32;
  const bool valid = active && seed_group_tab<8, 7, true>(seed, X, l, stab);
  if (!valid) {
#pragma unroll
    for (int k = 0; k < 96; k += 8) X[l + k] = 0;
    if (l == 0) X[96] = X[97] = 0;
  }
  wave_sync();
  const uint32_t c = X[97];
  const uint32_t e0 = valid ? j0 : 0u, e1 = valid ? j1 : 0u, e2 = valid ? j2 : 0u, e3 = valid ? j3 : 0u;
  if (B.wtab24)  // uniform: 5 factors for a 120-bit offset instead of 6
    jump_group<8, 24>(X, Bp, B.wtab24, e0, e1, e2, e3, wave_windows<24>(e0, e1, e2, e3), l, issued);
  else
    jump_group<8, 20>(X, Bp, B.wtab20, e0, e1, e2, e3, wave_windows<20>(e0, e1, e2, e3), l, issued);
  if (active && st) {
    gu32* dst = gptr((void*)(uintptr_t)st);
#pragma unroll
    for (int k = 0; k < 96; k += 8) dst[l + k] = valid ? X[l + k] : 0u;
    if (l == 0) {
      dst[96] = valid ? X[96] : 0u;
      dst[97] = valid ? c_jump(c, u128_mod_m(e0, e1, e2, e3)) : kInvalidC;
    }
  }
  wave_sync();
}

// Octet qi of a bin's slices without draws.
template <class Desc, class Hook>
__device__ __forceinline__ void batch_jump_oct(const Desc& D, const BHeader& h, const BatchBuffers& B,
                                               const BinInfo& bn, uint32_t qi, uint32_t* lds, const SeedLds<true>& stab,
                                               Hook issued) {
  const uint32_t lane = item_lane();
  const uint32_t rl0 = bn.nsc + 8u * qi;
  const uint32_t nv = bn.ns - rl0 < 8u ? bn.ns - rl0 : 8u;
  jump_octet(D.octet_raw(h, bn, rl0, nv, lane), nv, lane, lds, stab, B, issued);
}

// WPG independent one-wave workers per workgroup, sharing one copy of the
// seeding table (filled before the only barrier); worker w serves bin
// w mod n_bins.  The wave index is taken through readfirstlane, so the worker,
// the bin and everything derived from them stay wave-uniform (scalar
// registers), as they would with blockIdx.x alone.
template <int WPG, class Desc>
__device__ __forceinline__ void batch_persistent(const Desc& D, const BatchBuffers& B) {
  __shared__ __align__(16) uint32_t lds_all[WPG][kWaveLds];  // 16-byte rows: chunk transposes read u32x4
  __shared__ SeedLds<true> seed_tab;
  const BHeader h = D.header();
  if (blockIdx.x * WPG >= h.n_workers) return;  // whole workgroups leave together
  seed_lds_fill(seed_tab, threadIdx.x, 64u * WPG);
  __syncthreads();
  const uint32_t wv = WPG == 1 ? 0u : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t worker = blockIdx.x * WPG + wv;
  if (worker >= h.n_workers) return;  // the last workgroup's spare waves (no barrier follows)
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t* lds = lds_all[wv];
  const uint32_t x = worker % h.n_bins;
  const BinInfo bn = D.bin(x);
  uint32_t* ctr = D.counter(x, B.queue);
  const uint32_t n_jg = (bn.nsc + 1) / 2;           // jump pairs
  const uint32_t n_jq = (bn.ns - bn.nsc + 7) / 8;   // jump octets
  // Dequeue without a lane-conditional branch: every lane executes the
  // atomic, lane 0 adding 1 and the others 0, and lane 0's result is taken.
  // (With `if (lane == 0) item = atomicAdd(...)` only lane 0 holds the item,
  // and the compiler may merge that branch with other lane-0 branches of the
  // loop body so that lanes 1..63 re-enter the body on a stale item.)
  auto dequeue = [&]() { return atomicAdd(ctr, lane == 0 ? 1u : 0u); };
  uint32_t got = dequeue();
  for (;;) {
    const uint32_t item = __builtin_amdgcn_readfirstlane(got);
    if (item < bn.n_ju) {
      const uint32_t p1 = (item + 1) * bn.g < n_jg ? (item + 1) * bn.g : n_jg;
      for (uint32_t p = item * bn.g; p < p1; ++p) batch_jump_pair(D, h, B, bn, p, lds, seed_tab);
      got = dequeue();
    } else if (item < bn.n_ju + bn.n_cg) {
      batch_chunk_pair(D, h, B, bn, item - bn.n_ju, lds);
      got = dequeue();
    } else if (item < bn.n_ju + bn.n_cg + bn.n_qi) {
      // Octets come last in a bin, and nothing waits for them: the next item
      // is taken during the last octet's jump, so the atomic's round trip
      // (microseconds, at the device's coherence point) overlaps the jump.
      const uint32_t it = item - bn.n_ju - bn.n_cg;
      const uint32_t p1 = (it + 1) * bn.gq < n_jq ? (it + 1) * bn.gq : n_jq;
      for (uint32_t p = it * bn.gq; p < p1; ++p) {
        const bool last = p + 1 == p1;
        batch_jump_oct(D, h, B, bn, p, lds, seed_tab, [&]() {
          if (last) got = dequeue();
        });
      }
    } else {
      break;
    }
  }
  D.finish(B.queue);
}

// The direct mapping of a batch of jumps only: wave w of the grid seeds and
// jumps requests 8w .. 8w + 7 (no bins, no queue, no descriptor).  The
// octet's records are fetched before the table fill, which hides their latency.
template <int WPG>
__device__ __forceinline__ void batch_direct(const BatchBuffers& B, const DirectJumps& dj) {
  __shared__ uint32_t lds_all[WPG][8 * kOctStride];
  __shared__ SeedLds<true> seed_tab;
  const uint32_t wv = WPG == 1 ? 0u : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t rl0 = 8u * (blockIdx.x * WPG + wv);
  const uint32_t nv = rl0 < dj.n ? (dj.n - rl0 < 8u ? dj.n - rl0 : 8u) : 0u;
  const uint4 raw = octet_load(dj.recs + 32ull * rl0, nv, lane);
  seed_lds_fill(seed_tab, threadIdx.x, 64u * WPG);
  __syncthreads();
  if (nv) jump_octet(raw, nv, lane, lds_all[wv], seed_tab, B, NoHook{});
}

}  // namespace ranmar
