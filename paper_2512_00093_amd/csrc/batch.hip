// Batched execution of uneven requests in one persistent launch (host side).
//
// ranmar_batch_prepare cuts the requests into slices and chunks, spreads them
// over up to 64 bins of about equal work (one jump counted as one chunk) and
// writes the header, bin, chunk and slice tables to a pinned host staging
// buffer.  A request that straddles two bins is split at a chunk boundary; the
// second part is a request of its own (offset + first draw), so the draws are
// unchanged.  ranmar_batch_launch is one launch of a captured graph
//     [memcpy staging -> device tables]  ->  [persistent kernel]
// whose memcpy size and grid are set per launch (the grid: as many one-wave
// workers per bin as the bin has items, up to what the device holds at once).  The
// copy takes the header, the bins (zeroing their queue counters), the chunks
// and the slices with draws; the slices without draws (jumps only: 32 bytes
// per request, most of a large batch of jumps) stay in the staging buffer,
// which is coherent host memory mapped for the device, and the kernel reads
// each as it takes it, while other waves compute.
//
// ranmar_run_unbatched: the same kernel launched once per request with the
// request passed by value (no tables, no graph): the baseline the batched path
// is measured against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/ranmar.h"
#include "batch_dev.hpp"
#include "internal.hpp"

namespace ranmar {

// Four one-wave workers per workgroup: one copy of the seeding table per four
// waves keeps the LDS of 16 waves within a CU's 160 KB.
constexpr uint32_t kBatchWpg = 4;

// The kernels of the two graphs take the same arguments (the direct graph's
// kernel reads only B and dj, the other only desc, hdesc and B).
__global__ __launch_bounds__(64 * kBatchWpg) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_tables(
    uint8_t* desc, const uint8_t* hdesc, BatchBuffers B, DirectJumps) {
  batch_persistent<kBatchWpg>(TableDesc{desc, hdesc}, B);
}

__global__ __launch_bounds__(64 * kBatchWpg) void k_batch_direct(uint8_t*, const uint8_t*, BatchBuffers B,
                                                                 DirectJumps dj) {
  batch_direct<kBatchWpg>(B, dj);
}

__global__ __launch_bounds__(64) void k_batch_single(SingleDesc d, BatchBuffers B) { batch_persistent<1>(d, B); }

constexpr uint32_t kDefaultChunk = 16384;
// Chunk length of the one-launch-per-request path (and of a server's ticks that
// hold one request): a request's chunks run in parallel after its jump, so
// shorter chunks finish it sooner.  Served at 2e4 requests/s (median request
// about 30,000 draws): p50 65 us with 16,384, 55 us with 8,192 and 4,096,
// 54-58 us with 2,048; p99 105-108 us down to 8,192, 111-117 us at 4,096,
// 140-147 us at 2,048 (each chunk starts with a 97 x 97 application of P_qL).
constexpr uint32_t kUnbatchedChunk = 8192;
constexpr uint32_t kMaxChunkDraws = 1u << 24;

// Workgroups of `kernel` (block size `threads`) that fit the device at once
// (occupancy times the number of CUs): every workgroup of the grid is resident.
static unsigned persistent_grid(const void* kernel, int threads) {
  int dev = 0, cus = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
    per_cu = 2;
  return (unsigned)(cus > 0 ? cus : 256) * (unsigned)per_cu;
}

// P_{qL} for q < nq into ptab (97 words each), on `st`.
static hipError_t fill_ptab(uint32_t* ptab, uint64_t nq, uint32_t L, hipStream_t st) {
  std::vector<ranmar_u128> J(nq);
  for (uint64_t q = 0; q < nq; ++q) {
    const unsigned __int128 v = (unsigned __int128)q * L;
    J[q].lo = (uint64_t)v;
    J[q].hi = (uint64_t)(v >> 64);
  }
  ranmar_u128* dJ = nullptr;
  hipError_t e = hipMalloc(&dJ, sizeof(ranmar_u128) * nq);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(dJ, J.data(), sizeof(ranmar_u128) * nq, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_jump_poly(dJ, nq, ptab, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(dJ);
  return e;
}

// Checks one request and returns its chunk count (0 for count == 0).
static int check_request(const ranmar_request& q, uint32_t L, uint64_t* nq) {
  if (q.seed < 1 || q.seed > 900000000) return RANMAR_EINVAL;
  if (q.fmt != RANMAR_U24 && q.fmt != RANMAR_F32) return RANMAR_EINVAL;
  if (q.count > 0 && (!q.d_out || ((uintptr_t)q.d_out & 3))) return RANMAR_EINVAL;
  if (q.d_state && ((uintptr_t)q.d_state & 3)) return RANMAR_EINVAL;
  // Parts of a request cut at chunk boundaries start at offset + d (d <
  // count) as 128-bit offsets of their own: the last must not pass 2^128 - 1.
  const unsigned __int128 off = ((unsigned __int128)q.offset.hi << 64) | q.offset.lo;
  if (q.count > 0 && off > ~(unsigned __int128)0 - (q.count - 1)) return RANMAR_EINVAL;
  *nq = q.count ? (q.count - 1) / L + 1 : 0;  // no division for a jump
  return RANMAR_OK;
}

// body(lo, hi, part) over a split of [0, n) into parts: on up to eight
// threads for large n, else on the calling thread.  The split depends only on
// n, so two calls with the same n see the same parts.
template <class F>
static void parallel_parts(uint64_t n, uint32_t parts, F&& body) {
  if (parts <= 1) {
    body(0, n, 0u);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(parts - 1);
  for (uint32_t t = 1; t < parts; ++t) th.emplace_back([&, t] { body(n * t / parts, n * (t + 1) / parts, t); });
  body(0, n / parts, 0u);
  for (auto& x : th) x.join();
}

static uint32_t host_parts(uint64_t n) {
  if (n < 65536) return 1;
  const unsigned hw = std::thread::hardware_concurrency();
  return std::max(1u, std::min(8u, hw ? hw : 1u));
}

// A jump record written to the staging buffer with streaming stores (two
// 16-byte halves; the buffer is only read by the device, so the host need not
// fetch its lines first).  stage_fence() orders them before the launch.
typedef long long v2i64 __attribute__((vector_size(16)));
static void stage_bjump(BJump* dst, const ranmar_request& q) {
  v2i64 a, b;
  a[0] = (long long)(uint32_t)q.seed;
  a[1] = (long long)q.offset.lo;
  b[0] = (long long)q.offset.hi;
  b[1] = (long long)(uintptr_t)q.d_state;
  __builtin_nontemporal_store(a, (v2i64*)dst);
  __builtin_nontemporal_store(b, (v2i64*)dst + 1);
}
static void stage_fence() { __builtin_ia32_sfence(); }

static BReq to_breq(const ranmar_request& q) {
  BReq b{};
  b.seed = q.seed;
  b.fmt = q.fmt;
  b.off_lo = q.offset.lo;
  b.off_hi = q.offset.hi;
  b.count = q.count;
  b.out = (uint64_t)(uintptr_t)q.d_out;
  b.state = (uint64_t)(uintptr_t)q.d_state;
  return b;
}

}  // namespace ranmar

using namespace ranmar;

struct ranmar_batch {
  uint64_t max_req = 0, max_chunks = 0, max_slices = 0;
  uint32_t L = kDefaultChunk;
  size_t desc_cap = 0;        // device copy: header, bins, chunks, slices with draws
  size_t host_cap = 0;        // staging buffer: the same and the slices without draws
  uint8_t* d_desc = nullptr;
  uint8_t* h_desc = nullptr;
  uint8_t* h_desc_dev = nullptr;  // h_desc as the device addresses it
  uint32_t *d_req_states = nullptr, *d_done = nullptr, *d_queue = nullptr, *d_ptab = nullptr;
  int* h_err = nullptr;
  uint32_t epoch = 0;
  unsigned workers_max = 0;   // one-wave workers the device holds at once (kBatchWpg per workgroup)
  unsigned grid_node = 0;     // workers of the graph's kernel node now
  unsigned grid_dnode = 0;    // the same for the direct graph (0: its arguments must be set)
  unsigned grid_prepared = 0; // workers for the prepared tables
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // A batch of jumps only under the direct mapping reads no descriptor: it is
  // launched from a second graph that holds the kernel node alone.
  hipGraph_t graph_d = nullptr;
  hipGraphExec_t exec_d = nullptr;
  hipGraphNode_t kern_d = nullptr;
  hipGraphNode_t cpy = nullptr, kern = nullptr;
  hipEvent_t last = nullptr;
  bool launched = false;
  size_t prepared_bytes = 0;  // descriptor bytes staged by prepare, 0 = none
  BatchBuffers B{};
  std::vector<BReq> tmp;      // prepare: slices with draws, before the final layout
  bool tried_wtab = false;  // the 20-bit window table was asked for
  uint8_t* kdesc = nullptr;   // kernel argument storage for the graph node
  const uint8_t* khdesc = nullptr;
  DirectJumps kdirect{nullptr, 0u, 0u};      // kernel argument storage (copied when a node's arguments are set)
  DirectJumps kdirect_d{nullptr, 0u, 0u};    // the direct graph's node now
  DirectJumps dj_prepared{nullptr, 0u, 0u};  // the prepared batch's (n = 0: not direct)
  void* kargs[4] = {nullptr, nullptr, nullptr, nullptr};
  int variant = -1;           // mapping (BatchVariant); -1: the tuner's table
};

static hipKernelNodeParams kernel_params(ranmar_batch* b, unsigned workers, bool direct) {
  hipKernelNodeParams kp{};
  b->kargs[0] = (void*)&b->kdesc;
  b->kargs[1] = (void*)&b->khdesc;
  b->kargs[2] = (void*)&b->B;
  b->kargs[3] = (void*)&b->kdirect;
  kp.func = direct ? (void*)k_batch_direct : (void*)k_batch_tables;
  kp.gridDim = dim3((workers + kBatchWpg - 1) / kBatchWpg);
  kp.blockDim = dim3(64 * kBatchWpg);
  kp.sharedMemBytes = 0;
  kp.kernelParams = b->kargs;
  kp.extra = nullptr;
  return kp;
}

static void batch_free(ranmar_batch* b) {
  if (!b) return;
  if (b->last) hipEventSynchronize(b->last);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->exec_d) hipGraphExecDestroy(b->exec_d);
  if (b->graph_d) hipGraphDestroy(b->graph_d);
  if (b->last) hipEventDestroy(b->last);
  hipFree(b->d_desc);
  hipFree(b->d_req_states);
  hipFree(b->d_done);
  hipFree(b->d_queue);
  hipFree(b->d_ptab);
  if (b->h_desc) hipHostFree(b->h_desc);
  if (b->h_err) hipHostFree(b->h_err);
  delete b;
}

// Layout of the staging buffer: header, bins, chunk table, the slices with
// draws (these four are copied to the device before each launch), then the
// slices without draws, which the kernel reads from the staging buffer itself
// (a batch of jumps copies only its header and bins).
static uint64_t chunk_offset(uint32_t nb) { return 64 + sizeof(BBin) * (uint64_t)nb; }
static uint64_t align16(uint64_t v) { return (v + 15) & ~15ull; }
// Where a batch of jumps only keeps its records: past the header and the most
// bins any batch has (no slices or chunks precede them).
constexpr uint64_t kJumpsOnlyOff = 64 + sizeof(BBin) * (uint64_t)kMaxBins;

namespace ranmar {
void batch_set_variant(ranmar_batch* b, int v) {
  if (b) b->variant = (v >= 0 && v < BATCH_NUM_VARIANTS) ? v : -1;
}

void batch_use_wide_windows(ranmar_batch* b) {
  if (!b) return;
  b->tried_wtab = true;
  const uint32_t* T = window20_table();
  if (T && b->B.wtab20 != T) {
    b->B.wtab20 = T;
    b->grid_node = b->grid_dnode = 0;  // the kernel nodes take the pointer at the next launch
  }
}
}  // namespace ranmar

extern "C" {

int ranmar_batch_create(uint64_t max_requests, uint64_t max_chunks, uint64_t chunk_draws, ranmar_batch** out) {
  if (!out || max_requests == 0 || max_requests > (1ull << 26) || max_chunks > (1ull << 26)) return RANMAR_EINVAL;
  if (chunk_draws > kMaxChunkDraws) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  ranmar_batch* b = new ranmar_batch();
  b->max_req = max_requests;
  b->max_chunks = max_chunks ? max_chunks : 1;
  b->max_slices = b->max_req + kMaxBins;  // each bin boundary splits at most one request
  b->L = chunk_draws ? (uint32_t)chunk_draws : chunk_draws_default(kDefaultChunk);
  // Slices: each request once, plus at most one extra part per bin boundary.
  b->desc_cap = align16(chunk_offset(kMaxBins) + sizeof(BChunk) * b->max_chunks) + sizeof(BReq) * b->max_slices;
  b->host_cap = align16(b->desc_cap) + sizeof(BJump) * b->max_req;
  b->workers_max =
      std::max<unsigned>(kBatchWpg * persistent_grid((const void*)k_batch_tables, 64 * kBatchWpg), kMaxBins);
  const uint64_t nflags = b->max_slices + 1;  // slice flags + the spare
  hipStream_t st = nullptr;
  // The staging buffer is coherent host memory: the kernel reads the slices
  // without draws from it, and every launch must see what the host wrote last.
  bool ok = hipMalloc(&b->d_desc, b->desc_cap) == hipSuccess &&
            hipHostMalloc(&b->h_desc, b->host_cap, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
            hipHostGetDevicePointer((void**)&b->h_desc_dev, b->h_desc, 0) == hipSuccess &&
            hipHostMalloc(&b->h_err, sizeof(int), hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
            hipMalloc(&b->d_req_states, 4 * kWords * b->max_slices) == hipSuccess &&
            hipMalloc(&b->d_done, 4 * nflags) == hipSuccess && hipMalloc(&b->d_queue, 8) == hipSuccess &&
            hipMalloc(&b->d_ptab, 4 * 97 * b->max_chunks) == hipSuccess && hipEventCreate(&b->last) == hipSuccess;
  if (ok) {
    *b->h_err = 0;
    ok = hipMemset(b->d_done, 0, 4 * nflags) == hipSuccess && hipMemset(b->d_queue, 0, 8) == hipSuccess &&
         hipStreamCreate(&st) == hipSuccess;
  }
  if (ok) ok = fill_ptab(b->d_ptab, b->max_chunks, b->L, st) == hipSuccess;
  if (st) hipStreamDestroy(st);
  if (ok) {
    b->B.req_states = b->d_req_states;
    b->B.done = b->d_done;
    b->B.ptab = b->d_ptab;
    b->B.queue = b->d_queue;
    b->B.err = b->h_err;
    b->B.wtab = window_table();
    b->B.wtab20 = nullptr;  // set by the first batch with many requests without draws
    b->B.wtab24 = nullptr;  // set while the jump tuner's pick for such batches is the 24-bit table
    b->B.spare = (uint32_t)b->max_slices;
    ok = b->B.wtab != nullptr;
  }
  if (ok) {
    b->kdesc = b->d_desc;
    b->khdesc = b->h_desc_dev;
    ok = hipGraphCreate(&b->graph, 0) == hipSuccess &&
         hipGraphAddMemcpyNode1D(&b->cpy, b->graph, nullptr, 0, b->d_desc, b->h_desc, b->desc_cap,
                                 hipMemcpyHostToDevice) == hipSuccess;
    if (ok) {
      const unsigned grid = b->workers_max;  // workers
      const hipKernelNodeParams kp = kernel_params(b, grid, false);
      const hipKernelNodeParams kpd = kernel_params(b, grid, true);
      ok = hipGraphAddKernelNode(&b->kern, b->graph, &b->cpy, 1, &kp) == hipSuccess &&
           hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess &&
           hipGraphCreate(&b->graph_d, 0) == hipSuccess &&
           hipGraphAddKernelNode(&b->kern_d, b->graph_d, nullptr, 0, &kpd) == hipSuccess &&
           hipGraphInstantiate(&b->exec_d, b->graph_d, nullptr, nullptr, 0) == hipSuccess;
      b->grid_node = grid;
      b->grid_dnode = 0;
    }
  }
  if (!ok) {
    batch_free(b);
    return RANMAR_EHIP;
  }
  *out = b;
  return RANMAR_OK;
}

int ranmar_batch_prepare(ranmar_batch* b, const ranmar_request* reqs, uint64_t n) {
  if (!b || (n && !reqs)) return RANMAR_EINVAL;
  b->prepared_bytes = 0;
  if (n > b->max_req) return RANMAR_ENOMEM;
  if (n == 0) return RANMAR_OK;
  // The staging buffer may still be read by the previous run's copy and kernel.
  if (b->launched && hipEventSynchronize(b->last) != hipSuccess) return RANMAR_EHIP;
  // Validation and counts, in parts (large batches on several threads).  A
  // batch that starts with a request without draws is taken for one of jumps
  // only: its records are staged in the same pass, at the fixed place such a
  // batch keeps them (entry r for request r), and kept if the guess holds.
  const bool guess_jumps = reqs[0].count == 0;
  BJump* jo_fixed = (BJump*)(b->h_desc + kJumpsOnlyOff);
  const uint32_t parts = host_parts(n);
  std::vector<uint64_t> p_total(parts, 0), p_jo(parts, 0), p_draws(parts, 0);
  std::vector<int> p_rc(parts, RANMAR_OK);
  parallel_parts(n, parts, [&](uint64_t lo, uint64_t hi, uint32_t t) {
    uint64_t tot = 0, jo = 0, dr = 0;
    for (uint64_t r = lo; r < hi; ++r) {
      uint64_t nq = 0;
      const int rc = check_request(reqs[r], b->L, &nq);
      if (rc) {
        p_rc[t] = rc;
        return;
      }
      tot += nq;
      jo += nq == 0;
      dr += reqs[r].count;
      if (guess_jumps && nq == 0) stage_bjump(jo_fixed + r, reqs[r]);
    }
    if (guess_jumps) stage_fence();  // before anything later writes the same lines
    p_total[t] = tot;
    p_jo[t] = jo;
    p_draws[t] = dr;
  });
  uint64_t total = 0, n_jo = 0, draws = 0;  // chunks; requests without draws; draws
  for (uint32_t t = 0; t < parts; ++t) {
    if (p_rc[t]) return p_rc[t];
    total += p_total[t];
    n_jo += p_jo[t];
    draws += p_draws[t];
  }
  // The mapping: forced on this batch (the tuner), else the tuned table's
  // pick for this shape.
  const int bv = b->variant >= 0 ? b->variant : batch_variant_for(n, draws / n);
  if (total > b->max_chunks) return RANMAR_ENOMEM;
  // Many requests without draws: jump them with 20-bit windows (the 2.4 GB
  // table is built once per device, on first use; if it cannot be, the 8-bit
  // table serves).  The kernel node takes the new pointer at the next launch.
  if (n_jo >= 16384 && !b->B.wtab20 && !b->tried_wtab) {
    b->tried_wtab = true;
    b->B.wtab20 = window20_table();
    b->grid_node = b->grid_dnode = 0;  // forces the kernel nodes' arguments to be set again
  }
  // Octets take the 24-bit table where the jump kernel's pick for as many
  // requests does (the tuner's choice: 32.5 GB, 5 factors per 120-bit offset).
  {
    const uint32_t* t24 = n_jo >= 16384 && b->B.wtab20 && jump_variant_for(n_jo) == JUMP_EIGHTH_WINDOW24
                              ? window24_table()
                              : nullptr;
    if (t24 != b->B.wtab24) {
      b->B.wtab24 = t24;
      b->grid_node = b->grid_dnode = 0;  // the kernel nodes take the pointer at the next launch
    }
  }
  // The direct mapping applies to batches of jumps only, as octets (else the
  // default mapping serves): one bin, and a grid of one worker per octet.
  const bool direct = bv == BATCH_DIRECT && n_jo == n && b->B.wtab20 != nullptr;
  const bool fine = bv == BATCH_FINE || bv == BATCH_BINS16_FINE || direct;
  const uint32_t max_bins = direct ? 1u : (bv == BATCH_BINS16 || bv == BATCH_BINS16_FINE) ? 16u : kMaxBins;
  // Bins: about 4 units of work (jumps + chunks) per bin at least, at most 64.
  const uint64_t cost = n + total;
  const uint32_t nb = (uint32_t)std::min<uint64_t>(max_bins, std::max<uint64_t>(1, cost / 4));
  const uint64_t chunk_off = chunk_offset(nb), req_off = align16(chunk_off + sizeof(BChunk) * total);
  BHeader* h = (BHeader*)b->h_desc;
  BBin* bins = (BBin*)(b->h_desc + 64);
  BReq* sl = (BReq*)(b->h_desc + req_off);  // slices with draws
  BChunk* ch = (BChunk*)(b->h_desc + chunk_off);
  std::memset(b->h_desc, 0, chunk_off);  // header and bins (the bins' queue counters start at 0)
  const uint64_t L = b->L;

  // Requests with draws, in order, fill the bins one after the other with
  // about Tc units (one per slice jump, one per chunk) each; a request that
  // does not fit is cut at a chunk boundary and continues in the next bin.
  // Their slices are collected in b->tmp, in bin order.
  const uint64_t Tc = std::max<uint64_t>(2, (n - n_jo + total + nb - 1) / nb);
  std::vector<BReq>& tmp = b->tmp;
  tmp.clear();
  std::vector<uint32_t> nsc(nb, 0), nkb(nb, 0);
  uint64_t nc = 0, fill = 0;
  uint32_t x = 0;
  for (uint64_t r = 0; r < n; ++r) {
    const ranmar_request& q = reqs[r];
    const uint64_t nq = (q.count + L - 1) / L;
    if (nq == 0) continue;
    uint64_t first = 0;  // chunks of request r placed so far
    while (first < nq) {
      uint64_t take = nq - first;
      if (x + 1 < nb) {
        const uint64_t room = fill + 1 < Tc ? Tc - fill - 1 : 0;  // chunks that fit beside this slice's jump
        if (fill > 0 && room == 0) {
          ++x;
          fill = 0;
          continue;
        }
        if (take > room) take = room;  // >= 1: room >= Tc - 1 >= 1 in an empty bin
      }
      const uint64_t d0 = first * L;
      BReq s = to_breq(q);
      const unsigned __int128 off = ((unsigned __int128)q.offset.hi << 64 | q.offset.lo) + d0;
      s.off_lo = (uint64_t)off;
      s.off_hi = (uint64_t)(off >> 64);
      s.count = std::min<uint64_t>(q.count - d0, take * L);
      s.out += 4 * d0;
      s.state = (first + take == nq) ? s.state : 0;
      const uint32_t local = nsc[x]++;
      for (uint64_t k = 0; k < take; ++k, ++nc) {
        ch[nc].req = local;
        ch[nc].q = (uint32_t)k;
        const uint64_t rem = s.count - k * L;
        ch[nc].draws = (uint32_t)(rem < L ? rem : L);
        ch[nc].last = (k + 1 == take) ? 1u : 0u;
      }
      nkb[x] += (uint32_t)take;
      tmp.push_back(s);
      fill += 1 + take;
      first += take;
    }
  }
  // Slice table: per bin, its slices with draws, then its share of the
  // requests without draws (an equal split, in order).
  const bool octets = b->B.wtab20 != nullptr && bv != BATCH_PAIRS;
  const uint32_t grid_cap = bv == BATCH_HALF_GRID ? b->workers_max / 2 : bv == BATCH_QUARTER_GRID ? b->workers_max / 4
                                                                                                   : b->workers_max;
  const uint32_t wpb_max = std::max<uint32_t>(1, grid_cap / nb);
  // Jump items per dequeue: enough that each of the bin's workers takes
  // about two, at most 8 (16 coarse), or one each (fine).
  auto per_item = [&](uint32_t jobs) -> uint32_t {
    if (fine) return 1u;
    const uint32_t g = std::min<uint32_t>(8, std::max<uint32_t>(1, jobs / (2 * wpb_max)));
    return bv == BATCH_COARSE ? std::min<uint32_t>(16, 2 * g) : g;
  };
  uint64_t ns = 0, ti = 0, k0 = 0;
  uint32_t wpb = 1;
  for (uint32_t i = 0; i < nb; ++i) {
    BBin& bn = bins[i];
    bn.s0 = (uint32_t)ns;
    bn.a0 = (uint32_t)ti;
    bn.na = nsc[i];
    bn.b0 = (uint32_t)(n_jo * i / nb);
    for (uint32_t k = 0; k < nsc[i]; ++k, ++ti) sl[ti] = tmp[ti];  // the table holds tmp in order
    ns += nsc[i];
    ns += n_jo * (i + 1) / nb - n_jo * i / nb;  // filled below
    bn.ns = (uint32_t)(ns - bn.s0);
    bn.nsc = octets ? nsc[i] : bn.ns;  // without the 20-bit table, pair items take every slice
    bn.k0 = (uint32_t)k0;
    bn.nk = nkb[i];
    k0 += nkb[i];
    // Jump pairs and octets are taken several at a time when a bin has many.
    const uint32_t n_jg = (bn.nsc + 1) / 2, n_jq = (bn.ns - bn.nsc + 7) / 8;
    bn.g = per_item(n_jg);
    bn.n_ju = (n_jg + bn.g - 1) / bn.g;
    bn.n_cg = (bn.nk + 1) / 2;
    bn.gq = per_item(n_jq);
    bn.n_qi = (n_jq + bn.gq - 1) / bn.gq;
    // Workgroups per bin: as many as the fullest bin has items, within the device.
    wpb = std::max(wpb, std::min(wpb_max, bn.n_ju + bn.n_cg + bn.n_qi));
  }
  // Requests without draws: the k-th of them (in order) is entry k of their
  // table and belongs to bin i with n_jo i / nb <= k < n_jo (i + 1) / nb,
  // after that bin's slices with draws.
  // A batch of jumps only keeps them at a fixed place (staged above when the
  // first request had no draws); a mixed batch right after its slices.
  const uint64_t jo_off = n_jo == n ? kJumpsOnlyOff : align16(req_off + sizeof(BReq) * ti);
  BJump* jo = (BJump*)(b->h_desc + jo_off);
  if (n_jo && !(n_jo == n && guess_jumps)) {
    std::vector<uint64_t> jo_before(parts, 0);
    for (uint32_t t = 1; t < parts; ++t) jo_before[t] = jo_before[t - 1] + p_jo[t - 1];
    parallel_parts(n, parts, [&](uint64_t lo, uint64_t hi, uint32_t t) {
      uint64_t k = jo_before[t];
      for (uint64_t r = lo; r < hi && k < n_jo; ++r) {
        if (reqs[r].count != 0) continue;
        stage_bjump(jo + k++, reqs[r]);
      }
      stage_fence();
    });
  }
  h->n_bins = nb;
  h->n_workers = direct ? bins[0].n_qi : nb * wpb;
  b->dj_prepared = direct ? DirectJumps{b->h_desc_dev + jo_off, (uint32_t)n, 0u} : DirectJumps{nullptr, 0u, 0u};
  h->epoch = ++b->epoch;
  h->L = b->L;
  h->req_off = req_off;
  h->chunk_off = chunk_off;
  h->jo_off = jo_off;
  b->grid_prepared = h->n_workers;
  b->prepared_bytes = req_off + sizeof(BReq) * ti;  // the device copy: all but the slices without draws
  return RANMAR_OK;
}

int ranmar_batch_launch(ranmar_batch* b, void* stream) {
  if (!b || !b->prepared_bytes) return RANMAR_EINVAL;
  if (*(volatile int*)b->h_err) {
    *(volatile int*)b->h_err = 0;
    b->prepared_bytes = 0;
    return RANMAR_EHIP;
  }
  const size_t bytes = b->prepared_bytes;
  b->prepared_bytes = 0;
  if (b->dj_prepared.n) {
    // Direct mapping: the kernel node alone, its arguments set when they change.
    if (b->grid_prepared != b->grid_dnode || b->dj_prepared.recs != b->kdirect_d.recs ||
        b->dj_prepared.n != b->kdirect_d.n) {
      b->kdirect = b->dj_prepared;
      const hipKernelNodeParams kp = kernel_params(b, b->grid_prepared, true);
      if (hipGraphExecKernelNodeSetParams(b->exec_d, b->kern_d, &kp) != hipSuccess) return RANMAR_EHIP;
      b->kdirect_d = b->dj_prepared;
      b->grid_dnode = b->grid_prepared;
    }
    if (hipGraphLaunch(b->exec_d, (hipStream_t)stream) != hipSuccess) return RANMAR_EHIP;
  } else {
    if (hipGraphExecMemcpyNodeSetParams1D(b->exec, b->cpy, b->d_desc, b->h_desc, bytes, hipMemcpyHostToDevice) !=
        hipSuccess)
      return RANMAR_EHIP;
    if (b->grid_prepared != b->grid_node) {
      b->kdirect = DirectJumps{nullptr, 0u, 0u};
      const hipKernelNodeParams kp = kernel_params(b, b->grid_prepared, false);
      if (hipGraphExecKernelNodeSetParams(b->exec, b->kern, &kp) != hipSuccess) return RANMAR_EHIP;
      b->grid_node = b->grid_prepared;
    }
    if (hipGraphLaunch(b->exec, (hipStream_t)stream) != hipSuccess) return RANMAR_EHIP;
  }
  if (hipEventRecord(b->last, (hipStream_t)stream) != hipSuccess) return RANMAR_EHIP;
  b->launched = true;
  return RANMAR_OK;
}

int ranmar_batch_run(ranmar_batch* b, const ranmar_request* reqs, uint64_t n, void* stream) {
  if (!b || (n && !reqs)) return RANMAR_EINVAL;
  if (n == 0) return n > b->max_req ? RANMAR_ENOMEM : RANMAR_OK;
  const int rc = ranmar_batch_prepare(b, reqs, n);
  if (rc) return rc;
  return ranmar_batch_launch(b, stream);
}

int ranmar_batch_destroy(ranmar_batch* b) {
  if (!b) return RANMAR_EINVAL;
  batch_free(b);
  return RANMAR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One launch per request
// ---------------------------------------------------------------------------
namespace ranmar {
namespace {
struct UnbatchedCtx {
  uint64_t cap_chunks = 0;
  uint32_t *req_states = nullptr, *done = nullptr, *queue = nullptr, *ptab = nullptr;
  int* err = nullptr;
  uint32_t epoch = 0;
};
std::mutex g_ub_mu;
std::map<std::pair<int, uintptr_t>, UnbatchedCtx> g_ub;

int ub_reserve(UnbatchedCtx& c, uint64_t nq, hipStream_t st) {
  if (!c.req_states) {
    if (hipMalloc(&c.req_states, 4 * kWords) != hipSuccess || hipMalloc(&c.done, 8) != hipSuccess ||
        hipMalloc(&c.queue, 8) != hipSuccess ||
        hipHostMalloc(&c.err, sizeof(int), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
      return RANMAR_EHIP;
    *c.err = 0;
    if (hipMemsetAsync(c.done, 0, 8, st) != hipSuccess || hipMemsetAsync(c.queue, 0, 8, st) != hipSuccess)
      return RANMAR_EHIP;
  }
  if (nq > c.cap_chunks) {
    uint64_t cap = c.cap_chunks ? c.cap_chunks : 64;
    while (cap < nq) cap *= 2;
    if (hipStreamSynchronize(st) != hipSuccess) return RANMAR_EHIP;
    hipFree(c.ptab);
    c.ptab = nullptr;
    c.cap_chunks = 0;
    if (hipMalloc(&c.ptab, 4 * 97 * cap) != hipSuccess) return RANMAR_ENOMEM;
    if (fill_ptab(c.ptab, cap, kUnbatchedChunk, st) != hipSuccess) return RANMAR_EHIP;
    c.cap_chunks = cap;
  }
  return RANMAR_OK;
}
}  // namespace
}  // namespace ranmar

extern "C" int ranmar_run_unbatched(const ranmar_request* reqs, uint64_t n, void* stream) {
  if (n && !reqs) return RANMAR_EINVAL;
  if (n == 0) return RANMAR_OK;
  int rc = ensure_init();
  if (rc) return rc;
  for (uint64_t r = 0; r < n; ++r) {
    uint64_t nq = 0;
    rc = check_request(reqs[r], kUnbatchedChunk, &nq);
    if (rc) return rc;
  }
  int dev = 0;
  hipGetDevice(&dev);
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> g(g_ub_mu);
  UnbatchedCtx& c = g_ub[{dev, (uintptr_t)stream}];
  if (c.err && *(volatile int*)c.err) {
    *(volatile int*)c.err = 0;
    return RANMAR_EHIP;
  }
  const unsigned maxgrid = persistent_grid((const void*)k_batch_single, 64);
  for (uint64_t r = 0; r < n; ++r) {
    const uint64_t nq = (reqs[r].count + kUnbatchedChunk - 1) / kUnbatchedChunk;
    rc = ub_reserve(c, nq ? nq : 1, st);
    if (rc) return rc;
    SingleDesc d;
    d.r0 = to_breq(reqs[r]);
    d.L = kUnbatchedChunk;
    d.epoch = ++c.epoch;
    BatchBuffers B{c.req_states, c.done, c.ptab, window_table(), window20_table_ready(), nullptr, c.queue, c.err, 1u};
    if (!B.wtab) return RANMAR_ENOMEM;
    const uint64_t items = 1 + (nq + 1) / 2;
    const unsigned grid = (unsigned)(items < maxgrid ? items : maxgrid);
    hipLaunchKernelGGL(k_batch_single, dim3(grid), dim3(64), 0, st, d, B);
    if (hipGetLastError() != hipSuccess) return RANMAR_EHIP;
  }
  return RANMAR_OK;
}
