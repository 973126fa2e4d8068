// Batched execution of uneven requests in one persistent launch (host side).
//
// ranmar_batch_run: the request and chunk tables are written to a pinned host
// staging buffer and the run is one launch of a captured graph
//     [memcpy staging -> device tables]  ->  [persistent kernel]
// whose memcpy size is set per run; the kernel's arguments never change (they
// point at the batch's own device buffers), so the graph is built once.
//
// ranmar_run_unbatched: the same kernel launched once per request with the
// request passed by value (no tables, no graph): the baseline the batched path
// is measured against.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ranmar.h"
#include "batch_dev.hpp"
#include "internal.hpp"

namespace ranmar {

__global__ __launch_bounds__(64) void k_batch_tables(const uint8_t* __restrict__ desc, BatchBuffers B) {
  batch_persistent(TableDesc{desc}, B);
}

__global__ __launch_bounds__(64) void k_batch_single(SingleDesc d, BatchBuffers B) { batch_persistent(d, B); }

constexpr uint32_t kDefaultChunk = 16384;
constexpr uint32_t kMaxChunkDraws = 1u << 24;

// Workgroups that fit the device at once (the kernel's occupancy times the
// number of CUs): every workgroup of the persistent grid is resident.
static unsigned persistent_grid() {
  int dev = 0, cus = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch_tables, 64, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 8;
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
  *nq = (q.count + L - 1) / L;
  return RANMAR_OK;
}

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
  uint64_t max_req = 0, max_chunks = 0;
  uint32_t L = kDefaultChunk;
  size_t desc_cap = 0;
  uint8_t* d_desc = nullptr;
  uint8_t* h_desc = nullptr;
  uint32_t *d_req_states = nullptr, *d_done = nullptr, *d_queue = nullptr, *d_ptab = nullptr;
  int* h_err = nullptr;
  uint32_t epoch = 0;
  unsigned grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t cpy = nullptr, kern = nullptr;
  hipEvent_t last = nullptr;
  bool launched = false;
  size_t prepared_bytes = 0;  // descriptor bytes staged by prepare, 0 = none
  BatchBuffers B{};
  const uint8_t* kdesc = nullptr;  // kernel argument storage for the graph node
};

static void batch_free(ranmar_batch* b) {
  if (!b) return;
  if (b->last) hipEventSynchronize(b->last);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
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

extern "C" {

int ranmar_batch_create(uint64_t max_requests, uint64_t max_chunks, uint64_t chunk_draws, ranmar_batch** out) {
  if (!out || max_requests == 0 || max_requests > (1ull << 26) || max_chunks > (1ull << 26)) return RANMAR_EINVAL;
  if (chunk_draws > kMaxChunkDraws) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  ranmar_batch* b = new ranmar_batch();
  b->max_req = max_requests;
  b->max_chunks = max_chunks ? max_chunks : 1;
  b->L = chunk_draws ? (uint32_t)chunk_draws : kDefaultChunk;
  b->desc_cap = 64 + sizeof(BReq) * b->max_req + 16 + sizeof(BChunk) * b->max_chunks;
  b->grid = persistent_grid();
  const uint64_t ngroups = b->max_req + 1;  // request flags + the spare
  hipStream_t st = nullptr;
  bool ok = hipMalloc(&b->d_desc, b->desc_cap) == hipSuccess &&
            hipHostMalloc(&b->h_desc, b->desc_cap, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(&b->h_err, sizeof(int), hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
            hipMalloc(&b->d_req_states, 4 * kWords * b->max_req) == hipSuccess &&
            hipMalloc(&b->d_done, 4 * ngroups) == hipSuccess && hipMalloc(&b->d_queue, 8) == hipSuccess &&
            hipMalloc(&b->d_ptab, 4 * 97 * b->max_chunks) == hipSuccess && hipEventCreate(&b->last) == hipSuccess;
  if (ok) {
    *b->h_err = 0;
    ok = hipMemset(b->d_done, 0, 4 * ngroups) == hipSuccess && hipMemset(b->d_queue, 0, 8) == hipSuccess &&
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
    b->B.spare = (uint32_t)b->max_req;
    ok = b->B.wtab != nullptr;
  }
  if (ok) {
    b->kdesc = b->d_desc;
    ok = hipGraphCreate(&b->graph, 0) == hipSuccess &&
         hipGraphAddMemcpyNode1D(&b->cpy, b->graph, nullptr, 0, b->d_desc, b->h_desc, b->desc_cap,
                                 hipMemcpyHostToDevice) == hipSuccess;
    if (ok) {
      hipKernelNodeParams kp{};
      void* args[] = {(void*)&b->kdesc, (void*)&b->B};
      kp.func = (void*)k_batch_tables;
      kp.gridDim = dim3(b->grid);
      kp.blockDim = dim3(64);
      kp.sharedMemBytes = 0;
      kp.kernelParams = args;
      kp.extra = nullptr;
      ok = hipGraphAddKernelNode(&b->kern, b->graph, &b->cpy, 1, &kp) == hipSuccess &&
           hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
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
  uint64_t total = 0;
  for (uint64_t r = 0; r < n; ++r) {
    uint64_t nq = 0;
    int rc = check_request(reqs[r], b->L, &nq);
    if (rc) return rc;
    total += nq;
  }
  if (total > b->max_chunks) return RANMAR_ENOMEM;
  const uint64_t chunk_off = (64 + sizeof(BReq) * n + 15) & ~15ull;
  // The staging buffer may still be read by the previous run's copy.
  if (b->launched && hipEventSynchronize(b->last) != hipSuccess) return RANMAR_EHIP;
  BHeader* h = (BHeader*)b->h_desc;
  std::memset(h, 0, sizeof(BHeader));
  h->n_req = (uint32_t)n;
  h->n_jg = (uint32_t)((n + 1) / 2);
  h->n_chunks = (uint32_t)total;
  h->n_cg = (uint32_t)((total + 1) / 2);
  h->epoch = ++b->epoch;
  h->L = b->L;
  h->chunk_off = chunk_off;
  BReq* rq = (BReq*)(b->h_desc + 64);
  BChunk* ch = (BChunk*)(b->h_desc + chunk_off);
  uint64_t j = 0;
  for (uint64_t r = 0; r < n; ++r) {
    rq[r] = to_breq(reqs[r]);
    const uint64_t nq = (reqs[r].count + b->L - 1) / b->L;
    for (uint64_t q = 0; q < nq; ++q, ++j) {
      ch[j].req = (uint32_t)r;
      ch[j].q = (uint32_t)q;
      const uint64_t rem = reqs[r].count - q * b->L;
      ch[j].draws = (uint32_t)(rem < b->L ? rem : b->L);
      ch[j].last = (q + 1 == nq) ? 1u : 0u;
    }
  }
  b->prepared_bytes = chunk_off + sizeof(BChunk) * total;
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
  if (hipGraphExecMemcpyNodeSetParams1D(b->exec, b->cpy, b->d_desc, b->h_desc, bytes, hipMemcpyHostToDevice) !=
      hipSuccess)
    return RANMAR_EHIP;
  if (hipGraphLaunch(b->exec, (hipStream_t)stream) != hipSuccess) return RANMAR_EHIP;
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
    if (fill_ptab(c.ptab, cap, kDefaultChunk, st) != hipSuccess) return RANMAR_EHIP;
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
    rc = check_request(reqs[r], kDefaultChunk, &nq);
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
  const unsigned maxgrid = persistent_grid();
  for (uint64_t r = 0; r < n; ++r) {
    const uint64_t nq = (reqs[r].count + kDefaultChunk - 1) / kDefaultChunk;
    rc = ub_reserve(c, nq ? nq : 1, st);
    if (rc) return rc;
    SingleDesc d;
    d.r0 = to_breq(reqs[r]);
    d.L = kDefaultChunk;
    d.epoch = ++c.epoch;
    BatchBuffers B{c.req_states, c.done, c.ptab, window_table(), c.queue, c.err, 1u};
    if (!B.wtab) return RANMAR_ENOMEM;
    const uint64_t items = 1 + (nq + 1) / 2;
    const unsigned grid = (unsigned)(items < maxgrid ? items : maxgrid);
    hipLaunchKernelGGL(k_batch_single, dim3(grid), dim3(64), 0, st, d, B);
    if (hipGetLastError() != hipSuccess) return RANMAR_EHIP;
  }
  return RANMAR_OK;
}
