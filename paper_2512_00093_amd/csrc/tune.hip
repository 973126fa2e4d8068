// Kernel-variant tuner.  Every variant of a kernel produces the same bits; the
// tuner only records which is fastest for a shape bucket, measured with HIP
// events on synthetic states at the real shape.  The table can be saved to and
// loaded from a small text file ("kernel log2n log2count variant" per line).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/ranmar.h"
#include "common.hpp"
#include "internal.hpp"

namespace ranmar {

namespace {
std::mutex g_mu;
int g_forced[6] = {-1, -1, -1, -1, -1, -1};
int g_chunk_pick = -1;  // last tuned or loaded RANMAR_K_CHUNK variant
std::map<std::tuple<int, int, int>, int> g_table;  // (kernel, log2 n, log2 count) -> variant

int ilog2(uint64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

constexpr int kJumpVariants = JUMP_NUM_VARIANTS;
}  // namespace

int jump_variant_for(uint64_t n) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_forced[RANMAR_K_JUMP] >= 0) return g_forced[RANMAR_K_JUMP];
  auto it = g_table.find({RANMAR_K_JUMP, ilog2(n), 0});
  if (it != g_table.end()) return it->second;
  // Many requests: 8 lanes each (most useful multiply-adds per issue) and
  // 20-bit windows (6 applications for a 120-bit J, 2.4 GB table; measured on
  // 10^6 requests: 2.75 ms against 3.19 with 16-bit windows); few: 32 lanes
  // each (a third of the latency per request, more workgroups) and the 1.6 MB
  // table.
  return n >= 16384 ? JUMP_EIGHTH_WINDOW20 : JUMP_HALF_WINDOW;
}

int poly_variant_for(uint64_t n) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_forced[RANMAR_K_POLY] >= 0) return g_forced[RANMAR_K_POLY];
  auto it = g_table.find({RANMAR_K_POLY, ilog2(n), 0});
  if (it != g_table.end()) return it->second;
  // Table products: a fourth of square-and-multiply's multiply-adds for a
  // uniform 120-bit J with the 8-bit table, and one wave per J instead of one
  // lane (latency of one J: microseconds against a millisecond).
  return POLY_TABLE;
}

int family_variant_for(uint64_t n) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_forced[RANMAR_K_FAMILY] >= 0) return g_forced[RANMAR_K_FAMILY];
  auto it = g_table.find({RANMAR_K_FAMILY, ilog2(n), 0});
  if (it != g_table.end()) return it->second;
  // Measured (ms; radix rounds / 16-row product / 32-row product): 16,384
  // starts 0.018 / 0.017 / 0.022; 65,536: 0.035 / 0.025 / 0.022; 262,144:
  // 0.106 / 0.044 / 0.044; 2^20: 0.35 / 0.148 / 0.168 (the 32-row kernel
  // holds two waves per SIMD, the 16-row one four).
  if (n < 32768) return FAMILY_RADIX;
  return n < 524288 ? FAMILY_GEMM32 : FAMILY_GEMM;
}

int batch_variant_for(uint64_t n, uint64_t draws_per_request) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_forced[RANMAR_K_BATCH] >= 0) return g_forced[RANMAR_K_BATCH];
  auto it = g_table.find({RANMAR_K_BATCH, ilog2(n), ilog2(draws_per_request + 1)});
  if (it != g_table.end()) return it->second;
  // Batches of jumps only: the direct mapping (it falls back to BATCH_AUTO
  // where it does not apply).  10^6 requests, 120-bit offsets: 2.62-2.70 ms
  // against 2.79-2.90 ms for the best queue mapping.
  return draws_per_request == 0 ? BATCH_DIRECT : BATCH_AUTO;
}

uint32_t chunk_draws_default(uint32_t fallback) {
  std::lock_guard<std::mutex> g(g_mu);
  const int v = g_forced[RANMAR_K_CHUNK] >= 0 ? g_forced[RANMAR_K_CHUNK] : g_chunk_pick;
  return v >= 0 ? chunk_variant_draws(v) : fallback;
}

int gen_variant_for(uint64_t n, uint64_t count) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_forced[RANMAR_K_GENERATE] >= 0) return g_forced[RANMAR_K_GENERATE];
  auto it = g_table.find({RANMAR_K_GENERATE, ilog2(n), ilog2(count)});
  if (it != g_table.end()) return it->second;
  // Measured (float32, ms per launch): 2^20 streams x 1,024 draws: 16-byte
  // stores, neighbouring streams on different XCDs, 16 half-waves per
  // workgroup with at most 3 workgroups per CU 0.71-0.73, at most 2 0.74-0.75,
  // 4 0.74; 8 half-waves per workgroup with at most 5 per CU 0.755-0.76, 6
  // 0.765-0.77, 7 0.80, 4 0.82, uncapped 0.83; 32 half-waves 0.76-0.78; 65,536 x
  // 4,096: 4-byte stores with at most 2 workgroups per CU 0.172, uncapped
  // 0.190; 16,384 x 16,384 (every workgroup resident at once anyway):
  // ordinary 16-byte stores 0.203, the capped forms 0.21-0.23.  The wide
  // forms fall back to 4-byte stores for unaligned rows.
  if (count <= 2048) return GEN_WIDE16_NT_R3;
  return n >= 32768 ? GEN_LANES32_NT_R2 : GEN_WIDE4;
}

// Times every variant in `rounds` passes over all of them (so that slow
// drifts of clock or memory state hit each alike), `reps` launches per pass
// after one untimed launch, and keeps each variant's best pass.  Returns the
// fastest variant, or -1 on a HIP error.
template <class Run>
static int time_variants(int nv, Run run, double* ms_out, hipEvent_t e0, hipEvent_t e1, hipStream_t st,
                         int reps = 5, int rounds = 3) {
  std::vector<double> best(nv, 1e30);
  for (int rd = 0; rd < rounds; ++rd)
    for (int v = 0; v < nv; ++v) {
      if (run(v) != hipSuccess) return -1;
      hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r)
        if (run(v) != hipSuccess) return -1;
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) return -1;
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      best[v] = std::min(best[v], (double)ms / reps);
    }
  int bv = 0;
  for (int v = 0; v < nv; ++v) {
    if (ms_out) ms_out[v] = best[v];
    if (best[v] < best[bv]) bv = v;
  }
  return bv;
}

// Times the t^J mod phi variants on n uniform `bits`-bit exponents.
static int tune_poly(uint64_t n, int bits, double* ms_out, hipStream_t st) {
  if (n > (1ull << 24) || bits < 1 || bits > 128) return RANMAR_EINVAL;
  std::vector<ranmar_u128> J(n);
  uint64_t x = 0x2545F4914F6CDD1Dull;
  for (uint64_t i = 0; i < n; ++i) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    const uint64_t lo = x * 0x9E3779B97F4A7C15ull, hi = x;
    J[i].lo = bits >= 64 ? lo : lo & ((1ull << bits) - 1);
    J[i].hi = bits > 64 ? (bits == 128 ? hi : hi & ((1ull << (bits - 64)) - 1)) : 0;
  }
  ranmar_u128* d_J = nullptr;
  uint32_t* d_P = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = RANMAR_EHIP;
  int best_v = 0;
  if (hipMalloc(&d_J, 16 * n) != hipSuccess || hipMalloc(&d_P, 388 * n) != hipSuccess) goto done;
  if (hipMemcpyAsync(d_J, J.data(), 16 * n, hipMemcpyHostToDevice, st) != hipSuccess) goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  best_v = time_variants(
      POLY_NUM_VARIANTS,
      [&](int v) { return v == POLY_TABLE ? launch_jump_poly_tab(d_J, n, d_P, st) : launch_jump_poly(d_J, n, d_P, st); },
      ms_out, e0, e1, st, 3, 2);
  if (best_v < 0) goto done;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_table[{RANMAR_K_POLY, ilog2(n), 0}] = best_v;
  }
  rc = best_v;
done:
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(st);
  hipFree(d_P);
  hipFree(d_J);
  return rc;
}

// Times the jump variants on n seed+jump requests with `bits`-bit offsets.
static int tune_jump(uint64_t n, int bits, double* ms_out, hipStream_t st) {
  if (n > (1ull << 24) || bits < 1 || bits > 128) return RANMAR_EINVAL;
  std::vector<int32_t> seeds(n);
  std::vector<ranmar_u128> J(n);
  uint64_t x = 0x9E3779B97F4A7C15ull;
  auto next = [&x] {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
  };
  for (uint64_t i = 0; i < n; ++i) {
    seeds[i] = (int32_t)(1 + next() % 900000000ull);
    const uint64_t lo = next(), hi = next();
    J[i].lo = bits >= 64 ? lo : (bits == 64 ? lo : lo & ((1ull << bits) - 1));
    J[i].hi = bits > 64 ? (bits == 128 ? hi : hi & ((1ull << (bits - 64)) - 1)) : 0;
  }
  int32_t* d_seeds = nullptr;
  ranmar_u128* d_J = nullptr;
  uint32_t* d_states = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = RANMAR_EHIP;
  int best_v = 0;
  if (hipMalloc(&d_seeds, 4 * n) != hipSuccess || hipMalloc(&d_J, 16 * n) != hipSuccess ||
      hipMalloc(&d_states, sizeof(ranmar_state) * n) != hipSuccess)
    goto done;
  if (hipMemcpyAsync(d_seeds, seeds.data(), 4 * n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_J, J.data(), 16 * n, hipMemcpyHostToDevice, st) != hipSuccess)
    goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  best_v = time_variants(
      JUMP_NUM_VARIANTS, [&](int v) { return launch_jump_variant(v, d_states, d_seeds, d_J, n, st); }, ms_out, e0,
      e1, st, 3, 2);
  if (best_v < 0) goto done;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_table[{RANMAR_K_JUMP, ilog2(n), 0}] = best_v;
  }
  rc = best_v;
done:
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(st);
  hipFree(d_states);
  hipFree(d_J);
  hipFree(d_seeds);
  return rc;
}

// Times the family variants on n starts at spacing 2^lg from seed 1.
static int tune_family(uint64_t n, int lg, double* ms_out, hipStream_t st) {
  if (n < 2 || n > (1ull << 24) || lg < 0 || lg > 100) return RANMAR_EINVAL;
  ranmar_state h{};
  if (ranmar_seed(1, &h) != RANMAR_OK) return RANMAR_EINVAL;
  const unsigned __int128 d = (unsigned __int128)1 << lg;
  const ranmar_u128 delta{(uint64_t)d, (uint64_t)(d >> 64)};
  uint32_t *d_base = nullptr, *d_out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = RANMAR_EHIP;
  int best_v = 0;
  if (hipMalloc(&d_base, sizeof(ranmar_state)) != hipSuccess ||
      hipMalloc(&d_out, sizeof(ranmar_state) * n) != hipSuccess)
    goto done;
  if (hipMemcpyAsync(d_base, &h, sizeof h, hipMemcpyHostToDevice, st) != hipSuccess) goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  best_v = time_variants(
      FAMILY_NUM_VARIANTS, [&](int v) { return launch_family_variant(v, d_base, delta, n, d_out, st); }, ms_out, e0,
      e1, st);
  if (best_v < 0) goto done;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_table[{RANMAR_K_FAMILY, ilog2(n), 0}] = best_v;
  }
  rc = best_v;
done:
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(st);
  hipFree(d_out);
  hipFree(d_base);
  return rc;
}

// A batch of n requests of `count` draws each (uniform 120-bit offsets,
// pseudo-random seeds; every request also returns its final state), for the
// batch and chunk tuners.  Owns its device buffers.
struct TuneBatch {
  std::vector<ranmar_request> reqs;
  uint8_t* d_out = nullptr;
  uint32_t* d_states = nullptr;
  bool ok = false;
  TuneBatch(uint64_t n, uint64_t count) : reqs(n) {
    if (hipMalloc(&d_states, sizeof(ranmar_state) * n) != hipSuccess) return;
    if (count && hipMalloc(&d_out, 4 * n * count) != hipSuccess) return;
    uint64_t x = 0x2545F4914F6CDD1Dull;
    auto next = [&x] {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      return x;
    };
    for (uint64_t i = 0; i < n; ++i) {
      ranmar_request& q = reqs[i];
      q.seed = (int32_t)(1 + next() % 900000000ull);
      q.fmt = RANMAR_F32;
      q.offset.lo = next();
      q.offset.hi = next() & ((1ull << 56) - 1);
      q.count = count;
      q.d_out = count ? d_out + 4 * i * count : nullptr;
      q.d_state = (ranmar_state*)(d_states + (uint64_t)kWords * i);
    }
    ok = true;
  }
  ~TuneBatch() {
    hipDeviceSynchronize();
    if (d_out) hipFree(d_out);
    if (d_states) hipFree(d_states);
  }
};

// Device time of one prepared launch of `b` (ms), the best of `rounds`
// passes of `reps` launches after one untimed launch; each launch is timed
// alone (its host preparation is outside the events).
static double time_batch(ranmar_batch* b, const TuneBatch& tb, hipEvent_t e0, hipEvent_t e1, hipStream_t st,
                         int reps) {
  double sum = 0;
  for (int r = -1; r < reps; ++r) {
    if (ranmar_batch_prepare(b, tb.reqs.data(), tb.reqs.size()) != RANMAR_OK) return -1;
    if (hipEventRecord(e0, st) != hipSuccess) return -1;
    if (ranmar_batch_launch(b, st) != RANMAR_OK) return -1;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1;
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    if (r >= 0) sum += ms;
  }
  return sum / reps;
}

// Two prepared launches, of b1 on st and of b2 on st2, started together and
// timed to the end of both: half of that is the time per batch when a
// server's launches overlap on several streams.  Best of `rounds`, each
// after the untimed first; ms per batch.
static double time_batch_pair(ranmar_batch* b1, ranmar_batch* b2, const TuneBatch& t1, const TuneBatch& t2,
                              hipEvent_t e0, hipEvent_t e1, hipEvent_t e2, hipStream_t st, hipStream_t st2,
                              int reps) {
  double sum = 0;
  for (int r = -1; r < reps; ++r) {
    if (ranmar_batch_prepare(b1, t1.reqs.data(), t1.reqs.size()) != RANMAR_OK ||
        ranmar_batch_prepare(b2, t2.reqs.data(), t2.reqs.size()) != RANMAR_OK)
      return -1;
    if (hipEventRecord(e0, st) != hipSuccess || hipStreamWaitEvent(st2, e0, 0) != hipSuccess) return -1;
    if (ranmar_batch_launch(b1, st) != RANMAR_OK || ranmar_batch_launch(b2, st2) != RANMAR_OK) return -1;
    if (hipEventRecord(e2, st2) != hipSuccess || hipStreamWaitEvent(st, e2, 0) != hipSuccess) return -1;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1;
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    if (r >= 0) sum += ms / 2;
  }
  return sum / reps;
}

// A second stream and event for the overlapped timing (default priority).
struct PairTiming {
  hipStream_t st2 = nullptr;
  hipEvent_t e2 = nullptr;
  bool ok = false;
  PairTiming() {
    ok = hipStreamCreateWithFlags(&st2, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e2) == hipSuccess;
  }
  ~PairTiming() {
    if (st2) hipStreamSynchronize(st2);
    if (e2) hipEventDestroy(e2);
    if (st2) hipStreamDestroy(st2);
  }
};

static bool batch_shape_ok(uint64_t n, uint64_t count) {
  return n >= 1 && n <= (1ull << 22) && count <= (1ull << 24) && n * count <= (1ull << 31);
}

// Times the batch executor's mappings on a batch of the given shape.  A
// batch with draws (a server's launch) is timed as two launches overlapping
// on two streams, as a server's launches do; jumps only, alone.
static int tune_batch(uint64_t n, uint64_t count, double* ms_out, hipStream_t st) {
  if (!batch_shape_ok(n, count)) return RANMAR_EINVAL;
  const bool pair = count > 0;
  TuneBatch tb(n, count);
  if (!tb.ok) return RANMAR_ENOMEM;
  std::unique_ptr<TuneBatch> tb2(pair ? new TuneBatch(n, count) : nullptr);
  if (pair && !tb2->ok) return RANMAR_ENOMEM;
  PairTiming pt;
  if (!pt.ok) return RANMAR_EHIP;
  const uint32_t L = 8192;  // the server's chunk length (the mapping hardly depends on it)
  ranmar_batch *b = nullptr, *b2 = nullptr;
  int rc = ranmar_batch_create(n, n * ((count + L - 1) / L) + 1, L, &b);
  if (rc) return rc;
  if (pair && (rc = ranmar_batch_create(n, n * ((count + L - 1) / L) + 1, L, &b2)) != RANMAR_OK) {
    ranmar_batch_destroy(b);
    return rc;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<double> best(BATCH_NUM_VARIANTS, 1e30);
  rc = RANMAR_EHIP;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    rc = RANMAR_OK;
    for (int rd = 0; rd < 2 && rc == RANMAR_OK; ++rd)
      for (int v = 0; v < BATCH_NUM_VARIANTS; ++v) {
        batch_set_variant(b, v);
        batch_set_variant(b2, v);
        const double ms = pair ? time_batch_pair(b, b2, tb, *tb2, e0, e1, pt.e2, st, pt.st2, 2)
                               : time_batch(b, tb, e0, e1, st, 2);
        if (ms < 0) {
          rc = RANMAR_EHIP;
          break;
        }
        best[v] = std::min(best[v], ms);
      }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  ranmar_batch_destroy(b);
  if (b2) ranmar_batch_destroy(b2);
  if (rc) return rc;
  int bv = 0;
  for (int v = 0; v < BATCH_NUM_VARIANTS; ++v) {
    if (ms_out) ms_out[v] = best[v];
    if (best[v] < best[bv]) bv = v;
  }
  std::lock_guard<std::mutex> g(g_mu);
  g_table[{RANMAR_K_BATCH, ilog2(n), ilog2(count + 1)}] = bv;
  return bv;
}

// Times the chunk lengths: batch executors of each length, each running the
// batch with its tuned (or default) mapping, two launches overlapping on two
// streams as a server's do.
static int tune_chunk(uint64_t n, uint64_t count, double* ms_out, hipStream_t st) {
  if (!batch_shape_ok(n, count) || count == 0) return RANMAR_EINVAL;
  TuneBatch tb(n, count);
  if (!tb.ok) return RANMAR_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return RANMAR_EHIP;
  }
  std::vector<double> best(kChunkVariants, 1e30);
  TuneBatch tb2(n, count);
  PairTiming pt;
  int rc = (tb2.ok && pt.ok) ? RANMAR_OK : RANMAR_ENOMEM;
  for (int rd = 0; rd < 2 && rc == RANMAR_OK; ++rd)
    for (int v = 0; v < kChunkVariants && rc == RANMAR_OK; ++v) {
      const uint32_t L = chunk_variant_draws(v);
      ranmar_batch *b = nullptr, *b2 = nullptr;
      rc = ranmar_batch_create(n, n * ((count + L - 1) / L) + 1, L, &b);
      if (rc) break;
      rc = ranmar_batch_create(n, n * ((count + L - 1) / L) + 1, L, &b2);
      if (rc) {
        ranmar_batch_destroy(b);
        break;
      }
      const double ms = time_batch_pair(b, b2, tb, tb2, e0, e1, pt.e2, st, pt.st2, 2);
      ranmar_batch_destroy(b);
      ranmar_batch_destroy(b2);
      if (ms < 0) rc = RANMAR_EHIP;
      else best[v] = std::min(best[v], ms);
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  int bv = 0;
  for (int v = 0; v < kChunkVariants; ++v) {
    if (ms_out) ms_out[v] = best[v];
    if (best[v] < best[bv]) bv = v;
  }
  std::lock_guard<std::mutex> g(g_mu);
  g_table[{RANMAR_K_CHUNK, ilog2(n), ilog2(count + 1)}] = bv;
  g_chunk_pick = bv;
  return bv;
}

}  // namespace ranmar

using namespace ranmar;

extern "C" {

int ranmar_tune_variants(int kernel) {
  if (kernel == RANMAR_K_GENERATE) return GEN_NUM_VARIANTS;
  if (kernel == RANMAR_K_JUMP) return kJumpVariants;
  if (kernel == RANMAR_K_FAMILY) return FAMILY_NUM_VARIANTS;
  if (kernel == RANMAR_K_BATCH) return BATCH_NUM_VARIANTS;
  if (kernel == RANMAR_K_CHUNK) return kChunkVariants;
  if (kernel == RANMAR_K_POLY) return POLY_NUM_VARIANTS;
  return RANMAR_EINVAL;
}

const char* ranmar_tune_variant_name(int kernel, int variant) {
  if (kernel == RANMAR_K_GENERATE && variant >= 0 && variant < GEN_NUM_VARIANTS) return gen_variant_name(variant);
  if (kernel == RANMAR_K_JUMP && variant == JUMP_LANE_SQMUL) return "lane_square_multiply";
  if (kernel == RANMAR_K_JUMP && variant == JUMP_HALF_WINDOW) return "halfwave_window8";
  if (kernel == RANMAR_K_JUMP && variant == JUMP_QUARTER_WINDOW) return "lanes16_window8";
  if (kernel == RANMAR_K_JUMP && variant == JUMP_EIGHTH_WINDOW) return "lanes8_window8";
  if (kernel == RANMAR_K_JUMP && variant == JUMP_EIGHTH_WINDOW16) return "lanes8_window16";
  if (kernel == RANMAR_K_JUMP && variant == JUMP_EIGHTH_WINDOW20) return "lanes8_window20";
  if (kernel == RANMAR_K_JUMP && variant == JUMP_EIGHTH_WINDOW24) return "lanes8_window24";
  if (kernel == RANMAR_K_FAMILY && variant == FAMILY_RADIX) return "radix256_valu";
  if (kernel == RANMAR_K_FAMILY && variant == FAMILY_GEMM) return "product_mfma_i8";
  if (kernel == RANMAR_K_FAMILY && variant == FAMILY_GEMM32) return "product_mfma32_i8";
  static const char* const kBatchNames[BATCH_NUM_VARIANTS] = {"bins64_auto", "bins64_fine",    "bins64_coarse",
                                                               "bins16_auto", "bins16_fine",    "bins64_pairs",
                                                               "half_grid",   "quarter_grid",  "direct_jumps"};
  if (kernel == RANMAR_K_BATCH && variant >= 0 && variant < BATCH_NUM_VARIANTS) return kBatchNames[variant];
  static const char* const kChunkNames[kChunkVariants] = {"chunk4096", "chunk8192", "chunk16384", "chunk32768"};
  if (kernel == RANMAR_K_CHUNK && variant >= 0 && variant < kChunkVariants) return kChunkNames[variant];
  if (kernel == RANMAR_K_POLY && variant == POLY_LANE_SQMUL) return "lane_square_multiply";
  if (kernel == RANMAR_K_POLY && variant == POLY_TABLE) return "window_products";
  return nullptr;
}

int ranmar_tune_pick(int kernel, uint64_t n, uint64_t count) {
  if (ranmar_tune_variants(kernel) < 0 || n == 0) return RANMAR_EINVAL;
  if (kernel == RANMAR_K_GENERATE) return gen_variant_for(n, count);
  if (kernel == RANMAR_K_JUMP) return jump_variant_for(n);
  if (kernel == RANMAR_K_FAMILY) return family_variant_for(n);
  if (kernel == RANMAR_K_BATCH) return batch_variant_for(n, count);
  if (kernel == RANMAR_K_POLY) return poly_variant_for(n);
  std::lock_guard<std::mutex> g(g_mu);  // RANMAR_K_CHUNK: forced, tuned, else 16,384 draws
  return g_forced[RANMAR_K_CHUNK] >= 0 ? g_forced[RANMAR_K_CHUNK] : g_chunk_pick >= 0 ? g_chunk_pick : 2;
}

int ranmar_tune_set(int kernel, int variant) {
  const int nv = ranmar_tune_variants(kernel);
  if (nv < 0 || variant < -1 || variant >= nv) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(g_mu);
  g_forced[kernel] = variant;
  return RANMAR_OK;
}

int ranmar_tune_run(int kernel, uint64_t n, uint64_t count, double* ms_out, void* stream) {
  const int nv = ranmar_tune_variants(kernel);
  if (nv < 0 || n == 0) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (kernel == RANMAR_K_JUMP) return tune_jump(n, count ? (int)count : 120, ms_out, st);
  if (kernel == RANMAR_K_FAMILY) return tune_family(n, count ? (int)count : 40, ms_out, st);
  if (kernel == RANMAR_K_BATCH) return tune_batch(n, count, ms_out, st);
  if (kernel == RANMAR_K_CHUNK) return tune_chunk(n, count, ms_out, st);
  if (kernel == RANMAR_K_POLY) return tune_poly(n, count ? (int)count : 120, ms_out, st);
  if (count == 0 || n > (1ull << 24) || count > (1ull << 24) || n * count > (1ull << 31)) return RANMAR_EINVAL;
  // Synthetic states: seeds 1..n at offset 0.
  int32_t* d_seeds = nullptr;
  uint32_t* d_states = nullptr;
  float* d_out = nullptr;
  std::vector<int32_t> seeds(n);
  for (uint64_t i = 0; i < n; ++i) seeds[i] = (int32_t)(1 + (i * 2654435761ull) % 900000000ull);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = RANMAR_EHIP;
  int best_v = 0;
  if (hipMalloc(&d_seeds, 4 * n) != hipSuccess) goto done;
  if (hipMalloc(&d_states, sizeof(ranmar_state) * n) != hipSuccess) goto done;
  if (hipMalloc(&d_out, 4 * n * count) != hipSuccess) goto done;
  if (hipMemcpyAsync(d_seeds, seeds.data(), 4 * n, hipMemcpyHostToDevice, st) != hipSuccess) goto done;
  if (launch_seed(d_seeds, n, d_states, st) != hipSuccess) goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  best_v = time_variants(
      nv, [&](int v) { return launch_generate(v, d_states, nullptr, n, count, RANMAR_F32, d_out, count, st); },
      ms_out, e0, e1, st);
  if (best_v < 0) goto done;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_table[{kernel, ilog2(n), ilog2(count)}] = best_v;
  }
  rc = best_v;
done:
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(st);
  if (d_out) hipFree(d_out);
  if (d_states) hipFree(d_states);
  if (d_seeds) hipFree(d_seeds);
  return rc;
}

int ranmar_tune_clear(int kernel) {
  if (kernel != -1 && ranmar_tune_variants(kernel) < 0) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(g_mu);
  for (auto it = g_table.begin(); it != g_table.end();)
    it = (kernel == -1 || std::get<0>(it->first) == kernel) ? g_table.erase(it) : std::next(it);
  if (kernel == -1 || kernel == RANMAR_K_CHUNK) g_chunk_pick = -1;
  return RANMAR_OK;
}

int ranmar_tune_save(const char* path) {
  if (!path) return RANMAR_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(g_mu);
  std::fprintf(f, "# ranmar tune table: kernel log2n log2count variant\n");
  for (auto& kv : g_table)
    std::fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
  std::fclose(f);
  return RANMAR_OK;
}

int ranmar_tune_load(const char* path) {
  if (!path) return RANMAR_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return RANMAR_ENOENT;
  char line[256];
  std::map<std::tuple<int, int, int>, int> t;
  int chunk = -1;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int k, a, b, v;
    if (std::sscanf(line, "%d %d %d %d", &k, &a, &b, &v) == 4) {
      const int nv = ranmar_tune_variants(k);
      if (nv < 0 || v < 0 || v >= nv) {
        std::fclose(f);
        return RANMAR_EINVAL;
      }
      t[{k, a, b}] = v;
      if (k == RANMAR_K_CHUNK) chunk = v;  // the last chunk line is the pick
    }
  }
  std::fclose(f);
  std::lock_guard<std::mutex> g(g_mu);
  for (auto& kv : t) g_table[kv.first] = kv.second;
  if (chunk >= 0) g_chunk_pick = chunk;
  return RANMAR_OK;
}

}  // extern "C"
