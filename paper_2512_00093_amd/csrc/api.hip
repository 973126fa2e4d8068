// C ABI layer: argument validation, device checks and launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/ranmar.h"
#include "common.hpp"
#include "internal.hpp"

namespace ranmar {

namespace {
constexpr int kMaxDevices = 64;
std::atomic<int> g_dev_ok[kMaxDevices];  // 0 unknown, 1 gfx950, -1 not
}  // namespace

int ensure_init() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RANMAR_ENODEV;
  if (dev < 0 || dev >= kMaxDevices) return RANMAR_ENODEV;
  int ok = g_dev_ok[dev].load(std::memory_order_acquire);
  if (ok == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return RANMAR_EHIP;
    ok = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
    g_dev_ok[dev].store(ok, std::memory_order_release);
  }
  return ok == 1 ? RANMAR_OK : RANMAR_ENODEV;
}

static inline int hip_status(hipError_t e) { return e == hipSuccess ? RANMAR_OK : RANMAR_EHIP; }

static inline bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

static inline bool overlap(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Host-side Algorithm 3 (Appendix A) with the Remainder reading of the
// multiplicative step; u_ii goes to x[97 - ii].
static int seed_host(int64_t seed, ranmar_state* out) {
  if (seed < 1 || seed > 900000000) return RANMAR_EINVAL;
  const uint32_t s1 = (uint32_t)(seed - 1);
  const uint32_t ij = s1 / 30082u, kl = s1 - 30082u * ij;
  uint32_t i = (ij / 177u) % 177u + 2u, j = ij % 177u + 2u;
  uint32_t k = (kl / 169u) % 178u + 1u, l = kl % 169u;
  for (int ii = 1; ii <= 97; ++ii) {
    uint32_t word = 0;
    for (int b = 0; b < 24; ++b) {
      const uint32_t m = (i * j % 179u) * k % 179u;
      i = j;
      j = k;
      k = m;
      l = (53u * l + 1u) % 169u;
      word = (word << 1) | (((l * m) & 63u) >= 32u ? 1u : 0u);
    }
    out->x[97 - ii] = word;
  }
  out->c = kC0;
  return RANMAR_OK;
}

hipError_t launch_family_variant(int v, const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out,
                                 hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  if (v == FAMILY_GEMM || v == FAMILY_GEMM32) e = launch_family_gemm(base, delta, n, out, st, v == FAMILY_GEMM32 ? 32 : 16);
  if (e == hipErrorInvalidValue) e = launch_family_window(base, delta, n, out, st);
  if (e == hipErrorInvalidValue) e = launch_family(base, delta, n, out, st);
  return e;
}

}  // namespace ranmar

using namespace ranmar;

extern "C" {

const char* ranmar_strerror(int status) {
  switch (status) {
    case RANMAR_OK: return "ok";
    case RANMAR_EINVAL: return "invalid argument";
    case RANMAR_ENOMEM: return "request exceeds the memory budget";
    case RANMAR_EAGAIN: return "temporarily full, retry";
    case RANMAR_EHIP: return "HIP runtime error";
    case RANMAR_ENOENT: return "unknown ticket or handle";
    case RANMAR_ETIMEDOUT: return "timed out";
    case RANMAR_ENODEV: return "no gfx950 device";
    case RANMAR_ENOINIT: return "ranmar_init has not been called on this device";
    default: return "unknown status";
  }
}

int ranmar_version(void) { return 10000; }

int ranmar_init(void) {
  const int rc = ensure_init();
  return rc ? rc : noalloc_setup();
}

int ranmar_seed(int64_t seed, ranmar_state* out) {
  if (!out) return RANMAR_EINVAL;
  return seed_host(seed, out);
}

int ranmar_seed_batch(const int32_t* d_seeds, uint64_t n, ranmar_state* d_out, void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_seeds || !d_out || !aligned(d_seeds, 4) || !aligned(d_out, 4)) return RANMAR_EINVAL;
  if (overlap(d_seeds, 4 * n, d_out, sizeof(ranmar_state) * n)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  // Few seeds: 32 lanes per seed (latency); many: one lane per seed (throughput).
  if (n < 4096) return hip_status(launch_seed_coop(d_seeds, n, (uint32_t*)d_out, (hipStream_t)stream));
  return hip_status(launch_seed(d_seeds, n, (uint32_t*)d_out, (hipStream_t)stream));
}

int ranmar_jump_poly(const ranmar_u128* d_J, uint64_t n, uint32_t* d_P, void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_J || !d_P || !aligned(d_J, 8) || !aligned(d_P, 4)) return RANMAR_EINVAL;
  if (overlap(d_J, 16 * n, d_P, 388 * n)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(poly_variant_for(n) == POLY_TABLE ? launch_jump_poly_tab(d_J, n, d_P, (hipStream_t)stream)
                                                      : launch_jump_poly(d_J, n, d_P, (hipStream_t)stream));
}

int ranmar_apply_poly(ranmar_state* d_states, const uint32_t* d_P, uint64_t n, void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_states || !d_P || !aligned(d_states, 4) || !aligned(d_P, 4)) return RANMAR_EINVAL;
  if (overlap(d_states, sizeof(ranmar_state) * n, d_P, 388 * n)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_apply_poly((uint32_t*)d_states, d_P, n, (hipStream_t)stream));
}

int ranmar_jump(ranmar_state* d_states, const ranmar_u128* d_J, uint64_t n, void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_states || !d_J || !aligned(d_states, 4) || !aligned(d_J, 8)) return RANMAR_EINVAL;
  if (overlap(d_states, sizeof(ranmar_state) * n, d_J, 16 * n)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_jump_variant(jump_variant_for(n), (uint32_t*)d_states, nullptr, d_J, n, (hipStream_t)stream));
}

int ranmar_seed_jump(const int32_t* d_seeds, const ranmar_u128* d_offsets, uint64_t n, ranmar_state* d_out,
                     void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_seeds || !d_out || !aligned(d_seeds, 4) || !aligned(d_out, 4)) return RANMAR_EINVAL;
  if (d_offsets && !aligned(d_offsets, 8)) return RANMAR_EINVAL;
  const uint64_t sb = sizeof(ranmar_state) * n;
  if (overlap(d_seeds, 4 * n, d_out, sb) || (d_offsets && overlap(d_offsets, 16 * n, d_out, sb)))
    return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(
      launch_jump_variant(jump_variant_for(n), (uint32_t*)d_out, d_seeds, d_offsets, n, (hipStream_t)stream));
}

int ranmar_jump_family(const ranmar_state* d_base, ranmar_u128 delta, uint64_t n, ranmar_state* d_out,
                       void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_base || !d_out || !aligned(d_base, 4) || !aligned(d_out, 4)) return RANMAR_EINVAL;
  if (d_base != d_out && overlap(d_base, sizeof(ranmar_state), d_out, sizeof(ranmar_state) * n))
    return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_family_variant(family_variant_for(n), (const uint32_t*)d_base, delta, n, (uint32_t*)d_out,
                                          (hipStream_t)stream));
}

int ranmar_jump_family_noalloc(const ranmar_state* d_base, ranmar_u128 delta, uint64_t n, ranmar_state* d_out,
                               void* stream) {
  if (n == 0) return RANMAR_OK;
  if (!d_base || !d_out || !aligned(d_base, 4) || !aligned(d_out, 4)) return RANMAR_EINVAL;
  if (n > RANMAR_NOALLOC_FAMILY_MAX_N) return RANMAR_EINVAL;
  // (n - 1) delta must fit in 128 bits: beyond it the family needs the
  // polynomial path, which allocates.
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  if (n > 1 && D > ~(unsigned __int128)0 / (n - 1)) return RANMAR_EINVAL;
  if (d_base != d_out && overlap(d_base, sizeof(ranmar_state), d_out, sizeof(ranmar_state) * n))
    return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  uint32_t* H = noalloc_scratch();
  if (!H) return RANMAR_ENOINIT;
  const hipStream_t st = (hipStream_t)stream;
  const int v = family_variant_for(n);
  hipError_t e = hipErrorInvalidValue;
  if (v == FAMILY_GEMM || v == FAMILY_GEMM32)
    e = launch_family_gemm_fixed((const uint32_t*)d_base, delta, n, (uint32_t*)d_out, st, v == FAMILY_GEMM32 ? 32 : 16,
                                 H);
  // Too small for the product form: radix rounds of table factors (no scratch).
  if (e == hipErrorInvalidValue) e = launch_family_window((const uint32_t*)d_base, delta, n, (uint32_t*)d_out, st);
  return hip_status(e);
}

int ranmar_rank_streams(int32_t seed, ranmar_u128 J, uint64_t first_rank, uint64_t n_ranks, int discard_first,
                        ranmar_state* d_out, void* stream) {
  if (n_ranks == 0) return RANMAR_OK;
  if (!d_out || !aligned(d_out, 4) || seed < 1 || seed > 900000000 || (discard_first != 0 && discard_first != 1))
    return RANMAR_EINVAL;
  // Offset of the first rank, first_rank * J + discard_first, must fit in 128 bits.
  const unsigned __int128 Jv = ((unsigned __int128)J.hi << 64) | J.lo;
  const unsigned __int128 kMax = ~(unsigned __int128)0;
  if (first_rank && Jv > (kMax - (unsigned)discard_first) / first_rank) return RANMAR_EINVAL;
  const unsigned __int128 E0 = Jv * first_rank + (unsigned)discard_first;
  int rc = ensure_init();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const ranmar_u128 e0{(uint64_t)E0, (uint64_t)(E0 >> 64)};
  const int fv = n_ranks > 1 ? family_variant_for(n_ranks) : FAMILY_RADIX;
  if (fv == FAMILY_GEMM || fv == FAMILY_GEMM32) {
    // Seeding inside the product form's first launch (one launch fewer).
    const hipError_t g =
        launch_family_gemm_seeded(seed, e0, J, n_ranks, (uint32_t*)d_out, st, fv == FAMILY_GEMM32 ? 32 : 16);
    if (g != hipErrorInvalidValue) return hip_status(g);
  }
  hipError_t e = launch_seed_jump_one((uint32_t*)d_out, seed, e0, st);
  if (e == hipSuccess && n_ranks > 1)  // the rest as a family around d_out[0]
    e = launch_family_variant(family_variant_for(n_ranks), (const uint32_t*)d_out, J, n_ranks, (uint32_t*)d_out, st);
  return hip_status(e);
}

int ranmar_generate(const ranmar_state* d_in, ranmar_state* d_state_out, uint64_t n, uint64_t count, int fmt,
                    void* d_out, uint64_t ld, void* stream) {
  if (n == 0) return RANMAR_OK;
  if (fmt != RANMAR_U24 && fmt != RANMAR_F32 && fmt != RANMAR_U24_F32) return RANMAR_EINVAL;
  if (!d_in || !aligned(d_in, 4) || (d_state_out && !aligned(d_state_out, 4))) return RANMAR_EINVAL;
  if (count > 0 && (!d_out || !aligned(d_out, 4) || ld < count)) return RANMAR_EINVAL;
  if (ld > (UINT64_MAX / 8) / n) return RANMAR_EINVAL;
  const uint64_t sb = sizeof(ranmar_state) * n;
  if (d_state_out && d_state_out != d_in && overlap(d_in, sb, d_state_out, sb)) return RANMAR_EINVAL;
  if (count > 0) {
    const uint64_t planes = fmt == RANMAR_U24_F32 ? 2 : 1;
    const uint64_t ob = 4 * (ld * n * (planes - 1) + ld * (n - 1) + count);
    if (overlap(d_out, ob, d_in, sb) || (d_state_out && overlap(d_out, ob, d_state_out, sb))) return RANMAR_EINVAL;
  }
  int rc = ensure_init();
  if (rc) return rc;
  const int variant = gen_variant_for(n, count);
  return hip_status(launch_generate(variant, (const uint32_t*)d_in, (uint32_t*)d_state_out, n, count, fmt, d_out, ld,
                                    (hipStream_t)stream));
}


int ranmar_lfg_check(const ranmar_lfg_params* p) { return lfg_params_ok(p) ? RANMAR_OK : RANMAR_EINVAL; }

int ranmar_lfg_jump_poly(const ranmar_lfg_params* p, const ranmar_u128* d_J, uint64_t n, uint32_t* d_P,
                         void* stream) {
  if (!lfg_params_ok(p)) return RANMAR_EINVAL;
  if (n == 0) return RANMAR_OK;
  if (!d_J || !d_P || !aligned(d_J, 8) || !aligned(d_P, 4)) return RANMAR_EINVAL;
  if (n > (UINT64_MAX / 8) / p->r) return RANMAR_EINVAL;
  if (overlap(d_J, 16 * n, d_P, 4ull * p->r * n)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_lfg_jump(*p, d_J, nullptr, nullptr, d_P, n, (hipStream_t)stream));
}

int ranmar_lfg_jump(const ranmar_lfg_params* p, const uint32_t* d_in, uint32_t* d_out, const ranmar_u128* d_J,
                    uint64_t n, void* stream) {
  if (!lfg_params_ok(p)) return RANMAR_EINVAL;
  if (n == 0) return RANMAR_OK;
  if (!d_in || !d_out || !d_J || !aligned(d_in, 4) || !aligned(d_out, 4) || !aligned(d_J, 8)) return RANMAR_EINVAL;
  if (n > (UINT64_MAX / 8) / (p->r + 1)) return RANMAR_EINVAL;
  const uint64_t sb = 4ull * (p->r + 1) * n;
  if (d_out != d_in && overlap(d_in, sb, d_out, sb)) return RANMAR_EINVAL;
  if (overlap(d_J, 16 * n, d_out, sb) || overlap(d_J, 16 * n, d_in, sb)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_lfg_jump(*p, d_J, d_in, d_out, nullptr, n, (hipStream_t)stream));
}

int ranmar_lfg_jump_family(const ranmar_lfg_params* p, const uint32_t* d_base, ranmar_u128 delta, uint64_t n,
                           uint32_t* d_out, void* stream) {
  if (!lfg_params_ok(p)) return RANMAR_EINVAL;
  if (n == 0) return RANMAR_OK;
  if (!d_base || !d_out || !aligned(d_base, 4) || !aligned(d_out, 4)) return RANMAR_EINVAL;
  if (n > (1ull << 32)) return RANMAR_EINVAL;
  const unsigned __int128 D = ((unsigned __int128)delta.hi << 64) | delta.lo;
  if (n > 1 && D > ~(unsigned __int128)0 / (n - 1)) return RANMAR_EINVAL;
  const uint64_t rec = 4ull * (p->r + 1);
  if (d_base != d_out && overlap(d_base, rec, d_out, rec * n)) return RANMAR_EINVAL;
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_lfg_family(*p, d_base, delta, n, d_out, (hipStream_t)stream));
}

int ranmar_lfg_generate(const ranmar_lfg_params* p, const uint32_t* d_in, uint32_t* d_state_out, uint64_t n,
                        uint64_t count, int fmt, void* d_out, uint64_t ld, void* stream) {
  if (!lfg_params_ok(p)) return RANMAR_EINVAL;
  if (fmt != RANMAR_U24 && fmt != RANMAR_F32) return RANMAR_EINVAL;
  if (fmt == RANMAR_F32 && p->e > 24) return RANMAR_EINVAL;
  if (n == 0) return RANMAR_OK;
  if (!d_in || !aligned(d_in, 4) || (d_state_out && !aligned(d_state_out, 4))) return RANMAR_EINVAL;
  if (count > 0 && (!d_out || !aligned(d_out, 4) || ld < count)) return RANMAR_EINVAL;
  if (n > (UINT64_MAX / 8) / (p->r + 1) || ld > (UINT64_MAX / 8) / n) return RANMAR_EINVAL;
  const uint64_t sb = 4ull * (p->r + 1) * n;
  if (d_state_out && d_state_out != d_in && overlap(d_in, sb, d_state_out, sb)) return RANMAR_EINVAL;
  if (count > 0) {
    const uint64_t ob = 4 * (ld * (n - 1) + count);
    if (overlap(d_out, ob, d_in, sb) || (d_state_out && overlap(d_out, ob, d_state_out, sb))) return RANMAR_EINVAL;
  }
  int rc = ensure_init();
  if (rc) return rc;
  return hip_status(launch_lfg_generate(*p, d_in, d_state_out, n, count, fmt, d_out, ld, (hipStream_t)stream));
}

}  // extern "C"
