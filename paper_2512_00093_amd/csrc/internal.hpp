// Internal host-side interface between the C ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ranmar.h"

namespace ranmar {

// seeds -> state records at offset 0
hipError_t launch_seed(const int32_t* seeds, uint64_t n, uint32_t* out, hipStream_t st);
// t^J mod phi, 97 words per request
hipError_t launch_jump_poly(const ranmar_u128* J, uint64_t n, uint32_t* P, hipStream_t st);  // lane square-and-multiply
hipError_t launch_jump_poly_tab(const ranmar_u128* J, uint64_t n, uint32_t* P, hipStream_t st);  // window-table products
enum PolyVariant : int {
  POLY_LANE_SQMUL = 0,  // one J per lane, left-to-right square-and-multiply in VGPRs
  POLY_TABLE = 1,       // one J per wave, products of window-table factors
  POLY_NUM_VARIANTS = 2
};
int poly_variant_for(uint64_t n);
// x <- x P(A)
hipError_t launch_apply_poly(uint32_t* states, const uint32_t* P, uint64_t n, hipStream_t st);
// in-place f^J, optionally seeding first (seeds != nullptr)
hipError_t launch_jump(uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n, hipStream_t st);

// Half-wave cooperative variant (windowed jump, parallel seeding).
hipError_t launch_jump_coop(uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n,
                            hipStream_t st);
const uint32_t* window_table();    // T[w][d] = t^(d 2^(8w)) mod phi, per device
const uint32_t* window16_table();  // T[w][d] = t^(d 2^(16w)) mod phi, per device (nullptr if it cannot be built)
const uint32_t* window20_table();  // T[w][d] = t^(d 2^(20w)) mod phi: 6 x 2^20 + 2^8 rows (nullptr if it cannot be built)
const uint32_t* window20_table_ready();  // the same if already built on this device, else nullptr (never builds)
const uint32_t* window24_table();  // T[w][d] = t^(d 2^(24w)) mod phi: 5 x 2^24 + 2^8 rows, 32.5 GB (nullptr if it cannot be built)
// Makes the batch's jumps use the 20-bit table (building it now if needed).
void batch_use_wide_windows(ranmar_batch* b);
hipError_t launch_seed_coop(const int32_t* seeds, uint64_t n, uint32_t* out, hipStream_t st);
// One record: the state of a (checked) seed at offset E, values by argument.
hipError_t launch_seed_jump_one(uint32_t* out, int32_t seed, ranmar_u128 E, hipStream_t st);
// Family by table factors; hipErrorInvalidValue if an exponent needs > 128 bits.
hipError_t launch_family_window(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st);
// Family as a matrix product on the matrix cores; hipErrorInvalidValue if
// the family is too small for it or an exponent needs > 128 bits.
// tile_rows: 16 (v_mfma_i32_16x16x64_i8) or 32 (v_mfma_i32_32x32x32_i8).
hipError_t launch_family_gemm(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st,
                              uint32_t tile_rows);
// The same family around the state of a (checked) seed at offset e0: the
// seeding happens inside the first launch.
hipError_t launch_family_gemm_seeded(int32_t seed, ranmar_u128 e0, ranmar_u128 delta, uint64_t n, uint32_t* out,
                                     hipStream_t st, uint32_t tile_rows);
// No-allocation family: the product form's factor sequences in a fixed
// per-device array.  noalloc_setup (from ranmar_init, device current) takes the
// array's device address and builds the 8-bit window table; noalloc_scratch
// returns that address for the current device, or nullptr before set-up.
int noalloc_setup();
uint32_t* noalloc_scratch();
hipError_t launch_family_gemm_fixed(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out,
                                    hipStream_t st, uint32_t tile_rows, uint32_t* H);
// General lagged-Fibonacci generators (any r, s, e, m, d).
int lfg_params_ok(const ranmar_lfg_params* p);
uint32_t lfg_jump_threads(uint32_t r);
void lfg_gen_shape(uint32_t r, uint32_t s, uint32_t* lw, uint32_t* G, uint32_t* Z, uint32_t* waves);
// P_out != nullptr: polynomials only; else states s_in -> s_out (may alias).
hipError_t launch_lfg_jump(const ranmar_lfg_params& p, const ranmar_u128* J, const uint32_t* s_in, uint32_t* s_out,
                           uint32_t* P_out, uint64_t n, hipStream_t st);
// out[k] = f^{k delta}(*base), k < n; hipErrorInvalidValue if (n - 1) delta
// needs more than 128 bits or n > 2^32.
hipError_t launch_lfg_family(const ranmar_lfg_params& p, const uint32_t* base, ranmar_u128 delta, uint64_t n,
                             uint32_t* out, hipStream_t st);
hipError_t launch_lfg_generate(const ranmar_lfg_params& p, const uint32_t* s_in, uint32_t* s_out, uint64_t n,
                               uint64_t count, int fmt, void* out, uint64_t ld, hipStream_t st);
enum FamilyVariant : int {
  FAMILY_RADIX = 0,  // radix-256 rounds, one table application per start (VALU)
  FAMILY_GEMM = 1,   // ~sqrt(n) direct starts and factors, the rest as int8 MFMA products (16 x 16 x 64)
  FAMILY_GEMM32 = 2, // the same with 32 x 32 x 32 MFMAs and row / column 96 on the VALU
  FAMILY_NUM_VARIANTS = 3
};
int family_variant_for(uint64_t n);
// A family with the given variant, falling back (radix rounds, then the
// polynomial path) where the variant does not apply.
hipError_t launch_family_variant(int v, const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out,
                                 hipStream_t st);

enum JumpVariant : int {
  JUMP_LANE_SQMUL = 0,      // one request per lane, square-and-multiply in VGPRs
  JUMP_HALF_WINDOW = 1,     // one request per half-wave, 8-bit windows in LDS
  JUMP_QUARTER_WINDOW = 2,  // one request per 16 lanes, 8-bit windows in LDS
  JUMP_EIGHTH_WINDOW = 3,   // one request per 8 lanes, 8-bit windows in LDS
  JUMP_EIGHTH_WINDOW16 = 4, // one request per 8 lanes, 16-bit windows (203 MB table)
  JUMP_EIGHTH_WINDOW20 = 5, // one request per 8 lanes, 20-bit windows (2.4 GB table)
  JUMP_EIGHTH_WINDOW24 = 6, // one request per 8 lanes, 24-bit windows (32.5 GB table)
  JUMP_NUM_VARIANTS = 7
};
int jump_variant_for(uint64_t n);
// Seed (seeds != nullptr) and jump with the given variant.
hipError_t launch_jump_variant(int v, uint32_t* states, const int32_t* seeds, const ranmar_u128* J, uint64_t n,
                               hipStream_t st);

// Generation variants (all bit-identical).
enum GenVariant : int {
  GEN_LANES32 = 0,     // 32 lanes per stream, cross-lane shift via ds_bpermute
  GEN_LANES32_NT = 1,  // same, non-temporal output stores
  GEN_WIDE4 = 2,       // four blocks per step, LDS transpose, 16-byte stores
  GEN_WIDE4_NT = 3,    // same, non-temporal
  GEN_PIPE_NT = 4,     // 32 lanes per stream, several streams per half-wave with the next state prefetched
  // Residency-capped forms: the launch reserves LDS (unused by the kernel) so
  // that at most R workgroups share a CU.  Fewer rows are then written at
  // once, and each is written faster, which HBM takes more efficiently.
  GEN_LANES32_NT_R2 = 5,
  GEN_LANES32_NT_R3 = 6,
  GEN_WIDE4_NT_R4 = 7,
  GEN_WIDE4_NT_R6 = 8,
  GEN_WIDE4_NT_R5 = 9,
  // The wide form with 16 half-waves per workgroup (512 threads), at most R
  // such workgroups per CU.
  GEN_WIDE16_NT_R2 = 10,
  GEN_WIDE16_NT_R3 = 11,
  GEN_NUM_VARIANTS = 12
};
const char* gen_variant_name(int v);
hipError_t launch_generate(int variant, const uint32_t* sin, uint32_t* sout, uint64_t n, uint64_t count, int fmt,
                           void* out, uint64_t ld, hipStream_t st);

// Stream family by prefix doubling: out[k] = f^(k*delta)(base), k < n.
hipError_t launch_family(const uint32_t* base, ranmar_u128 delta, uint64_t n, uint32_t* out, hipStream_t st);

// Batch executor mappings (all bit-identical): how prepare cuts the work
// into bins and items.  Picked per (requests, draws per request) bucket.
enum BatchVariant : int {
  BATCH_AUTO = 0,         // up to 64 bins; jump pairs / octets per dequeue from the bin's fill
  BATCH_FINE = 1,         // one jump pair / octet per dequeue (finest balance)
  BATCH_COARSE = 2,       // twice BATCH_AUTO's items per dequeue (fewer dequeues)
  BATCH_BINS16 = 3,       // at most 16 bins (more workgroups per bin)
  BATCH_BINS16_FINE = 4,  // both
  BATCH_PAIRS = 5,        // slices without draws by pair items (32 lanes each) instead of octets (8 lanes)
  BATCH_HALF_GRID = 6,    // BATCH_AUTO on at most half the workgroups the device holds (fewer waves per CU)
  BATCH_QUARTER_GRID = 7, // the same on at most a quarter
  BATCH_DIRECT = 8,       // batches of jumps only: one octet per worker, one bin, no queue (else BATCH_AUTO)
  BATCH_NUM_VARIANTS = 9
};
int batch_variant_for(uint64_t n, uint64_t draws_per_request);
void batch_set_variant(ranmar_batch* b, int v);  // -1: from the table
// Chunk lengths the tuner chooses among (create time): 4096 << v draws.
constexpr int kChunkVariants = 4;
inline uint32_t chunk_variant_draws(int v) { return 4096u << v; }
// Chunk length for a batch or server created with chunk_draws = 0: the
// forced or tuned pick, else `fallback`.
uint32_t chunk_draws_default(uint32_t fallback);

// Library-wide state.
int ensure_init();          // RANMAR_OK / RANMAR_ENODEV / RANMAR_EHIP
int gen_variant_for(uint64_t n, uint64_t count);   // tuned or default
void set_error_from_hip(hipError_t e);

}  // namespace ranmar
