/*
 * ranmar.h -- C ABI of the MI355X (gfx950) RANMAR library.
 *
 * RANMAR as restated by Haramoto & Suzuki, "Making the RANMAR pseudorandom
 * number generator in LAMMPS up to four times faster, with an implementation
 * of jump-ahead" (arXiv 2512.00093): a lagged Fibonacci sequence
 *     x_n = x_{n-97} - x_{n-33}  mod 2^24                    (Sec. 2, Sec. 3.1)
 * combined with the arithmetic sequence c_n = c_{n-1} - d' mod m, m = 2^24-3,
 * d' = 7654321 (Sec. 2, Sec. 3.2), each output being (x_n - c_n) mod 2^24
 * (Algorithm 2).  Streams are placed with the paper's exact jump-ahead:
 * t^J mod phi(t), phi = t^97 + t^64 - 1, over Z/2^24 applied to the state
 * (Sec. 3.1) and the closed form for c (Sec. 3.2).
 *
 * General conventions
 *   - Every function returns a status: RANMAR_OK (0) or a negative
 *     ranmar_status.  Argument errors are detected on the host before any
 *     work is queued and leave all buffers untouched.
 *   - "d_" pointers are device pointers (HIP device memory of the current
 *     device); other pointers are host memory.  The caller owns every buffer
 *     it passes; the library never frees caller memory and never keeps a
 *     caller pointer after the call returns (the server keeps only the arena
 *     it is given, until ranmar_serve_destroy).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is queued asynchronously on it; results are ready once the
 *     stream has been synchronised.  A failure of queued device work is
 *     reported as RANMAR_EHIP by the next call that checks the device.
 *   - Sizes are element counts unless the name says bytes.  n == 0 is valid
 *     and does nothing.
 *   - All arithmetic is integer and exact: results are bit-identical to the
 *     definitions cited, whatever the launch shape or tuning.
 */
#ifndef RANMAR_H
#define RANMAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Types                                                                     */
/* ------------------------------------------------------------------------ */

/* Generator state: the automaton state (u_1, ..., u_97, c) of Sec. 2 with
 * every word in integer form (Sec. 3.1: sigma maps the 24-bit reals to
 * Z/2^24; Sec. 3.2: c is kept as its numerator c').
 *   x[0] = u_1 is the oldest word (lag 97), x[96] = u_97 the newest; every
 *   x[k] < 2^24.  c is the numerator of the arithmetic sequence, c < m.
 * The next draw computes u_1 - u_65 (the new newest word), steps c to
 * (c - 7654321) mod m, and outputs the difference of the two mod 2^24.
 * 98 words = 392 bytes, 4-byte aligned; arrays of states are packed. */
typedef struct ranmar_state {
    uint32_t x[97];
    uint32_t c;
} ranmar_state;

/* Unsigned 128-bit jump length or offset J = hi * 2^64 + lo. */
typedef struct ranmar_u128 {
    uint64_t lo;
    uint64_t hi;
} ranmar_u128;

typedef enum ranmar_status {
    RANMAR_OK = 0,
    RANMAR_EINVAL = -1,    /* bad argument (range, NULL, misalignment) */
    RANMAR_ENOMEM = -2,    /* larger than the memory budget it was given */
    RANMAR_EAGAIN = -3,    /* budget or queue temporarily full; retry later */
    RANMAR_EHIP = -4,      /* HIP runtime error (launch or queued work) */
    RANMAR_ENOENT = -5,    /* unknown ticket / handle */
    RANMAR_ETIMEDOUT = -6, /* wait timed out */
    RANMAR_ENODEV = -7,    /* no gfx950 device current */
    RANMAR_ENOINIT = -8    /* per-device set-up (ranmar_init) not done */
} ranmar_status;

/* Output format of generated draws. */
typedef enum ranmar_fmt {
    RANMAR_U24 = 0,     /* uint32 k, 0 <= k < 2^24 (the value is k * 2^-24) */
    RANMAR_F32 = 1,     /* float k * 2^-24, exact in binary32 */
    RANMAR_U24_F32 = 2  /* both, in two planes (ranmar_generate only) */
} ranmar_fmt;

/* ------------------------------------------------------------------------ */
/* Library                                                                   */
/* ------------------------------------------------------------------------ */

/* Static text for a status code (never NULL). */
const char *ranmar_strerror(int status);

/* ABI version, major * 10000 + minor * 100 + patch. */
int ranmar_version(void);

/* Checks that the current HIP device is a gfx950 and sets up per-device
 * state: the 1.6 MB table of 8-bit jump digits and the address of the fixed
 * scratch array of ranmar_jump_family_noalloc.  The check is made implicitly
 * by every device entry point; the set-up (which allocates the table) only
 * here, once per device.  Call it with each device current before using
 * ranmar_jump_family_noalloc there. */
int ranmar_init(void);

/* ------------------------------------------------------------------------ */
/* a1: seeding (Appendix A, Algorithm 3; reading: the inner step is         */
/* Remainder(Remainder(i*j,179)*k,179))                                      */
/* ------------------------------------------------------------------------ */

/* Host: state at offset 0 for `seed`, i.e. right after Algorithm 3.
 * seed must be in [1, 900000000] (Algorithm 3 admits up to 9e8; seed 0
 * would need the quotient of -1, which the paper does not define), else
 * RANMAR_EINVAL.  out is host memory. */
int ranmar_seed(int64_t seed, ranmar_state *out);

/* Device: d_out[r] = state at offset 0 for d_seeds[r], r < n.  Seeds outside
 * [1, 9e8] produce an all-zero record with c = 0xFFFFFFFF (an invalid c
 * marks it) -- validate on the host first if needed.  d_seeds: n int32;
 * d_out: n records.  The two buffers must not overlap. */
int ranmar_seed_batch(const int32_t *d_seeds, uint64_t n, ranmar_state *d_out, void *stream);

/* ------------------------------------------------------------------------ */
/* a2-a4: jump-ahead (Sec. 3.1 and 3.2)                                      */
/* ------------------------------------------------------------------------ */

/* a3: d_P[r*97 + i] = coefficient b_i of P_J(t) = t^J mod phi(t) over
 * Z/2^24 for J = d_J[r] (Sec. 3.1; the quantity the paper times in
 * Table 2).  By default one wave per J multiplies the window table's factors
 * t^(d 2^(8w)) (2^(20w) once that table exists) over J's nonzero digits,
 * reducing each product mod phi; RANMAR_K_POLY variant 0 is left-to-right
 * square-and-multiply, one J per lane (the paper's method).  Both give the
 * same coefficients.  d_J: n values; d_P: 97*n uint32, each < 2^24. */
int ranmar_jump_poly(const ranmar_u128 *d_J, uint64_t n, uint32_t *d_P, void *stream);

/* a4: in place, x <- x P(A) for each state, with P = d_P[r*97 .. r*97+96]
 * and A the companion matrix of the lagged Fibonacci step (Horner's rule of
 * Sec. 3.1: x P(A) = sum_i b_i x A^i); c is not changed.  d_states: n
 * records; d_P: 97*n uint32 (values are taken mod 2^24). */
int ranmar_apply_poly(ranmar_state *d_states, const uint32_t *d_P, uint64_t n, void *stream);

/* a2+a3+a4: in place, d_states[r] <- f^J(d_states[r]) with J = d_J[r]:
 * x by P_J(A) (Sec. 3.1), c by (c - (J mod m) d') mod m (Sec. 3.2).
 * Equal to J single transitions.  J = 0 leaves the state unchanged.
 * Memory: P_J is formed as a product of precomputed powers of t, one per
 * nonzero digit of J.  The library keeps, per device and until the process
 * ends, a 1.6 MB table of 8-bit digits and, from the first call with at
 * least 16384 requests, a 2.4 GB table of 20-bit digits (6 factors for a
 * 120-bit J instead of 15), which later calls of any size then use; if that
 * allocation fails, the 16-bit table of 203 MB or the 8-bit one serves;
 * results are the same either way.  Where
 * the RANMAR_K_JUMP variant for the call's size is lanes8_window24 (forced,
 * or picked by the tuner), a 32.5 GB table of 24-bit digits (5 factors;
 * built in about 0.2 s on first use, kept like the others; the 20-bit table
 * serves if it cannot be allocated). */
int ranmar_jump(ranmar_state *d_states, const ranmar_u128 *d_J, uint64_t n, void *stream);

/* a1-a4 fused in one launch: d_out[r] = f^J(seed state of d_seeds[r]) with
 * J = d_offsets[r] (d_offsets may be NULL: offset 0).  This is the paper's
 * block splitting (Sec. 1): a stream is rebuilt from (seed, offset) alone.
 * Invalid seeds behave as in ranmar_seed_batch. */
int ranmar_seed_jump(const int32_t *d_seeds, const ranmar_u128 *d_offsets, uint64_t n,
                     ranmar_state *d_out, void *stream);

/* Stream family (Sec. 1, block splitting): d_out[k] = f^(k*delta)(*d_base)
 * for k < n, i.e. unit k starts at state s_{k*delta}.  Computed on the GPU
 * and bit-identical to n separate jumps: from 32,768 starts (by default) as
 * int8 matrix-core products of ~sqrt(n) direct starts with ~sqrt(n) shared
 * factor matrices (the jump is the matrix P(A_c), Sec. 3.1), otherwise in
 * radix-256 rounds of table factors.  The exponent k*delta is used exactly
 * (it may exceed 2^128, unlike the J of ranmar_jump; then by prefix doubling
 * of polynomials).  d_base: 1 record (may lie inside d_out only as d_out[0]).
 * Scratch: the product form takes (n / ~sqrt(n)) * 784 bytes of
 * stream-ordered device memory for the duration of the call. */
int ranmar_jump_family(const ranmar_state *d_base, ranmar_u128 delta, uint64_t n,
                       ranmar_state *d_out, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * ranmar_jump_family with the same result, bit for bit, that calls no
 * allocating routine.  The product form keeps its factor sequences in a
 * fixed array of RANMAR_NOALLOC_FAMILY_BYTES that each device the library
 * runs on holds until the process ends; ranmar_init() must have been called
 * with the device current (else RANMAR_ENOINIT, nothing launched).
 * Limits: n <= RANMAR_NOALLOC_FAMILY_MAX_N and (n - 1) * delta < 2^128, else
 * RANMAR_EINVAL (nothing launched).  All calls on one device share that array
 * and leave their contents in it: calls that overlap in time on one device
 * (on different streams, or from different host threads) race and must be
 * ordered by the caller. */
#define RANMAR_NOALLOC_FAMILY_MAX_N (1ull << 24)
#define RANMAR_NOALLOC_FAMILY_BYTES (4096ull * 196 * 4)
int ranmar_jump_family_noalloc(const ranmar_state *d_base, ranmar_u128 delta, uint64_t n, ranmar_state *d_out,
                               void *stream);

/* Per-rank streams of one seed (Sec. 1, block splitting, as a parallel code
 * uses it: rank p draws the block that starts at s_{p*J}): d_out[k] = state
 * of `seed` at offset (first_rank + k) * J + discard_first, for k < n_ranks.
 * discard_first = 1 drops one draw after seeding before the split, for codes
 * whose generator consumes one uniform when it is constructed; the paper
 * describes no such warm-up, and 0 is its own convention.  seed must be in
 * [1, 9e8], discard_first 0 or 1, and first_rank * J + discard_first below
 * 2^128, else RANMAR_EINVAL (nothing launched).  Seeding and every jump run on
 * the GPU: with the product-form family the seeding happens inside its first
 * launch, otherwise one seed-and-jump record is made and the family built
 * around it.  d_out: n_ranks records, 4-byte aligned. */
int ranmar_rank_streams(int32_t seed, ranmar_u128 J, uint64_t first_rank, uint64_t n_ranks, int discard_first,
                        ranmar_state *d_out, void *stream);

/* ------------------------------------------------------------------------ */
/* a5: generation (Algorithm 2)                                              */
/* ------------------------------------------------------------------------ */

/* For each stream r < n: `count` consecutive draws of Algorithm 2 starting
 * from d_in[r], written to row r of d_out (row stride `ld` elements,
 * ld >= count; element type uint32 for RANMAR_U24, float for RANMAR_F32).
 * RANMAR_U24_F32 writes every draw in both forms in one launch: uint32 k in
 * plane 0 (d_out, as for RANMAR_U24) and float k * 2^-24 in plane 1 (starting
 * n * ld elements after d_out, same row layout).
 * If d_state_out is not NULL the state after the draws is written there
 * (d_state_out may equal d_in: in-place advance; otherwise it must not
 * overlap d_in).  d_out must be 4-byte aligned and must not overlap the
 * states.  count == 0 copies the states (if d_state_out != d_in). */
int ranmar_generate(const ranmar_state *d_in, ranmar_state *d_state_out, uint64_t n,
                    uint64_t count, int fmt, void *d_out, uint64_t ld, void *stream);

/* ------------------------------------------------------------------------ */
/* a6: batched execution of uneven work in one persistent launch             */
/* ------------------------------------------------------------------------ */

/* One request of a batch: stream (seed, offset) -> `count` draws written
 * contiguously at d_out (element type per fmt).  If d_state is not NULL the
 * state after the draws is stored there.  Requests of any size share one
 * launch: each is cut into fixed-size chunks whose start states come from
 * the exact jump (offset + q*chunk), so the result equals ranmar_seed_jump
 * followed by ranmar_generate(count) for the request alone. */
typedef struct ranmar_request {
    int32_t seed;
    uint32_t fmt;       /* ranmar_fmt: RANMAR_U24 or RANMAR_F32 */
    ranmar_u128 offset; /* J of the first draw's predecessor state */
    uint64_t count;     /* draws */
    void *d_out;        /* device, count elements */
    ranmar_state *d_state; /* device, optional */
} ranmar_request;

typedef struct ranmar_batch ranmar_batch;

/* Creates a reusable batch executor able to take up to max_requests
 * requests and max_chunks chunks per run.  It owns device descriptor
 * buffers of fixed size (allocated here, once) and a captured hipGraph of
 * the persistent launch, re-played by every run.  chunk_draws = 0 takes the
 * RANMAR_K_CHUNK tuner's pick (16384 if nothing was tuned).  Each run's
 * mapping (bins, items per dequeue, jump width) comes from the
 * RANMAR_K_BATCH tuner's table for its shape.  *out receives the handle. */
int ranmar_batch_create(uint64_t max_requests, uint64_t max_chunks, uint64_t chunk_draws,
                        ranmar_batch **out);

/* Runs n requests (host array) in one graph launch on `stream`.  Returns
 * RANMAR_EINVAL for bad requests (bad seed, NULL output with count > 0,
 * bad fmt, offset + count - 1 beyond 2^128 - 1) and RANMAR_ENOMEM if n or
 * the chunk total exceed the capacity.
 * The batch may be reused once the stream has passed this run. */
int ranmar_batch_run(ranmar_batch *b, const ranmar_request *reqs, uint64_t n, void *stream);

/* ranmar_batch_run split in two: ranmar_batch_prepare validates the requests
 * and writes their descriptors into the batch's pinned staging buffer (host
 * work only, same errors as ranmar_batch_run); ranmar_batch_launch launches
 * the graph for the prepared batch on `stream` (RANMAR_EINVAL if nothing is
 * prepared).  prepare waits for the batch's previous launch to have read the
 * staging buffer; from 65,536 requests it validates and stages them on up to
 * eight host threads (it returns after all have finished). */
int ranmar_batch_prepare(ranmar_batch *b, const ranmar_request *reqs, uint64_t n);
int ranmar_batch_launch(ranmar_batch *b, void *stream);

/* Same work as ranmar_batch_run, one ordinary launch per request (the
 * baseline the batched path is measured against). */
int ranmar_run_unbatched(const ranmar_request *reqs, uint64_t n, void *stream);

int ranmar_batch_destroy(ranmar_batch *b);

/* ------------------------------------------------------------------------ */
/* a7: serving -- continuous batching of (seed, offset, count) requests      */
/* ------------------------------------------------------------------------ */

typedef struct ranmar_serve_cfg {
    uint64_t max_inflight;   /* requests admitted but not released (0 = 65536) */
    uint64_t chunk_draws;    /* draws per chunk (0 = 8192; longer chunks serve
                                more at capacity, shorter ones give large
                                requests more lanes at light load) */
    uint64_t max_tick_chunks;/* chunks per launch (0: 2^27 draws' worth, at
                                least 1024; 16384 chunks of 8192) */
    uint32_t lanes;          /* concurrent HIP streams for ticks (1..8, 0 = 2) */
    uint32_t queue_when_full;/* 1: over-budget requests wait; 0: EAGAIN */
    uint32_t unbatched;      /* 1: no batching -- each request is one launch of
                                its own (the baseline); 0: continuous batching */
    uint32_t reserved;
} ranmar_serve_cfg;

typedef struct ranmar_serve_stats {
    uint64_t submitted, completed, released, rejected;
    uint64_t ticks;            /* launches issued */
    uint64_t draws;            /* draws completed */
    uint64_t bytes_in_use;     /* arena bytes held by admitted requests */
    uint64_t bytes_peak;
    double p50_ns, p99_ns, max_ns; /* submit -> completion observed, ns */
    double busy_s;             /* wall time from first submit to last completion */
} ranmar_serve_stats;

typedef struct ranmar_server ranmar_server;

/* Starts a server thread on the current device.  d_arena/arena_bytes is the
 * HBM budget: all request outputs are sub-allocated from it (256-byte
 * aligned); the caller keeps ownership and must keep it alive until
 * ranmar_serve_destroy.  cfg may be NULL for defaults.  Besides the arena,
 * the library keeps the 2.4 GB table of 20-bit jump digits (see ranmar_jump),
 * built here if it does not exist yet, so that no request waits for it. */
int ranmar_serve_create(void *d_arena, uint64_t arena_bytes, const ranmar_serve_cfg *cfg,
                        ranmar_server **out);

/* Queues a request; *ticket identifies it.  RANMAR_ENOMEM if its output can
 * never fit the arena, RANMAR_EAGAIN if the budget or in-flight limit is
 * full and the server was configured not to queue, RANMAR_EINVAL for a bad
 * seed or format or when offset + count - 1 passes 2^128 - 1 (the server
 * cuts requests into parts that start at 128-bit offsets of their own).  t_arrival_ns (CLOCK_MONOTONIC, 0 = now) is the time from
 * which its latency is measured. */
int ranmar_serve_submit(ranmar_server *s, int32_t seed, ranmar_u128 offset, uint64_t count,
                        int fmt, uint64_t t_arrival_ns, uint64_t *ticket);

/* Non-blocking: *done = 1 once the request's output is complete on device. */
int ranmar_serve_poll(ranmar_server *s, uint64_t ticket, int *done);

/* Blocks until done or timeout_ns elapses (RANMAR_ETIMEDOUT); < 0 = forever. */
int ranmar_serve_wait(ranmar_server *s, uint64_t ticket, int64_t timeout_ns);

/* Device pointer to the request's output (server-owned until release) and
 * its element count; RANMAR_EAGAIN if not complete yet. */
int ranmar_serve_result(ranmar_server *s, uint64_t ticket, const void **d_ptr, uint64_t *count);

/* Returns the request's arena bytes to the budget; the pointer from
 * ranmar_serve_result is invalid afterwards. */
int ranmar_serve_release(ranmar_server *s, uint64_t ticket);

int ranmar_serve_stats_get(ranmar_server *s, ranmar_serve_stats *out);

/* Stops the server after draining admitted work; outstanding tickets are
 * released. */
int ranmar_serve_destroy(ranmar_server *s);

/* Open-loop load driver (benchmark support): submits request r at
 * t_arrival_s[r] seconds after the call starts (a schedule, not a wait for
 * the previous request), releases every request as soon as it completes, and
 * returns when all are released.  Latency of request r, from its scheduled
 * arrival to the server observing its completion, goes to latency_ns[r]
 * (may be NULL).  Host arrays of n entries; t_arrival_s non-decreasing.
 * Requests submitted meanwhile through ranmar_serve_submit are left to their
 * submitter.  One replay per server at a time (RANMAR_EINVAL otherwise).
 * Returns the first error of any submission (RANMAR_EINVAL, RANMAR_ENOMEM). */
int ranmar_serve_replay(ranmar_server *s, uint64_t n, const double *t_arrival_s, const int32_t *seeds,
                        const ranmar_u128 *offsets, const uint64_t *counts, int fmt, double *latency_ns);

/* ------------------------------------------------------------------------ */
/* General lagged-Fibonacci generators (Sec. 2 with other parameters; Sec. 5 */
/* anticipates a larger order r)                                             */
/* ------------------------------------------------------------------------ */

/* The combined generator of Sec. 2 with lags (r, s), precision e and the
 * arithmetic sequence (m, d), M = 2^e:
 *     x_n = x_{n-r} - x_{n-s} mod 2^e,   c_n = c_{n-1} - d mod m,
 * each draw being (x_n - c_n) mod 2^e after both have stepped.  RANMAR is
 * (97, 33, 24, 2^24 - 3, 7654321); the entry points above serve it faster.
 * Valid parameters: 2 <= r <= RANMAR_LFG_MAX_R, 1 <= s < r, 1 <= e <= 32,
 * 1 <= m < 2^e (any m >= 1 when e = 32), d < m.  m need not be prime.
 * State records are r + 1 uint32 words: x[0] = u_1 (the oldest word) ..
 * x[r-1] = u_r, then c; packed, 4-byte aligned.  Words are taken mod 2^e on
 * input; c must be < m. */
typedef struct ranmar_lfg_params {
    uint32_t r, s, e, m, d;
} ranmar_lfg_params;

/* Largest order: the jump keeps 3r words of polynomial in LDS (60 KiB). */
#define RANMAR_LFG_MAX_R 5120

/* RANMAR_OK if the parameters are valid, else RANMAR_EINVAL (host only). */
int ranmar_lfg_check(const ranmar_lfg_params *p);

/* d_P[q*r + i] = coefficient b_i of t^J mod (t^r + t^(r-s) - 1) over Z/2^e
 * for J = d_J[q], q < n (Sec. 3.1), each < 2^e.  Binary powering from the
 * leading bits of J (Sec. 5: cost O(r^2 log J)).  d_J: n values; d_P: r*n
 * uint32, not overlapping d_J. */
int ranmar_lfg_jump_poly(const ranmar_lfg_params *p, const ranmar_u128 *d_J, uint64_t n, uint32_t *d_P,
                         void *stream);

/* d_out[q] = f^J(d_in[q]) with J = d_J[q], q < n: the words by P_J(A)
 * (Sec. 3.1), c by (c - (J mod m) d) mod m (Sec. 3.2).  Equal to J single
 * transitions.  d_in, d_out: n records of r + 1 words; d_out may equal d_in
 * (in place) and must not otherwise overlap it or d_J. */
int ranmar_lfg_jump(const ranmar_lfg_params *p, const uint32_t *d_in, uint32_t *d_out, const ranmar_u128 *d_J,
                    uint64_t n, void *stream);

/* Stream family of a general generator (Sec. 1, block splitting):
 * d_out[k] = f^(k*delta)(*d_base) for k < n, bit-identical to n separate
 * jumps.  About sqrt(n) starts are direct jumps, about sqrt(n) shared
 * polynomials P_{b A delta} are formed, and every other start is one of
 * them applied to a direct start (Sec. 3.1; an r^2 application instead of a
 * whole jump).  (n - 1) * delta must be below 2^128 and n <= 2^32, else
 * RANMAR_EINVAL.  d_base: one record; it may be d_out itself (d_out[0]) and
 * must not otherwise overlap d_out.  Scratch: (about 2 sqrt(n)) * 16 + (about
 * sqrt(n)) * 4r bytes of stream-ordered device memory for the call. */
int ranmar_lfg_jump_family(const ranmar_lfg_params *p, const uint32_t *d_base, ranmar_u128 delta, uint64_t n,
                           uint32_t *d_out, void *stream);

/* For each stream q < n: `count` consecutive draws from d_in[q], written to
 * row q of d_out (row stride ld >= count elements).  fmt RANMAR_U24 writes
 * uint32 k < 2^e; RANMAR_F32 writes float k * 2^-e and needs e <= 24 (exact).
 * If d_state_out is not NULL the state after the draws is written there (it
 * may equal d_in; otherwise it must not overlap it).  d_out must not overlap
 * the states. */
int ranmar_lfg_generate(const ranmar_lfg_params *p, const uint32_t *d_in, uint32_t *d_state_out, uint64_t n,
                        uint64_t count, int fmt, void *d_out, uint64_t ld, void *stream);

/* ------------------------------------------------------------------------ */
/* Tuning                                                                     */
/* ------------------------------------------------------------------------ */

/* Kernel variant selection.  Every variant of a kernel computes the same
 * bits; the tuner only picks the fastest for a shape. */
typedef enum ranmar_kernel {
    RANMAR_K_GENERATE = 0,
    RANMAR_K_JUMP = 1,    /* ranmar_jump / ranmar_seed_jump: lanes per request
                             and window-table width (8 to 24 bits) */
    RANMAR_K_FAMILY = 2,  /* ranmar_jump_family: radix rounds on the VALU, or
                             a matrix product on the matrix cores (MFMA) */
    RANMAR_K_BATCH = 3,   /* the batch executor's tile and lane mapping, chosen
                             by ranmar_batch_prepare per shape: bins, jump
                             items per dequeue, 8- or 32-lane jumps for
                             requests without draws, or (batches of jumps
                             only) the direct mapping of one 8-request octet
                             per wave without a queue.  Its jumps take the
                             window table of RANMAR_K_JUMP's pick.  Shape: n
                             requests of `count` draws each (0: jumps only). */
    RANMAR_K_CHUNK = 4,   /* draws per chunk of the batch executor (4096 <<
                             variant), taken by ranmar_batch_create when it is
                             given 0.  Same shape as RANMAR_K_BATCH. */
    RANMAR_K_POLY = 5     /* ranmar_jump_poly: square-and-multiply per lane, or
                             window-table products per wave.  Shape: n
                             exponents of `count` bits. */
} ranmar_kernel;

/* Number of variants of a kernel, and a short name for each. */
int ranmar_tune_variants(int kernel);
const char *ranmar_tune_variant_name(int kernel, int variant);

/* Forces a variant for subsequent calls (-1 = automatic). */
int ranmar_tune_set(int kernel, int variant);

/* The variant that calls of this shape take now (forced, tuned, or the
 * built-in default), with n and count as for ranmar_tune_run (count is not
 * used for RANMAR_K_JUMP and RANMAR_K_FAMILY).  A variant whose table
 * cannot be allocated on the device falls back to the next narrower one when
 * it runs.  Returns the variant index, or RANMAR_EINVAL. */
int ranmar_tune_pick(int kernel, uint64_t n, uint64_t count);

/* Times every variant of `kernel` on synthetic data of the given shape
 * (n streams/requests; count = draws, jump bits, or for RANMAR_K_FAMILY
 * log2 of the spacing delta; for RANMAR_K_BATCH and RANMAR_K_CHUNK, draws
 * per request of a batch of n requests at uniform 120-bit offsets, each
 * launch timed alone on the device) on `stream`, stores the
 * winner for the shape bucket (log2 n, log2 count) and writes the per-variant
 * time (ms per launch, the best of several passes over all variants) to
 * ms_out[variant] (host, ranmar_tune_variants() entries, may be NULL).
 * Returns the winning variant index, or a negative status.  Allocates its
 * own synthetic inputs and outputs for the duration of the call. */
int ranmar_tune_run(int kernel, uint64_t n, uint64_t count, double *ms_out, void *stream);

/* Forgets what the tuner recorded for `kernel` (every shape; -1: every
 * kernel), so that later calls take the built-in defaults again.  Forced
 * variants (ranmar_tune_set) are not affected. */
int ranmar_tune_clear(int kernel);

/* Saves / loads the tuned table (text file, one line per bucket). */
int ranmar_tune_save(const char *path);
int ranmar_tune_load(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* RANMAR_H */
