"""Seeded synthetic inputs for the RANMAR workloads.

This module holds the input recipes only (seeds, jump lengths, stream offsets,
request arrivals and sizes) and none of the generator's arithmetic, so that
the GPU path and the CPU oracle can both draw their inputs from it without
sharing any of the method's code.

Every generator is a numpy PCG64 stream seeded from ``BASE_SEED`` plus a
per-workload offset, so a workload is reproducible from its name alone.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20251202
SEED_MIN, SEED_MAX = 1, 900_000_000     # seed range accepted by the initialisation

# Workload shapes (name -> parameters).  The sizes follow the paper's use of
# the generator: one stream per compute unit, each starting at a multiple of a
# fixed jump length, and jump lengths up to about 2^120.
SINGLE_STREAM = dict(seed=12345, draws=1_000_000, jump=1 << 20)
FAMILY_65K = dict(seed=4711, streams=65_536, spacing=1 << 40, draws=4_096)
BULK_1M = dict(seed=900_000, streams=1 << 20, spacing=1 << 100, draws=1_024)
BATCH_JUMPS = dict(requests=1_000_000, jump_bits=120)
# The paper's own workloads (Tables 1 and 2): one stream of 10^9 draws, and
# t^J mod phi for all-ones J of 64 and 120 bits.
PAPER_TABLE1 = dict(seed=12345, draws=1_000_000_000, segments=62_500)  # 62,500 rows of 16,000 = 10^9 (rows of 500 x 128 B)
PAPER_TABLE2 = dict(jumps=((1 << 64) - 1, (1 << 120) - 1))
SERVE = dict(requests=200_000, count_log10=(2.0, 7.0), offset_bits=120, budget_bytes=64 << 30)


def rng(offset: int) -> np.random.Generator:
    return np.random.default_rng(BASE_SEED + offset)


def seeds(n: int, offset: int = 4) -> np.ndarray:
    """n seeds uniform on [1, 9e8] (int32)."""
    return rng(offset).integers(SEED_MIN, SEED_MAX + 1, size=n, dtype=np.int64).astype(np.int32)


def u128_uniform(g: np.random.Generator, n: int, bits: int = 120):
    """n integers uniform on [0, 2^bits) as (lo, hi) uint64 limb arrays."""
    if not 0 < bits <= 128:
        raise ValueError("bits must be in (0, 128]")
    lo = g.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False) if bits >= 64 else \
        g.integers(0, 1 << bits, size=n, dtype=np.uint64)
    if bits > 64:
        hb = bits - 64
        hi = g.integers(0, 1 << hb, size=n, dtype=np.uint64) if hb < 64 else \
            g.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)
    else:
        hi = np.zeros(n, np.uint64)
    return lo, hi


def u128_to_int(lo, hi) -> list:
    return [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]


def int_to_u128(vals):
    vals = [int(v) for v in vals]
    lo = np.array([v & ((1 << 64) - 1) for v in vals], np.uint64)
    hi = np.array([v >> 64 for v in vals], np.uint64)
    return lo, hi


def batch_jumps(n: int, bits: int = 120, offset: int = 4):
    """Batched jump requests: (seeds int32[n], J lo uint64[n], J hi uint64[n])."""
    g = rng(offset)
    s = g.integers(SEED_MIN, SEED_MAX + 1, size=n, dtype=np.int64).astype(np.int32)
    lo, hi = u128_uniform(g, n, bits)
    return s, lo, hi


def family_offsets(n: int, spacing: int):
    """Stream k of a family starts at offset k * spacing: (lo, hi) limbs."""
    return int_to_u128([k * spacing for k in range(n)])


def family_sample(n_streams: int, k: int = 64, offset: int = 2) -> np.ndarray:
    """Stream 0, the last stream and k distinct streams from 1..n-2."""
    g = rng(offset)
    mid = g.choice(np.arange(1, n_streams - 1), size=min(k, max(n_streams - 2, 0)), replace=False)
    return np.unique(np.concatenate([[0, n_streams - 1], mid]).astype(np.int64))


def serve_requests(n: int, qps: float, offset: int = 5, count_log10=(2.0, 7.0), bits: int = 120):
    """Served requests: Poisson arrival times (s), seeds, offsets and counts.

    Counts are floor(10^U) with U uniform on count_log10 (log-uniform sizes)."""
    g = rng(offset)
    gaps = g.exponential(1.0 / qps, size=n)
    arrival = np.cumsum(gaps) - gaps[0]
    s = g.integers(SEED_MIN, SEED_MAX + 1, size=n, dtype=np.int64).astype(np.int32)
    lo, hi = u128_uniform(g, n, bits)
    counts = np.floor(10.0 ** g.uniform(count_log10[0], count_log10[1], size=n)).astype(np.uint64)
    return dict(arrival=arrival, seeds=s, off_lo=lo, off_hi=hi, counts=counts)


# General lagged-Fibonacci generators (Sec. 2 with other (r, s), precision e
# and arithmetic-sequence constants (m, d); Sec. 5 anticipates larger r).
# name -> (r, s, e, m, d).  (r, s) pairs whose trinomial t^r + t^(r-s) + 1 is
# primitive over GF(2) are the classic long-period choices (97/33 is RANMAR's,
# 55/24 the lags of the subtractive generator in Knuth's TAOCP, and 607/273,
# 1279/418, 4423/2098 have Mersenne-prime degree); the small ones cover the
# shapes a kernel must handle (s = 1, s = r - 1, s > r/2, e = 1, e = 32, m = 1).
LFG_CASES = {
    "ranmar": (97, 33, 24, 16777213, 7654321),
    "r2s1e3": (2, 1, 3, 7, 3),
    "r5s1e8": (5, 1, 8, 251, 100),
    "r5s4e8": (5, 4, 8, 241, 7),
    "r7s3e8": (7, 3, 8, 251, 17),
    "r7s6e1": (7, 6, 1, 1, 0),
    "r10s7e16": (10, 7, 16, 65521, 4321),
    "r17s3e32": (17, 3, 32, 4294967291, 2654435761),
    "r31s28e16": (31, 28, 16, 65521, 999),
    "r33s32e24": (33, 32, 24, 16777213, 12345),
    "r55s24e32": (55, 24, 32, 4294967291, 2654435761),
    "r97s64e24": (97, 64, 24, 16777213, 7654321),
    "r607s273e24": (607, 273, 24, 16777213, 7654321),
    "r1279s418e32": (1279, 418, 32, 4294967291, 2654435761),
    "r4423s2098e24": (4423, 2098, 24, 16777213, 7654321),
    "r1000s3e16": (1000, 3, 16, 65521, 77),  # large r, small s: many small rings per wave
    "r1279s418e24": (1279, 418, 24, 16777213, 7654321),  # RANMAR's precision and c constants
    "r200s150e20": (200, 150, 20, 1048573, 12345),  # 128 <= s < 256: two 64-word steps at once
    "r5120s2000e24": (5120, 2000, 24, 16777213, 7654321),  # the largest order the library accepts
}
# Throughput workload of the general path: 65,536 streams of the r = 1279
# generator, 4,096 draws each (the family65k shape at a 13x larger state).
LFG_GEN = dict(case="r1279s418e24", streams=65_536, draws=4_096)
LFG_JUMPS = dict(case="r1279s418e24", jumps=4_096, jump_bits=120)


def lfg_states(r: int, e: int, m: int, n: int, offset: int = 10) -> np.ndarray:
    """n state records of r + 1 uint32 words: r words uniform on [0, 2^e),
    then c uniform on [0, m)."""
    g = rng(offset)
    out = np.empty((n, r + 1), np.uint32)
    out[:, :r] = g.integers(0, 1 << e, size=(n, r), dtype=np.uint64).astype(np.uint32)
    out[:, r] = g.integers(0, m, size=n, dtype=np.uint64).astype(np.uint32)
    return out
