#!/usr/bin/env python3
"""Benchmark of the RANMAR hot path on one MI355X.

Workloads (all synthetic, seeded; see synth/):
  bulk1m     (default line) generation only: 2^20 streams at offsets k*2^100
             already on the device, 1,024 float32 draws each (2^30 draws,
             4 GiB per step); measured against HBM peak and against a plain
             4 GiB store launch timed in the same process.
  family65k  one step = seed 4711 on the GPU, 65,536 stream starts at offsets
             k*2^40 by exact GPU jump-ahead, then 4,096 draws per stream
             written as uint32 and as float32 (2^28 draws per step).
  jumps1m    10^6 seed+jump requests, J uniform on [0, 2^120), one launch.
  serve      200,000 served requests (Poisson arrivals, log-uniform counts),
             continuous batching against one launch per request.

Prints ONE JSON line for the chosen workload; the default run also measures
the other workloads briefly and reports them, compactly, under "also".
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import re
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 24-bit integer multiply-adds per second (lane-ops), 39.32 T

MACS_SQUARE = 97 * 98 // 2     # symmetric schoolbook squaring: 4753 multiply-adds
MACS_APPLY = 97 * 97           # one application of a polynomial to a window: 9409 multiply-adds
WIN_BITS = 20                  # bulk windowed jump: one table application per 20-bit digit of J
SERVE_TICK = (160, 870_000)    # a serving launch at capacity: requests x draws each (the mean count)


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _include_closure(src):
    """`src` (a file of the kernel sources) and every header it includes,
    directly or not, by quoted #include."""
    seen, todo = [], [os.path.normpath(os.path.join(ROOT, "paper_2512_00093_amd", "csrc", src))]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(f):
            continue
        seen.append(f)
        with open(f) as fh:
            for line in fh:
                m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
                if m:
                    todo.append(os.path.normpath(os.path.join(os.path.dirname(f), m.group(1))))
    return sorted(seen)


def source_digest(src=None):
    """Digest of the kernel sources: of `src` and the headers it includes, or
    of every source file and the public header."""
    h = hashlib.sha256()
    if src:
        files = _include_closure(src)
    else:
        files = sorted(glob.glob(os.path.join(ROOT, "paper_2512_00093_amd", "csrc", "*"))) + \
            sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, grid, src):
    """HBM bytes (fetched + written) per dispatch of `kernel` (a prefix of the
    kernel's name, e.g. without its last template argument) at `grid` threads
    from the committed rocprofv3 counter summaries, or None when no summary was
    taken from the current sources of that kernel (`src` and its includes)."""
    digest = source_digest(src)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md"))):
        with open(path) as fh:
            text = fh.read()
        m = re.search(r"Source digest: `([0-9a-f]+)`", text)
        if not m or m.group(1) != digest:
            continue
        for line in text.splitlines():
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) == 5 and kernel in cells[0] and cells[1] == str(grid):
                return (float(cells[3]) + float(cells[4])) * 2 ** 20
    return None


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bulk1m",
                    choices=["family65k", "bulk1m", "jumps1m", "serve", "lfg_gen", "lfg_jumps", "lfg_family"])
    ap.add_argument("--serve-requests", type=int, default=synth.SERVE["requests"])
    ap.add_argument("--serve-qps", type=float, default=2e4,
                    help="--workload serve: offered load (requests/s) of the light-load comparison")
    ap.add_argument("--serve-lanes", type=int, default=8, help="HIP streams of the server, both arms")
    ap.add_argument("--serve-capacity-only", action="store_true",
                    help="--workload serve: only the batched arm at capacity (for profiling)")
    ap.add_argument("--jump", default="family", choices=["family", "lanes"],
                    help="family65k: stream starts by prefix doubling or one jump per stream")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the library's autotuner (defaults instead of measured variants)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--force", default="",
                    help="kernel variants to force, e.g. jump=lanes8_window24,batch=direct_jumps (names as "
                         "ranmar_tune_variant_name gives them; for reproducible profiles without the tuner)")
    return ap.parse_args()


def force_variants(R, spec):
    """Applies --force: kernel=variant-name pairs, by ranmar_tune_set."""
    kernels = {"generate": R.RANMAR_K_GENERATE, "jump": R.RANMAR_K_JUMP, "family": R.RANMAR_K_FAMILY,
               "batch": R.RANMAR_K_BATCH, "chunk": R.RANMAR_K_CHUNK}
    out = {}
    for item in filter(None, spec.split(",")):
        k, name = item.split("=")
        kern = kernels[k]
        names = [R.ranmar_tune_variant_name(kern, v) for v in range(R.ranmar_tune_variants(kern))]
        if name not in names:
            raise SystemExit(f"--force: {k} has no variant {name!r} (variants: {', '.join(names)})")
        R.ranmar_tune_set(kern, names.index(name))
        out[k] = name
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample of the workload.
# ---------------------------------------------------------------------------
def _cpu_worker(args):
    kind, ks, budget = args
    from oracle import oracle as O
    t0 = time.perf_counter()
    done = 0
    units = 0
    for k in ks:
        if kind == "family65k":
            p = synth.FAMILY_65K
            st = O.jump(O.state_from_seed(p["seed"]), int(k) * p["spacing"])
            O.state_draws(st, p["draws"])
            units += p["draws"]
        elif kind == "bulk1m":
            p = synth.BULK_1M
            st = O.jump(O.state_from_seed(p["seed"]), int(k) * p["spacing"])
            O.state_draws(st, p["draws"])
            units += p["draws"]
        elif kind == "lfg_gen":
            g = O.LFG(*synth.LFG_CASES[synth.LFG_GEN["case"]])
            g.draws_many(k, synth.LFG_GEN["draws"], want_states=True)
            units += synth.LFG_GEN["draws"]
        elif kind in ("lfg_jumps", "lfg_family"):
            g = O.LFG(*synth.LFG_CASES[synth.LFG_JUMPS["case"]])
            st, J = k
            g.jump_many(st, [J])
            units += 1
        else:
            s, lo, hi = k
            O.seed_jump_many([s], [(int(hi) << 64) | int(lo)])
            units += 1
        done += 1
        if time.perf_counter() - t0 > budget:
            break
    return units, time.perf_counter() - t0, done


def cpu_baseline(kind: str, seconds: float):
    workers = max(1, min(16, os.cpu_count() or 1))
    if kind == "jumps1m":
        s, lo, hi = synth.batch_jumps(4000 * workers, 120, offset=4)
        items = list(zip(s.tolist(), lo.tolist(), hi.tolist()))
        unit, sample = "jumps/s", "seed + jump of 10^6-workload requests (J uniform 120-bit)"
    elif kind == "lfg_family":
        r, _, e, m, _ = synth.LFG_CASES[synth.LFG_GEN["case"]]
        base = synth.lfg_states(r, e, m, 1, offset=38)[0]
        n = synth.FAMILY_65K["streams"]
        ks = synth.rng(39).choice(n, size=64 * workers, replace=False)
        items = [(base, int(k) * synth.FAMILY_65K["spacing"]) for k in ks]
        unit, sample = "starts/s", f"starts of the r = {r} family: oracle jump of the base state to k * 2^40"
    elif kind in ("lfg_gen", "lfg_jumps"):
        r, _, e, m, _ = synth.LFG_CASES[synth.LFG_GEN["case"]]
        n_items = (4096 if kind == "lfg_gen" else 64) * workers
        st = synth.lfg_states(r, e, m, n_items, offset=30 if kind == "lfg_gen" else 31)
        if kind == "lfg_gen":
            items = [st[i] for i in range(n_items)]
            unit, sample = "draws/s", f"streams of the r = {r} generator: oracle draws of {synth.LFG_GEN['draws']} each"
        else:
            lo, hi = synth.u128_uniform(synth.rng(32), n_items, synth.LFG_JUMPS["jump_bits"])
            items = list(zip([st[i] for i in range(n_items)], synth.u128_to_int(lo, hi)))
            unit, sample = "jumps/s", f"states of the r = {r} generator: oracle jump by a uniform 120-bit J"
    else:
        n = synth.FAMILY_65K["streams"] if kind == "family65k" else synth.BULK_1M["streams"]
        g = synth.rng(77)
        items = [int(v) for v in g.choice(n, size=min(n, 4000 * workers), replace=False)]
        unit = "draws/s"
        sample = ("streams of the 65,536-stream family: oracle jump to k*2^40 + 4,096 draws"
                  if kind == "family65k" else "streams of the 2^20 family: oracle jump + 1,024 draws")
    chunks = [(kind, items[i::workers], seconds) for i in range(workers)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        res = pool.map(_cpu_worker, chunks)
    units = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    done = sum(r[2] for r in res)
    return {"value": units / wall, "unit": unit, "cores": workers, "kind": "oracle",
            "sample": f"{done} {sample}, {workers} processes, {wall:.1f} s", **host_info()}


def host_info():
    """The host's logical CPU count and model (the oracle's processes are
    capped at 16, the CPU share of one GPU on the benchmark machines)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_nproc": os.cpu_count(), "host_cpu": model}


def cpu_single_thread():
    """The oracle on one core, on the paper's own workload shapes: Table 1
    (one stream, real arithmetic as in Algorithm 1 against the integer form of
    Algorithm 2; a 10^8-draw sample of the 10^9-draw shape, as ten calls of
    10^7 from seeds 12345..12354) and Table 2 (t^J mod phi for the all-ones J
    of 64 and 120 bits, by left-to-right binary powering with schoolbook
    products; mean of 10 calls).  The paper's CPUs are quoted beside them."""
    from oracle import oracle as O
    n, calls = 10 ** 7, 10
    t = {}
    for name, fn in (("alg1_real", O.real_draws), ("alg2_integer", O.int_draws)):
        t0 = time.perf_counter()
        for k in range(calls):
            fn(12345 + k, n)
        t[name] = n * calls / (time.perf_counter() - t0)
    # The single-stream workload (seed 12345, 10^6 draws, one jump of 2^20
    # checked against as many single steps): seconds on one core.
    c1 = synth.SINGLE_STREAM
    t0 = time.perf_counter()
    st = O.state_from_seed(c1["seed"])
    O.state_draws(st, c1["draws"])
    t_draws = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.jump(st, c1["jump"])
    t_jump = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.step(st, c1["jump"])
    t_step = time.perf_counter() - t0
    jumps = {}
    for J in synth.PAPER_TABLE2["jumps"]:
        O.xpow(J)
        t0 = time.perf_counter()
        for _ in range(10):
            O.xpow(J)
        jumps[f"J=2^{J.bit_length()}-1"] = (time.perf_counter() - t0) / 10 * 1e6
    return {"threads": 1, "table1_draws_per_s": {k: v for k, v in t.items()},
            "table1_integer_over_real": t["alg2_integer"] / t["alg1_real"],
            "table1_sample": f"{n * calls:.0e} draws (ten streams of 1e7)",
            "table2_us": jumps,
            "single_stream_s": {"seed_and_1e6_draws": t_draws, "jump_2^20": t_jump, "2^20_single_steps": t_step},
            "paper_table1_s_1e9": {"real": {"apple": 3.30, "arm": 16.60, "ryzen": 8.45, "intel": 3.31},
                                   "integer": {"apple": 1.27, "arm": 6.14, "ryzen": 2.07, "intel": 1.01}},
            "paper_table2_us_ntl": {"J=2^64-1": [946, 10395], "J=2^120-1": [1946, 21411]}}


# ---------------------------------------------------------------------------
# GPU workloads
# ---------------------------------------------------------------------------
def _hip_runtime():
    """The HIP runtime this process already uses (the one torch and the
    library launch through), found among the loaded shared objects."""
    import ctypes
    path = None
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64.so" in line:
                path = line.split()[-1]
                break
    if path is None:
        raise RuntimeError("libamdhip64 is not loaded")
    hip = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(vp), ctypes.c_uint]
    hip.hipEventRecord.argtypes = [vp, vp]
    hip.hipEventSynchronize.argtypes = [vp]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), vp, vp]
    hip.hipEventDestroy.argtypes = [vp]
    return hip


class Timer:
    """HIP events on torch's current stream (the stream the library launches
    on), created with hipEventDisableSystemFence: timing-only events whose
    record skips the system-scope cache write-back and invalidation of an
    ordinary event, which would otherwise idle the stream between launches."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    class _Event:
        def __init__(self, timer):
            import ctypes
            self.timer = timer
            self.h = ctypes.c_void_p()
            rc = timer.hip.hipEventCreateWithFlags(ctypes.byref(self.h), Timer.DISABLE_SYSTEM_FENCE)
            if rc != 0:
                raise RuntimeError(f"hipEventCreateWithFlags: {rc}")

        def record(self):
            import ctypes
            st = ctypes.c_void_p(self.timer.t.cuda.current_stream().cuda_stream)
            rc = self.timer.hip.hipEventRecord(self.h, st)
            if rc != 0:
                raise RuntimeError(f"hipEventRecord: {rc}")

    def __init__(self, torch):
        self.t = torch
        self.hip = _hip_runtime()
        self.spans = {}

    def span(self, name):
        a, b = Timer._Event(self), Timer._Event(self)
        self.spans.setdefault(name, []).append((a, b))
        return a, b

    def all_ms(self, name):
        import ctypes
        v = []
        for a, b in self.spans.get(name, []):
            ms = ctypes.c_float()
            if self.hip.hipEventSynchronize(b.h) != 0 or self.hip.hipEventElapsedTime(ctypes.byref(ms), a.h, b.h) != 0:
                raise RuntimeError("hipEventElapsedTime failed")
            v.append(ms.value)
        return v

    def mean_ms(self, name):
        v = self.all_ms(name)
        return sum(v) / len(v) if v else float("nan")

    def median_ms(self, name):
        v = sorted(self.all_ms(name))
        return v[len(v) // 2] if v else float("nan")


def run_family65k(R, torch, steps, warmup, jump_mode):
    p = synth.FAMILY_65K
    n, cnt = p["streams"], p["draws"]
    dev = torch.device("cuda:0")
    states = torch.empty((n, 98), dtype=torch.int32, device=dev)
    out_u = torch.empty((n, cnt), dtype=torch.int32, device=dev)
    out_f = torch.empty((n, cnt), dtype=torch.float32, device=dev)
    seeds_n = torch.full((n,), p["seed"], dtype=torch.int32, device=dev)
    import numpy as np
    lo, hi = synth.family_offsets(n, p["spacing"])
    offs = torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev)
    tm = Timer(torch)

    def starts(timed=False):
        a, e = tm.span("starts") if timed else (None, None)
        if a: a.record()
        if jump_mode == "family":
            R.ranmar_rank_streams(p["seed"], p["spacing"], 0, n, out=states)
        else:
            R.ranmar_seed_jump(seeds_n, offs, out=states)
        if e: e.record()

    def gen(timed=False, f32_span=None):
        # Two passes (uint32, then float32 with the state written back): on
        # this shape they write faster than the one-pass RANMAR_U24_F32 form.
        a, e = tm.span("gen_u24") if timed else (None, None)
        if a: a.record()
        R.ranmar_generate(states, cnt, R.RANMAR_U24, out=out_u)
        if e: e.record()
        a, e = tm.span(f32_span or "gen_f32") if (timed or f32_span) else (None, None)
        if a: a.record()
        R.ranmar_generate(states, cnt, R.RANMAR_F32, out=out_f, states_out=states)
        if e: e.record()

    for _ in range(warmup):
        starts()
        gen()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        starts()
        gen(f32_span="gen_f32_timed")  # the roofline's launch time, in the timed steps
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # Per-phase times from a second, instrumented pass: event records between
    # the phases add idle time on the stream, so the timed steps carry only
    # the two around the float32 launch.
    for _ in range(steps):
        starts(True)
        gen(True)
    torch.cuda.synchronize()
    draws = n * cnt
    gen_ms = tm.mean_ms("gen_f32_timed")
    gen_bytes = 4 * draws + 2 * 392 * n          # float32 output + state read + state write-back
    res = {
        "metric": "draws/s", "value": draws / dt, "unit": "draws/s", "ms_per_step": dt * 1e3,
        "dtype": "u24", "config": {"workload": "family65k: 65,536 streams from seed 4711 at offsets k*2^40 "
                                   f"({'int8 MFMA family' if jump_mode == 'family' else 'one jump per stream'}), "
                                   "4,096 draws each as uint32 and as float32",
                                   "streams": n, "draws_per_stream": cnt, "jump": jump_mode},
        "breakdown_ms": {k: tm.mean_ms(k) for k in ("starts", "gen_u24", "gen_f32")},
        "roofline": {"bound": "hbm", "kernel": "k_gen32<f32>", "achieved": gen_bytes / (gen_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gen_bytes / (gen_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": profiled_traffic("k_gen32<1, true>", n // 8 * 256, "generate.hip"),
                     "bytes_per_launch": gen_bytes, "launch_ms": gen_ms},
    }
    return res


def run_bulk1m(R, torch, steps, warmup):
    p = synth.BULK_1M
    n, cnt = p["streams"], p["draws"]
    dev = torch.device("cuda:0")
    seed1 = torch.tensor([p["seed"]], dtype=torch.int32, device=dev)
    base = R.ranmar_seed_batch(seed1)
    states = R.ranmar_jump_family(base, p["spacing"], n)
    out = torch.empty((n, cnt), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    tm = Timer(torch)
    for _ in range(warmup):
        R.ranmar_generate(states, cnt, R.RANMAR_F32, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b = tm.span("gen")
        a.record()
        R.ranmar_generate(states, cnt, R.RANMAR_F32, out=out)
        b.record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = tm.mean_ms("gen")
    draws = n * cnt
    algo = 4 * draws + 392 * n      # output + state read (no write-back)
    return {
        "metric": "draws/s", "value": draws / dt, "unit": "draws/s", "ms_per_step": dt * 1e3, "dtype": "f32",
        "config": {"workload": "bulk1m: 2^20 streams at offsets k*2^100 from seed 900000 (states on device), "
                               "1,024 float32 draws each", "streams": n, "draws_per_stream": cnt},
        "output_write_GBps": 4 * draws / (ms * 1e-3) / 1e9,
        "output_write_frac": 4 * draws / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": "k_gen32_wide<f32>", "achieved": algo / (ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": profiled_traffic("k_gen32_wide<1, true", n // 8 * 256, "generate.hip"),
                     "bytes_per_launch": algo, "launch_ms": ms},
    }


def run_jumps1m(R, torch, steps, warmup):
    import numpy as np
    n = synth.BATCH_JUMPS["requests"]
    s, lo, hi = synth.batch_jumps(n, 120, offset=4)
    dev = torch.device("cuda:0")
    seeds = torch.from_numpy(s.copy()).to(dev)
    offs = torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev)
    out = torch.empty((n, 98), dtype=torch.int32, device=dev)
    tm = Timer(torch)
    for _ in range(warmup):
        R.ranmar_seed_jump(seeds, offs, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b = tm.span("jump")
        a.record()
        R.ranmar_seed_jump(seeds, offs, out=out)
        b.record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = tm.mean_ms("jump")
    # The same jumps on states already seeded (ranmar_jump, no seeding in the
    # launch): the difference is what seeding costs inside the launch.
    st0 = R.ranmar_seed_batch(seeds)
    R.ranmar_jump(st0, offs)
    torch.cuda.synchronize()
    for _ in range(steps):
        a, b = tm.span("jump_only")
        a.record()
        R.ranmar_jump(st0, offs)
        b.record()
    torch.cuda.synchronize()
    ms_jump_only = tm.mean_ms("jump_only")
    # Algorithmic work of the launch: one 97 x 97 application (9409
    # multiply-adds) per non-zero 20-bit digit of J (the windowed method of
    # the tables t^(d 2^(20w)) mod phi).  Seeding (Appendix A, done in the
    # same launch) is not counted; the committed instruction counters of this
    # launch give its share.
    # The window width of the variant the launch took (the tuner's pick).
    name = R.ranmar_tune_variant_name(R.RANMAR_K_JUMP, R.ranmar_tune_pick(R.RANMAR_K_JUMP, n))
    wb = int(name.split("window")[1]) if "window" in name else WIN_BITS
    Js = synth.u128_to_int(lo, hi)
    digits = sum(sum(1 for w in range(128 // wb + 1) if (J >> (wb * w)) & ((1 << wb) - 1)) for J in Js)
    macs = float(digits) * MACS_APPLY
    sqmul = sum(max(J.bit_length() - 1, 0) * MACS_SQUARE + max(bin(J).count("1") - 1, 0) * 2 for J in Js[:10000])
    ach = macs / (ms * 1e-3) / 1e12
    return {
        "metric": "jumps/s", "value": n / dt, "unit": "jumps/s", "ms_per_step": dt * 1e3, "dtype": "u24",
        "config": {"workload": "jumps1m: 10^6 seed+jump requests, seeds uniform on [1, 9e8], J uniform on "
                               "[0, 2^120), one launch", "requests": n},
        "roofline": {"bound": "alu", "kernel": "k_jump_grp<8,%d,seed>" % wb, "achieved": ach,
                     "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s", "frac": ach / VALU_PEAK_TOPS, "traffic": None,
                     "basis": "24-bit multiply-adds of the table applications, %.0f per jump (9409 per non-zero "
                              "%d-bit digit); seeding not counted; square-and-multiply would need %.3g per jump"
                              % (macs / n, wb, sqmul / min(n, 10000) + MACS_APPLY),
                     "ops_per_launch": macs, "launch_ms": ms},
        "jump_only_launch_ms": ms_jump_only,
    }


def _lfg_setup(R, torch, n, offset):
    import numpy as np
    cfg = synth.LFG_GEN
    r, s_, e, m, d = synth.LFG_CASES[cfg["case"]]
    st = synth.lfg_states(r, e, m, n, offset=offset)
    d_st = torch.from_numpy(st.view(np.int32).copy()).to(torch.device("cuda:0"))
    return R.lfg_params(r, s_, e, m, d), d_st


def run_lfg_gen(R, torch, steps, warmup):
    """General lagged-Fibonacci generation (Sec. 2 with r = 1279, s = 418,
    e = 24): 65,536 streams x 4,096 uint32 draws per step, states advanced in
    place.  HBM-bound: the draws are written once and each state (r + 1
    words) is read and written once."""
    cfg = synth.LFG_GEN
    n, count = cfg["streams"], cfg["draws"]
    p, d_st = _lfg_setup(R, torch, n, offset=30)
    out = torch.empty((n, count), dtype=torch.int32, device=torch.device("cuda:0"))
    tm = Timer(torch)
    for _ in range(warmup):
        R.ranmar_lfg_generate(p, d_st, count, R.RANMAR_U24, out=out, states_out=d_st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b = tm.span("lfg_gen")
        a.record()
        R.ranmar_lfg_generate(p, d_st, count, R.RANMAR_U24, out=out, states_out=d_st)
        b.record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = tm.mean_ms("lfg_gen")
    algo = 4.0 * n * count + 2 * 4.0 * n * (p.r + 1)
    lanes = 64
    return {
        "metric": "draws/s", "value": n * count / dt, "unit": "draws/s", "ms_per_step": dt * 1e3, "dtype": "u24",
        "config": {"workload": f"lfg_gen: general lagged-Fibonacci generator (r, s, e) = ({p.r}, {p.s}, {p.e}), "
                               f"{n} streams x {count} uint32 draws, states advanced in place", "streams": n,
                   "draws": count},
        "roofline": {"bound": "hbm", "kernel": "k_lfg_gen<0, 4>", "achieved": algo / (ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": profiled_traffic("k_lfg_gen<0, 4>", n // 4 * 4 * lanes, "lfg.hip"),
                     "bytes_per_launch": algo, "launch_ms": ms},
    }


def lfg_squarings(J: int, r: int) -> int:
    """Squarings of the left-to-right powering of t after the monomial start
    (the leading bits of J that form an exponent below r)."""
    bit, v = J.bit_length() - 1, 0
    while bit >= 0:
        b = (J >> bit) & 1
        if 2 * v + b >= r:
            break
        v = 2 * v + b
        bit -= 1
    return bit + 1


def run_lfg_jumps(R, torch, steps, warmup):
    """General lagged-Fibonacci jump-ahead (Sec. 3.1 and 3.2 at r = 1279,
    Sec. 5 cost O(r^2 log J)): 4,096 states, each jumped by its own uniform
    120-bit J, one launch.  ALU-bound: r (r + 1) / 2 multiply-adds per
    symmetric squaring and r^2 for the final application."""
    import numpy as np
    jc = synth.LFG_JUMPS
    n = jc["jumps"]
    p, d_st = _lfg_setup(R, torch, n, offset=31)
    lo, hi = synth.u128_uniform(synth.rng(32), n, jc["jump_bits"])
    dev = torch.device("cuda:0")
    jt = torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev)
    out = torch.empty_like(d_st)
    tm = Timer(torch)
    for _ in range(warmup):
        R.ranmar_lfg_jump(p, d_st, jt, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b = tm.span("lfg_jump")
        a.record()
        R.ranmar_lfg_jump(p, d_st, jt, out=out)
        b.record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = tm.mean_ms("lfg_jump")
    r = p.r
    sq = sum(lfg_squarings(J, r) for J in synth.u128_to_int(lo, hi))
    macs = float(sq) * r * (r + 1) / 2 + float(n) * r * r
    ach = macs / (ms * 1e-3) / 1e12
    return {
        "metric": "jumps/s", "value": n / dt, "unit": "jumps/s", "ms_per_step": dt * 1e3, "dtype": "u24",
        "config": {"workload": f"lfg_jumps: general lagged-Fibonacci generator (r, s, e) = ({p.r}, {p.s}, {p.e}), "
                               f"{n} states each jumped by a uniform 120-bit J, one launch", "jumps": n},
        "roofline": {"bound": "alu", "kernel": "k_lfg_jump<false>", "achieved": ach, "peak": VALU_PEAK_TOPS,
                     "unit": "T lane-ops/s (24-bit multiply-adds of the squarings and the application)",
                     "frac": ach / VALU_PEAK_TOPS, "traffic": None, "ops_per_launch": macs, "launch_ms": ms},
    }


def run_lfg_family(R, torch, steps, warmup):
    """General-generator family (block splitting at r = 1279, e = 24): 65,536
    starts spaced 2^40 apart from one base state, one call.  ALU-bound: ~256
    direct jumps and ~256 shared polynomials (squarings of r (r + 1) / 2
    multiply-adds), and an r^2 application for every start."""
    import math
    n, delta = synth.FAMILY_65K["streams"], synth.FAMILY_65K["spacing"]
    p, base = _lfg_setup(R, torch, 1, offset=38)
    out = torch.empty((n, p.r + 1), dtype=torch.int32, device=torch.device("cuda:0"))
    tm = Timer(torch)
    for _ in range(warmup):
        R.ranmar_lfg_jump_family(p, base, delta, n, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b = tm.span("lfg_family")
        a.record()
        R.ranmar_lfg_jump_family(p, base, delta, n, out=out)
        b.record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms = tm.mean_ms("lfg_family")
    r = p.r
    A = max(1, min(n, math.ceil(math.sqrt(n))))
    B = (n + A - 1) // A
    sq = sum(lfg_squarings(a * delta, r) for a in range(A)) + sum(lfg_squarings(b * A * delta, r) for b in range(1, B))
    macs = float(sq) * r * (r + 1) / 2 + float(A) * r * r + float(n - A) * r * r
    ach = macs / (ms * 1e-3) / 1e12
    return {
        "metric": "starts/s", "value": n / dt, "unit": "starts/s", "ms_per_step": dt * 1e3, "dtype": "u24",
        "config": {"workload": f"lfg_family: {n} starts spaced 2^40 of the general generator (r, s, e) = "
                               f"({p.r}, {p.s}, {p.e}), one call ({A} direct jumps, {B - 1} shared polynomials, "
                               f"{n - A} applications)", "starts": n},
        "roofline": {"bound": "alu", "kernel": "k_lfg_jump + k_lfg_family (whole call)", "achieved": ach,
                     "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s (24-bit multiply-adds)",
                     "frac": ach / VALU_PEAK_TOPS, "traffic": None, "ops_per_launch": macs, "launch_ms": ms},
    }


def run_paper_table1(R, torch, steps, warmup):
    """The paper's Table 1 workload on the GPU: 10^9 draws of ONE stream (seed
    12345, uint32).  Block splitting (Sec. 1): segment k of 16,000 draws starts
    at offset k * 16,000, so the 62,500 rows of the [62500][16000] output,
    contiguous in memory, are the stream itself, bit for bit."""
    p = synth.PAPER_TABLE1
    K = p["segments"]
    L = p["draws"] // K
    dev = torch.device("cuda:0")
    states = torch.empty((K, 98), dtype=torch.int32, device=dev)
    out = torch.empty((K, L), dtype=torch.int32, device=dev)

    def step():
        R.ranmar_rank_streams(p["seed"], L, 0, K, out=states)
        R.ranmar_generate(states, L, R.RANMAR_U24, out=out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"value": p["draws"] / dt, "unit": "draws/s", "seconds_for_1e9_draws": dt,
            "paper_seconds_cpu": {"apple": 1.27, "arm": 6.14, "ryzen": 2.07, "intel": 1.01},
            "config": {"workload": "paper Table 1 shape: 10^9 uint32 draws of one stream (seed 12345) as 62,500 "
                                   "segments of 16,000 jumped to their offsets and generated at once; the output "
                                   "array is the single stream in order"}}


def run_paper_table2(R, torch, reps=20):
    """The paper's Table 2 workload: t^J mod phi for one all-ones J (64 and
    120 bits), one request per launch (latency), and the full jump of one
    state with the windowed tables."""
    import numpy as np
    dev = torch.device("cuda:0")
    tm = Timer(torch)
    res = {}
    for J in synth.PAPER_TABLE2["jumps"]:
        bits = J.bit_length()
        jt = torch.from_numpy(np.array([[J & ((1 << 64) - 1), J >> 64]], dtype=np.uint64).view(np.int64)).to(dev)
        st = R.ranmar_seed_batch(torch.tensor([12345], dtype=torch.int32, device=dev))
        for name, poly, fn in (("jump_poly_us", -1, lambda: R.ranmar_jump_poly(jt)),
                               ("jump_poly_square_multiply_us", 0, lambda: R.ranmar_jump_poly(jt)),
                               ("windowed_jump_us", -1, lambda: R.ranmar_jump(st, jt))):
            R.ranmar_tune_set(R.RANMAR_K_POLY, poly)
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            for _ in range(reps):
                a, e = tm.span(f"{name}{bits}")
                a.record()
                fn()
                e.record()
            torch.cuda.synchronize()
            R.ranmar_tune_set(R.RANMAR_K_POLY, -1)
            res.setdefault(f"J=2^{bits}-1", {})[name] = tm.median_ms(f"{name}{bits}") * 1e3
    res["paper_us_cpu_ntl"] = {"J=2^64-1": {"apple": 1347, "arm": 10395, "ryzen": 946, "intel": 2702},
                               "J=2^120-1": {"apple": 2556, "arm": 21411, "ryzen": 1946, "intel": 4697}}
    res["config"] = {"workload": "paper Table 2 shape: one all-ones J per launch, median of 20 launches; "
                                 "jump_poly = t^J mod phi alone "
                                 "(window-table products, one wave; _square_multiply: the paper's method, one "
                                 "lane), windowed_jump = the whole jump of one state (table factors, 32 lanes)"}
    return res


def run_jumps1m_batched(R, torch, steps, warmup):
    """The 10^6 seed+jump requests through the batch executor: one persistent,
    graph-launched kernel (count 0, state out)."""
    import numpy as np
    n = synth.BATCH_JUMPS["requests"]
    s, lo, hi = synth.batch_jumps(n, 120, offset=4)
    dev = torch.device("cuda:0")
    out = torch.empty((n, 98), dtype=torch.int32, device=dev)
    reqs = (R.ranmar_request * n)()
    base = out.data_ptr()
    for i in range(n):
        reqs[i].seed = int(s[i])
        reqs[i].fmt = 0
        reqs[i].offset.lo = int(lo[i])
        reqs[i].offset.hi = int(hi[i])
        reqs[i].count = 0
        reqs[i].d_out = None
        reqs[i].d_state = base + 392 * i
    b = R.ranmar_batch_create(n, 1)
    tm = Timer(torch)
    try:
        for _ in range(warmup):
            R.ranmar_batch_run(b, reqs)
        torch.cuda.synchronize()
        prep = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            tp = time.perf_counter()
            R.ranmar_batch_prepare(b, reqs)      # host: validate + stage descriptors
            prep += time.perf_counter() - tp
            a, e = tm.span("run")
            a.record()
            R.ranmar_batch_launch(b)             # device: one graph launch
            e.record()
            torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        b2 = R.ranmar_batch_create(n, 1)
        try:
            pair = (b, b2)
            R.ranmar_batch_run(b2, reqs)
            # The same requests by ranmar_seed_jump, in alternation with the
            # batch launches, so that both see the same clock (it drifts over
            # a run): the batch executor's device time against the plain
            # launch.  The host prepares the next batch (the other object)
            # while the device runs both launches, so neither follows an idle
            # device, and the order alternates between steps.
            seeds = torch.from_numpy(s.copy()).to(dev)
            offs = torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev)
            direct = torch.empty_like(out)
            R.ranmar_seed_jump(seeds, offs, out=direct)
            torch.cuda.synchronize()
            R.ranmar_batch_prepare(pair[0], reqs)
            for k in range(2 * steps):
                def batch_launch():
                    a, e = tm.span("alt_batch")
                    a.record()
                    R.ranmar_batch_launch(pair[k % 2])
                    e.record()

                def direct_launch():
                    a, e = tm.span("alt_direct")
                    a.record()
                    R.ranmar_seed_jump(seeds, offs, out=direct)
                    e.record()
                for fn in ((batch_launch, direct_launch) if k % 2 == 0 else (direct_launch, batch_launch)):
                    fn()
                R.ranmar_batch_prepare(pair[(k + 1) % 2], reqs)
            torch.cuda.synchronize()
            same = bool(torch.equal(out, direct))
            # Two batch objects in turn: the host prepares one batch while the
            # device runs the other (prepare waits only for its own object's
            # previous launch), as a serving loop would.
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                R.ranmar_batch_prepare(pair[k % 2], reqs)
                R.ranmar_batch_launch(pair[k % 2])
            torch.cuda.synchronize()
            dt_pipe = (time.perf_counter() - t0) / steps
        finally:
            R.ranmar_batch_destroy(b2)
    finally:
        R.ranmar_batch_destroy(b)
    # Device time of a graph launch: from the alternating loop, where the
    # device stays busy between launches.  The first loop leaves it idle
    # while the host prepares each batch (2+ ms), and a launch that starts on
    # an idle device measured about a tenth slower (reported as well).
    dev_ms = tm.mean_ms("alt_batch")
    return {"value": n / (dev_ms * 1e-3), "unit": "jumps/s", "ms_per_step": dev_ms,
            "launch_ms": dev_ms, "launch_ms_after_idle": tm.mean_ms("run"),
            "host_prepare_ms": prep / steps * 1e3, "end_to_end_jumps_per_s": n / dt,
            "end_to_end_two_batches_in_turn_jumps_per_s": n / dt_pipe,
            "alternating_ms": {"batch_launch": tm.mean_ms("alt_batch"), "seed_jump": tm.mean_ms("alt_direct"),
                               "same_states": same},
            "config": {"workload": "jumps1m through the batch executor: one graph launch of 10^6 seed+jump "
                                   "requests; value = device time of the graph launch (alternating with "
                                   "ranmar_seed_jump launches on the same requests), host descriptor preparation "
                                   "reported separately"}}


def serve_arm(R, torch, tr, n, qps, lanes, unbatched, arena):
    """One open-loop serving run: the first n requests of the trace `tr`
    (arrival times rescaled to the offered rate `qps`), float32 output, every
    request released as soon as it completes.  Returns a compact summary."""
    import numpy as np
    cfg = R.ranmar_serve_cfg()
    cfg.queue_when_full = 1
    cfg.lanes = lanes
    cfg.unbatched = 1 if unbatched else 0
    arrival = tr["unit_arrival"][:n] / qps
    srv = R.ranmar_serve_create(arena, cfg)
    try:
        t0 = time.perf_counter()
        lat = R.ranmar_serve_replay(srv, arrival, tr["seeds"][:n], tr["off_lo"][:n], tr["off_hi"][:n],
                                    tr["counts"][:n], R.RANMAR_F32)
        wall = time.perf_counter() - t0
        st = R.ranmar_serve_stats_get(srv)
    finally:
        R.ranmar_serve_destroy(srv)
    draws = float(tr["counts"][:n].sum())
    return {"req": n, "qps_offered": qps, "req_per_s": n / wall, "draws_per_s": draws / wall,
            "p50_ms": float(np.percentile(lat, 50)) / 1e6, "p99_ms": float(np.percentile(lat, 99)) / 1e6,
            "max_ms": float(lat.max()) / 1e6, "ticks": int(st.ticks), "wall_s": wall,
            "arena_peak_GiB": st.bytes_peak / 2 ** 30}


def run_serve(R, torch, n_req, light_qps, lanes, capacity_only=False):
    """Serving (200,000 requests: Poisson arrivals, seed uniform on [1, 9e8],
    offset uniform on [0, 2^120), count log-uniform on [1e2, 1e7], float32
    output, 64 GiB budget), continuous batching against one launch per
    request, both arms on the same requests with the same number of streams:
      capacity   every request offered at once: the sustained rate (batched:
                 the median of three runs);
      light      both arms at the same stated rate (below either capacity);
      NNpct      each arm at 50% and 80% of its own capacity (the one launch
                 per request arm: 80% only, its 50% is about the light rate)."""
    tr = synth.serve_requests(n_req, qps=1.0, offset=5)
    tr["unit_arrival"] = tr["arrival"]          # arrival times at 1 request/s, rescaled per run
    arena = torch.empty(synth.SERVE["budget_bytes"] // 4, dtype=torch.int32, device=torch.device("cuda:0"))
    out = {"config": {"workload": f"serve: {n_req} requests, seed U[1,9e8], offset U[0,2^120), count "
                                  "log-uniform [1e2,1e7] (total %.3g draws), float32, 64 GiB budget, %d streams; "
                                  "arms on the same requests" % (float(tr["counts"].sum()), lanes)}}
    for arm, ub in (("batched", False), ("one_launch_per_request", True)):
        res = {}
        # The batched arm's capacity run takes about 0.15 s and varies by a few
        # percent: the median of three sets the loaded rates below (one run
        # when only the capacity is asked for, as under a profiler).
        reps = 1 if ub or capacity_only else 3
        caps = sorted((serve_arm(R, torch, tr, n_req, 1e12, lanes, ub, arena) for _ in range(reps)),
                      key=lambda c: c["req_per_s"])
        cap = caps[len(caps) // 2]
        if len(caps) > 1:
            cap["req_per_s_runs"] = [c["req_per_s"] for c in caps]
        res["capacity"] = cap
        _progress(f"serve {arm} capacity: {cap['req_per_s']:.4g} req/s")
        if capacity_only:
            out[arm] = res
            break
        res[f"light_{light_qps:g}qps"] = serve_arm(R, torch, tr, n_req, light_qps, lanes, ub, arena)
        for frac in ((0.5, 0.8) if not ub else (0.8,)):
            res[f"{int(frac * 100)}pct"] = serve_arm(R, torch, tr, n_req, frac * cap["req_per_s"], lanes, ub, arena)
        out[arm] = res
        _progress(f"serve {arm} done")
    del arena
    torch.cuda.synchronize()
    return out


def run_store_ceiling(torch, steps, warmup):
    """A plain 4 GiB store (torch's fill of a float32 tensor, 16-byte stores
    in address order), timed with HIP events like the generation launch: the
    write rate this device reaches with no arithmetic and no reads."""
    buf = torch.empty(1 << 30, dtype=torch.float32, device=torch.device("cuda:0"))
    tm = Timer(torch)
    for _ in range(warmup):
        buf.fill_(0.5)
    torch.cuda.synchronize()
    for _ in range(steps):
        a, b = tm.span("fill")
        a.record()
        buf.fill_(0.5)
        b.record()
    torch.cuda.synchronize()
    ms = tm.mean_ms("fill")
    del buf
    gbs = 4.0 * (1 << 30) / (ms * 1e-3) / 1e9
    return {"kernel": "torch fill, 4 GiB float32", "launch_ms": ms, "GBps": gbs, "frac": gbs / HBM_PEAK_GBS}


def autotune(R, workload, extras):
    """Runs the library's autotuner on this device for the shapes the timed
    workloads use; later calls with those shapes take the fastest variant.
    Returns {shape: variant name}."""
    shapes = []
    if workload == "family65k" or extras:
        shapes += [(R.RANMAR_K_FAMILY, synth.FAMILY_65K["streams"], 40),
                   (R.RANMAR_K_GENERATE, synth.FAMILY_65K["streams"], synth.FAMILY_65K["draws"])]
    if workload == "bulk1m" or extras:
        shapes.append((R.RANMAR_K_GENERATE, synth.BULK_1M["streams"], synth.BULK_1M["draws"]))
    if workload == "jumps1m" or extras:
        shapes.append((R.RANMAR_K_JUMP, synth.BATCH_JUMPS["requests"], 120))
    if extras or workload == "serve":
        # The batch executor's mapping: for the jump-only batch of the
        # 10^6-request workload, and for a serving launch at capacity (about
        # 160 requests of the mean count, 8.7e5 draws; the server's chunks of
        # 8,192 draws).
        shapes += [(R.RANMAR_K_BATCH, synth.BATCH_JUMPS["requests"], 0),
                   (R.RANMAR_K_BATCH, SERVE_TICK[0], SERVE_TICK[1])]
    names = {R.RANMAR_K_GENERATE: "generate", R.RANMAR_K_JUMP: "jump", R.RANMAR_K_FAMILY: "family",
             R.RANMAR_K_BATCH: "batch", R.RANMAR_K_CHUNK: "chunk"}
    out = {}
    for k, n, c in shapes:
        best, _ = R.ranmar_tune_run(k, n, c)
        out[f"{names[k]} {n}x{c}"] = R.ranmar_tune_variant_name(k, best)
    return out


def _c(x):
    """Rounds floats to 4 significant digits, recursively (keeps the one
    JSON line short enough to be read whole)."""
    if isinstance(x, float):
        return float(f"{x:.4g}")
    if isinstance(x, dict):
        return {k: _c(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_c(v) for v in x]
    return x


def _brief(res, keys=("value", "unit", "ms_per_step")):
    out = {k: res[k] for k in keys if k in res}
    rf = res.get("roofline")
    if rf:
        out["roofline"] = {k: rf[k] for k in ("bound", "kernel", "achieved", "peak", "unit", "frac", "traffic",
                                               "launch_ms", "basis") if k in rf}
    return out


def main():
    a = _parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is by disjoint "
                                   "stream ranges and needs no collective (see the design notes)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import paper_2512_00093_amd as R
    torch.cuda.set_device(0)
    R.ranmar_init()
    if a.profile_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    extras = not a.no_extras and a.workload == "bulk1m"
    forced = force_variants(R, a.force)
    tuned = {} if a.no_tune else autotune(R, a.workload, extras)
    if tuned:
        _progress("autotuned: " + json.dumps(tuned))
    if a.workload == "serve":
        r = run_serve(R, torch, a.serve_requests, a.serve_qps, a.serve_lanes, a.serve_capacity_only)
        print(json.dumps(_c({"metric": "served draws/s (p50/p99 latency)",
                             "value": r["batched"]["capacity"]["draws_per_s"], "unit": "draws/s", "n_gpus": 1,
                             "higher_is_better": True, "data": "synthetic", **r})), flush=True)
        return
    runners = {"family65k": lambda: run_family65k(R, torch, a.steps, a.warmup, a.jump),
               "bulk1m": lambda: run_bulk1m(R, torch, a.steps, a.warmup),
               "lfg_gen": lambda: run_lfg_gen(R, torch, a.steps, a.warmup),
               "lfg_jumps": lambda: run_lfg_jumps(R, torch, a.steps, a.warmup),
               "lfg_family": lambda: run_lfg_family(R, torch, a.steps, a.warmup),
               "jumps1m": lambda: run_jumps1m(R, torch, a.steps, a.warmup)}
    res = runners[a.workload]()
    _progress(f"{a.workload} done")
    line = {"metric": res["metric"], "value": res["value"], "unit": res["unit"], "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": res["dtype"], "data": "synthetic", "config": res["config"],
            "roofline": res["roofline"]}
    for k in ("breakdown_ms", "output_write_GBps", "output_write_frac", "jump_only_launch_ms"):
        if k in res:
            line[k] = res[k]
    if a.workload == "jumps1m":
        # The same requests through the batch executor (one graph launch).
        r = run_jumps1m_batched(R, torch, a.steps, a.warmup)
        line["batched"] = {k: r[k] for k in ("value", "unit", "launch_ms", "launch_ms_after_idle", "host_prepare_ms",
                                             "alternating_ms")}
        _progress("jumps1m_batched done")
    if a.workload == "bulk1m":
        ceil = run_store_ceiling(torch, a.steps, a.warmup)
        line["store_ceiling"] = ceil
        line["output_write_frac_of_store_ceiling"] = res["output_write_GBps"] / ceil["GBps"]
        _progress("store ceiling done")
    line["tuned"] = tuned
    if forced:
        line["forced"] = forced
    if extras:
        also = {}
        r = run_family65k(R, torch, 10, 2, a.jump)
        also["family65k"] = {**_brief(r), "breakdown_ms": r["breakdown_ms"]}
        _progress("family65k done")
        r = run_jumps1m(R, torch, 10, 2)
        also["jumps1m"] = {**_brief(r), "jump_only_launch_ms": r["jump_only_launch_ms"]}
        _progress("jumps1m done")
        r = run_jumps1m_batched(R, torch, 5, 1)
        also["jumps1m_batched"] = {k: r[k] for k in ("value", "unit", "launch_ms", "host_prepare_ms",
                                                      "end_to_end_jumps_per_s",
                                                      "end_to_end_two_batches_in_turn_jumps_per_s",
                                                      "launch_ms_after_idle", "alternating_ms")}
        _progress("jumps1m_batched done")
        r = run_serve(R, torch, a.serve_requests, a.serve_qps, a.serve_lanes)
        also["serve"] = r
        for name, fn, st_, wu_ in (("lfg_gen", run_lfg_gen, 20, 5), ("lfg_jumps", run_lfg_jumps, 5, 1),
                                   ("lfg_family", run_lfg_family, 5, 1)):
            r = fn(R, torch, st_, wu_)
            also[name] = _brief(r)
            _progress(f"{name} done")
        r = run_paper_table1(R, torch, 5, 1)
        also["paper_table1"] = {"value": r["value"], "unit": r["unit"], "s_for_1e9_draws": r["seconds_for_1e9_draws"]}
        r = run_paper_table2(R, torch)
        also["paper_table2_us"] = {k: v for k, v in r.items() if k.startswith("J=")}
        _progress("paper tables done")
        line["also"] = also
    # The oracle's CPU baselines run last: they fork worker processes, and the
    # GPU timings are taken before that.
    if not a.no_cpu and a.workload not in ("lfg_gen", "lfg_jumps", "lfg_family"):
        _progress("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_seconds)
        if extras:
            line["cpu_baseline"]["single_thread"] = cpu_single_thread()
    if extras and not a.no_cpu:
        for name in ("family65k", "jumps1m", "lfg_gen", "lfg_jumps", "lfg_family"):
            cb = cpu_baseline(name, min(a.cpu_seconds, 3.0))
            line["also"][name]["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "sample")}
    print(json.dumps(_c(line)), flush=True)


if __name__ == "__main__":
    main()
