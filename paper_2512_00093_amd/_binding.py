"""ctypes binding of libranmar.so -- argument marshalling only.

Every function here has the name of the C entry point it calls (see
include/ranmar.h) and forwards torch tensors as raw device pointers together
with the current HIP stream.  No step of the generator runs in Python: when the
HIP library is missing the import fails loudly instead of falling back.

Tensor conventions (torch has no native uint32/uint64 arithmetic on GPU, so
raw words travel in int32/int64 tensors of the same width):
  states   int32  [n, 98]   ranmar_state records (x[0..96], c)
  jumps    int64  [n, 2]    ranmar_u128 records (lo, hi) as raw 64-bit limbs
  polys    int32  [n, 97]   coefficients b_0..b_96 of t^J mod phi
  seeds    int32  [n]
  draws    int32 (RANMAR_U24) or float32 (RANMAR_F32), [n, ld]; RANMAR_U24_F32: int32 [2, n, ld]
           (plane 1 holds float32 bit patterns: view it as float32)
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (the HIP runtime of torch must be loaded first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libranmar.so")

RANMAR_OK = 0
RANMAR_EINVAL = -1
RANMAR_ENOMEM = -2
RANMAR_EAGAIN = -3
RANMAR_EHIP = -4
RANMAR_ENOENT = -5
RANMAR_ETIMEDOUT = -6
RANMAR_ENODEV = -7
RANMAR_ENOINIT = -8
RANMAR_NOALLOC_FAMILY_MAX_N = 1 << 24
RANMAR_U24 = 0
RANMAR_F32 = 1
RANMAR_U24_F32 = 2
RANMAR_K_GENERATE = 0
RANMAR_K_JUMP = 1
RANMAR_K_FAMILY = 2
RANMAR_K_BATCH = 3
RANMAR_K_CHUNK = 4
RANMAR_K_POLY = 5
STATE_WORDS = 98


class RanmarError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {ranmar_strerror(status)} ({status})")


class ranmar_state(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint32 * 97), ("c", ctypes.c_uint32)]


class ranmar_u128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class ranmar_request(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_int32), ("fmt", ctypes.c_uint32), ("offset", ranmar_u128),
                ("count", ctypes.c_uint64), ("d_out", ctypes.c_void_p), ("d_state", ctypes.c_void_p)]


class ranmar_serve_cfg(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint64), ("chunk_draws", ctypes.c_uint64),
                ("max_tick_chunks", ctypes.c_uint64), ("lanes", ctypes.c_uint32),
                ("queue_when_full", ctypes.c_uint32), ("unbatched", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ranmar_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("released", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("ticks", ctypes.c_uint64), ("draws", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("bytes_peak", ctypes.c_uint64),
                ("p50_ns", ctypes.c_double), ("p99_ns", ctypes.c_double), ("max_ns", ctypes.c_double),
                ("busy_s", ctypes.c_double)]


class ranmar_lfg_params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_uint32), ("s", ctypes.c_uint32), ("e", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("d", ctypes.c_uint32)]


RANMAR_LFG_MAX_R = 5120

_lib = None

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_int = ctypes.c_int
_SIGS = {
    "ranmar_strerror": (ctypes.c_char_p, [_int]),
    "ranmar_version": (_int, []),
    "ranmar_init": (_int, []),
    "ranmar_seed": (_int, [ctypes.c_int64, ctypes.POINTER(ranmar_state)]),
    "ranmar_seed_batch": (_int, [_vp, _u64, _vp, _vp]),
    "ranmar_jump_poly": (_int, [_vp, _u64, _vp, _vp]),
    "ranmar_apply_poly": (_int, [_vp, _vp, _u64, _vp]),
    "ranmar_jump": (_int, [_vp, _vp, _u64, _vp]),
    "ranmar_seed_jump": (_int, [_vp, _vp, _u64, _vp, _vp]),
    "ranmar_jump_family": (_int, [_vp, ranmar_u128, _u64, _vp, _vp]),
    "ranmar_jump_family_noalloc": (_int, [_vp, ranmar_u128, _u64, _vp, _vp]),
    "ranmar_rank_streams": (_int, [_i32, ranmar_u128, _u64, _u64, _int, _vp, _vp]),
    "ranmar_generate": (_int, [_vp, _vp, _u64, _u64, _int, _vp, _u64, _vp]),
    "ranmar_batch_create": (_int, [_u64, _u64, _u64, ctypes.POINTER(_vp)]),
    "ranmar_batch_run": (_int, [_vp, ctypes.POINTER(ranmar_request), _u64, _vp]),
    "ranmar_batch_prepare": (_int, [_vp, ctypes.POINTER(ranmar_request), _u64]),
    "ranmar_batch_launch": (_int, [_vp, _vp]),
    "ranmar_run_unbatched": (_int, [ctypes.POINTER(ranmar_request), _u64, _vp]),
    "ranmar_batch_destroy": (_int, [_vp]),
    "ranmar_serve_create": (_int, [_vp, _u64, ctypes.POINTER(ranmar_serve_cfg), ctypes.POINTER(_vp)]),
    "ranmar_serve_submit": (_int, [_vp, _i32, ranmar_u128, _u64, _int, _u64, ctypes.POINTER(_u64)]),
    "ranmar_serve_poll": (_int, [_vp, _u64, ctypes.POINTER(_int)]),
    "ranmar_serve_wait": (_int, [_vp, _u64, ctypes.c_int64]),
    "ranmar_serve_result": (_int, [_vp, _u64, ctypes.POINTER(_vp), ctypes.POINTER(_u64)]),
    "ranmar_serve_release": (_int, [_vp, _u64]),
    "ranmar_serve_stats_get": (_int, [_vp, ctypes.POINTER(ranmar_serve_stats)]),
    "ranmar_serve_destroy": (_int, [_vp]),
    "ranmar_serve_replay": (_int, [_vp, _u64, _vp, _vp, _vp, _vp, _int, _vp]),
    "ranmar_lfg_check": (_int, [ctypes.POINTER(ranmar_lfg_params)]),
    "ranmar_lfg_jump_poly": (_int, [ctypes.POINTER(ranmar_lfg_params), _vp, _u64, _vp, _vp]),
    "ranmar_lfg_jump": (_int, [ctypes.POINTER(ranmar_lfg_params), _vp, _vp, _vp, _u64, _vp]),
    "ranmar_lfg_generate": (_int, [ctypes.POINTER(ranmar_lfg_params), _vp, _vp, _u64, _u64, _int, _vp, _u64, _vp]),
    "ranmar_lfg_jump_family": (_int, [ctypes.POINTER(ranmar_lfg_params), _vp, ranmar_u128, _u64, _vp, _vp]),
    "ranmar_tune_variants": (_int, [_int]),
    "ranmar_tune_variant_name": (ctypes.c_char_p, [_int, _int]),
    "ranmar_tune_set": (_int, [_int, _int]),
    "ranmar_tune_pick": (_int, [_int, _u64, _u64]),
    "ranmar_tune_run": (_int, [_int, _u64, _u64, ctypes.POINTER(ctypes.c_double), _vp]),
    "ranmar_tune_clear": (_int, [_int]),
    "ranmar_tune_save": (_int, [ctypes.c_char_p]),
    "ranmar_tune_load": (_int, [ctypes.c_char_p]),
}


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run python -m paper_2512_00093_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ranmar_strerror(status: int) -> str:
    return lib().ranmar_strerror(status).decode()


def _check(status: int, where: str) -> int:
    if status < 0:
        raise RanmarError(status, where)
    return status


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _u128(v: int) -> ranmar_u128:
    v = int(v)
    if v < 0 or v >= 1 << 128:
        raise ValueError("u128 out of range")
    return ranmar_u128(v & ((1 << 64) - 1), v >> 64)


# ---------------------------------------------------------------------------
def ranmar_version() -> int:
    return lib().ranmar_version()


def ranmar_init() -> None:
    _check(lib().ranmar_init(), "ranmar_init")


def ranmar_seed(seed: int):
    """Host seeding; returns a list of 98 ints (x[0..96], c)."""
    st = ranmar_state()
    _check(lib().ranmar_seed(int(seed), ctypes.byref(st)), "ranmar_seed")
    return list(st.x) + [st.c]


def new_states(n: int, device="cuda"):
    return torch.empty((n, STATE_WORDS), dtype=torch.int32, device=device)


def ranmar_seed_batch(seeds, out=None, stream=None):
    n = seeds.numel()
    if out is None:
        out = new_states(n, seeds.device)
    _check(lib().ranmar_seed_batch(_ptr(seeds), n, _ptr(out), _stream(stream)), "ranmar_seed_batch")
    return out


def ranmar_jump_poly(jumps, out=None, stream=None):
    n = jumps.shape[0]
    if out is None:
        out = torch.empty((n, 97), dtype=torch.int32, device=jumps.device)
    _check(lib().ranmar_jump_poly(_ptr(jumps), n, _ptr(out), _stream(stream)), "ranmar_jump_poly")
    return out


def ranmar_apply_poly(states, polys, stream=None):
    n = states.shape[0]
    _check(lib().ranmar_apply_poly(_ptr(states), _ptr(polys), n, _stream(stream)), "ranmar_apply_poly")
    return states


def ranmar_jump(states, jumps, stream=None):
    n = states.shape[0]
    _check(lib().ranmar_jump(_ptr(states), _ptr(jumps), n, _stream(stream)), "ranmar_jump")
    return states


def ranmar_seed_jump(seeds, offsets=None, out=None, stream=None):
    n = seeds.numel()
    if out is None:
        out = new_states(n, seeds.device)
    _check(lib().ranmar_seed_jump(_ptr(seeds), _ptr(offsets), n, _ptr(out), _stream(stream)), "ranmar_seed_jump")
    return out


def ranmar_jump_family(base, delta: int, n: int, out=None, stream=None):
    if out is None:
        out = new_states(n, base.device)
    _check(lib().ranmar_jump_family(_ptr(base), _u128(delta), n, _ptr(out), _stream(stream)),
           "ranmar_jump_family")
    return out


def ranmar_jump_family_noalloc(base, delta: int, n: int, out, stream=None):
    """ranmar_jump_family without any device allocation: `out` must be given
    (n records) and ranmar_init() must have run on this device."""
    _check(lib().ranmar_jump_family_noalloc(_ptr(base), _u128(delta), n, _ptr(out), _stream(stream)),
           "ranmar_jump_family_noalloc")
    return out


def ranmar_rank_streams(seed: int, J: int, first_rank: int, n_ranks: int, discard_first: bool = False, out=None,
                        device=None, stream=None):
    if out is None:
        out = new_states(n_ranks, device if device is not None else torch.device("cuda"))
    _check(lib().ranmar_rank_streams(int(seed), _u128(J), int(first_rank), int(n_ranks), int(bool(discard_first)),
                                     _ptr(out), _stream(stream)), "ranmar_rank_streams")
    return out


def ranmar_generate(states_in, count: int, fmt: int = RANMAR_U24, out=None, states_out=None, ld=None,
                    stream=None):
    n = states_in.shape[0]
    planes = 2 if fmt == RANMAR_U24_F32 else 1
    if ld is None:
        ld = count if out is None else out.shape[-1]
    if out is None:
        dt = torch.float32 if fmt == RANMAR_F32 else torch.int32
        out = torch.empty((planes, n, ld) if planes == 2 else (n, ld), dtype=dt, device=states_in.device)
    elif count and (not out.is_contiguous() or out.numel() < planes * n * ld or out.element_size() != 4):
        raise ValueError("out must be a contiguous 4-byte tensor of at least planes * n * ld elements")
    _check(lib().ranmar_generate(_ptr(states_in), _ptr(states_out), n, count, fmt, _ptr(out) if count else None,
                                 ld, _stream(stream)), "ranmar_generate")
    return out


# --- general lagged-Fibonacci generators (any r, s, e, m, d) ------------------
def lfg_params(r: int, s: int, e: int, m: int, d: int) -> ranmar_lfg_params:
    p = ranmar_lfg_params(r, s, e, m, d)
    _check(lib().ranmar_lfg_check(ctypes.byref(p)), "ranmar_lfg_check")
    return p


def ranmar_lfg_jump_poly(p: ranmar_lfg_params, jumps, out=None, stream=None):
    """jumps: (n, 2) int64 device tensor of (lo, hi); returns (n, r) int32."""
    n = jumps.shape[0]
    if out is None:
        out = torch.empty((n, p.r), dtype=torch.int32, device=jumps.device)
    _check(lib().ranmar_lfg_jump_poly(ctypes.byref(p), _ptr(jumps), n, _ptr(out), _stream(stream)),
           "ranmar_lfg_jump_poly")
    return out


def ranmar_lfg_jump(p: ranmar_lfg_params, states, jumps, out=None, stream=None):
    """states: (n, r + 1) int32 device tensor; out defaults to in place."""
    n = states.shape[0]
    if out is None:
        out = states
    _check(lib().ranmar_lfg_jump(ctypes.byref(p), _ptr(states), _ptr(out), _ptr(jumps), n, _stream(stream)),
           "ranmar_lfg_jump")
    return out


def ranmar_lfg_jump_family(p: ranmar_lfg_params, base, delta: int, n: int, out=None, stream=None):
    """out[k] = f^(k*delta)(base), k < n; base: one (r + 1)-word record (device)."""
    if out is None:
        out = torch.empty((n, p.r + 1), dtype=torch.int32, device=base.device)
    _check(lib().ranmar_lfg_jump_family(ctypes.byref(p), _ptr(base), _u128(delta), n, _ptr(out), _stream(stream)),
           "ranmar_lfg_jump_family")
    return out


def ranmar_lfg_generate(p: ranmar_lfg_params, states_in, count: int, fmt: int = RANMAR_U24, out=None,
                        states_out=None, ld=None, stream=None):
    n = states_in.shape[0]
    if ld is None:
        ld = count if out is None else out.shape[-1]
    if out is None:
        dt = torch.float32 if fmt == RANMAR_F32 else torch.int32
        out = torch.empty((n, ld), dtype=dt, device=states_in.device)
    elif count and (not out.is_contiguous() or out.numel() < n * ld or out.element_size() != 4):
        raise ValueError("out must be a contiguous 4-byte tensor of at least n * ld elements")
    _check(lib().ranmar_lfg_generate(ctypes.byref(p), _ptr(states_in), _ptr(states_out), n, count, fmt,
                                     _ptr(out) if count else None, ld, _stream(stream)), "ranmar_lfg_generate")
    return out


# --- batch (one persistent launch for uneven requests) ----------------------
def make_requests(items):
    """items: list of dict(seed, offset, count, fmt, out (tensor), state (tensor or None))."""
    arr = (ranmar_request * len(items))()
    for r, it in enumerate(items):
        arr[r].seed = int(it["seed"])
        arr[r].fmt = int(it.get("fmt", RANMAR_U24))
        arr[r].offset = _u128(it.get("offset", 0))
        arr[r].count = int(it["count"])
        arr[r].d_out = it["out"].data_ptr() if it.get("out") is not None else None
        st = it.get("state")
        arr[r].d_state = st.data_ptr() if st is not None else None
    return arr


def ranmar_batch_create(max_requests: int, max_chunks: int, chunk_draws: int = 0):
    h = ctypes.c_void_p()
    _check(lib().ranmar_batch_create(max_requests, max_chunks, chunk_draws, ctypes.byref(h)), "ranmar_batch_create")
    return h


def ranmar_batch_run(batch, reqs, stream=None):
    return _check(lib().ranmar_batch_run(batch, reqs, len(reqs), _stream(stream)), "ranmar_batch_run")


def ranmar_batch_prepare(batch, reqs):
    return _check(lib().ranmar_batch_prepare(batch, reqs, len(reqs)), "ranmar_batch_prepare")


def ranmar_batch_launch(batch, stream=None):
    return _check(lib().ranmar_batch_launch(batch, _stream(stream)), "ranmar_batch_launch")


def ranmar_run_unbatched(reqs, stream=None):
    return _check(lib().ranmar_run_unbatched(reqs, len(reqs), _stream(stream)), "ranmar_run_unbatched")


def ranmar_batch_destroy(batch):
    return _check(lib().ranmar_batch_destroy(batch), "ranmar_batch_destroy")


# --- serving ---------------------------------------------------------------
def ranmar_serve_create(arena, cfg: ranmar_serve_cfg | None = None):
    h = ctypes.c_void_p()
    nbytes = arena.numel() * arena.element_size()
    _check(lib().ranmar_serve_create(_ptr(arena), nbytes, ctypes.byref(cfg) if cfg is not None else None,
                                     ctypes.byref(h)), "ranmar_serve_create")
    return h


def ranmar_serve_submit(server, seed: int, offset: int, count: int, fmt: int = RANMAR_F32, t_arrival_ns: int = 0):
    t = ctypes.c_uint64()
    st = lib().ranmar_serve_submit(server, int(seed), _u128(offset), int(count), fmt, int(t_arrival_ns),
                                   ctypes.byref(t))
    return st, t.value


def ranmar_serve_poll(server, ticket: int) -> bool:
    d = ctypes.c_int()
    _check(lib().ranmar_serve_poll(server, ticket, ctypes.byref(d)), "ranmar_serve_poll")
    return bool(d.value)


def ranmar_serve_wait(server, ticket: int, timeout_ns: int = -1) -> int:
    return lib().ranmar_serve_wait(server, ticket, timeout_ns)


def ranmar_serve_result(server, ticket: int):
    p = ctypes.c_void_p()
    c = ctypes.c_uint64()
    _check(lib().ranmar_serve_result(server, ticket, ctypes.byref(p), ctypes.byref(c)), "ranmar_serve_result")
    return p.value, c.value


def ranmar_serve_release(server, ticket: int):
    return _check(lib().ranmar_serve_release(server, ticket), "ranmar_serve_release")


def ranmar_serve_stats_get(server) -> ranmar_serve_stats:
    s = ranmar_serve_stats()
    _check(lib().ranmar_serve_stats_get(server, ctypes.byref(s)), "ranmar_serve_stats_get")
    return s


def ranmar_serve_destroy(server):
    return _check(lib().ranmar_serve_destroy(server), "ranmar_serve_destroy")


def ranmar_serve_replay(server, t_arrival_s, seeds, off_lo, off_hi, counts, fmt: int = RANMAR_F32):
    """Open-loop replay of a request trace (numpy arrays); returns latencies in ns."""
    import numpy as np
    n = len(seeds)
    t = np.ascontiguousarray(t_arrival_s, np.float64)
    s = np.ascontiguousarray(seeds, np.int32)
    off = np.ascontiguousarray(np.stack([np.asarray(off_lo, np.uint64), np.asarray(off_hi, np.uint64)], 1))
    c = np.ascontiguousarray(counts, np.uint64)
    lat = np.zeros(n, np.float64)
    _check(lib().ranmar_serve_replay(server, n, t.ctypes.data, s.ctypes.data, off.ctypes.data, c.ctypes.data, fmt,
                                     lat.ctypes.data), "ranmar_serve_replay")
    return lat


# --- tuning ----------------------------------------------------------------
def ranmar_tune_variants(kernel: int) -> int:
    return _check(lib().ranmar_tune_variants(kernel), "ranmar_tune_variants")


def ranmar_tune_variant_name(kernel: int, variant: int) -> str:
    r = lib().ranmar_tune_variant_name(kernel, variant)
    return r.decode() if r else ""


def ranmar_tune_set(kernel: int, variant: int):
    return _check(lib().ranmar_tune_set(kernel, variant), "ranmar_tune_set")


def ranmar_tune_pick(kernel: int, n: int, count: int = 0) -> int:
    return _check(lib().ranmar_tune_pick(kernel, n, count), "ranmar_tune_pick")


def ranmar_tune_run(kernel: int, n: int, count: int, stream=None):
    nv = ranmar_tune_variants(kernel)
    ms = (ctypes.c_double * nv)()
    best = _check(lib().ranmar_tune_run(kernel, n, count, ms, _stream(stream)), "ranmar_tune_run")
    return best, list(ms)


def ranmar_tune_clear(kernel: int = -1):
    return _check(lib().ranmar_tune_clear(kernel), "ranmar_tune_clear")


def ranmar_tune_save(path: str):
    return _check(lib().ranmar_tune_save(path.encode()), "ranmar_tune_save")


def ranmar_tune_load(path: str):
    return _check(lib().ranmar_tune_load(path.encode()), "ranmar_tune_load")
