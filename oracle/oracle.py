"""RANMAR oracle, Python side -- TEST INFRASTRUCTURE ONLY.

Loads the plain C oracle in ``ranmar_oracle.c`` (building it with gcc when no
build is present) and wraps it with numpy.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this module; the GPU library
never does, and this module imports nothing from it.

Each wrapper names the passage of Haramoto & Suzuki (arXiv 2512.00093) that
the C function follows; see the header of ``ranmar_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ranmar_oracle.c")
_SRC_LFG = os.path.join(_HERE, "lfg_oracle.c")  # general (r, s, e, m, d) generator
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD_DIR, "libranmar_oracle.so")

# Parameters of Sec. 2 (lags, precision, arithmetic-sequence constants).
R, S, E = 97, 33, 24
MOD = 16777213          # m = 2^24 - 3
D = 7654321             # d' (d = d' / 2^24)
C0 = 362436             # c'_0
MASK = (1 << 24) - 1

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into oracle/_build/."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_LFG))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", _SRC, _SRC_LFG, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dblp = ctypes.POINTER(ctypes.c_double)
        i64, u64, u32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        sig = {
            "orc_seed_setup": (ctypes.c_int, [i64, i32p]),
            "orc_seed_sequences": (None, [i32p, ctypes.c_int32, i32p, i32p]),
            "orc_seed_real": (ctypes.c_int, [i64, dblp]),
            "orc_seed_int": (ctypes.c_int, [i64, u32p]),
            "orc_real_draws": (ctypes.c_int, [i64, u64, dblp]),
            "orc_int_draws": (ctypes.c_int, [i64, u64, u32p]),
            "orc_state_from_seed": (ctypes.c_int, [i64, u32p, u32p]),
            "orc_state_draws": (None, [u32p, u32, u64, u32p, u32p, u32p]),
            "orc_step": (None, [u32p, u32, u64, u32p, u32p]),
            "orc_poly_mulmod": (None, [u32p, u32p, u32p]),
            "orc_xpow": (None, [u64, u64, u32p]),
            "orc_apply": (None, [u32p, u32p, u32p]),
            "orc_c_jump": (u32, [u32, u64, u64]),
            "orc_jump": (None, [u32p, u32, u64, u64, u32p, u32p]),
            "orc_seed_jump_many": (ctypes.c_int, [u64, i64p, u64p, u64p, u32p]),
            "orc_draws_many": (None, [u64, u32p, u64, u32p, u64, u32p]),
            "orc_xpow_many": (None, [u64, u64p, u64p, u32p]),
            "lfg_check": (ctypes.c_int, [u32, u32, u32, u32, u32]),
            "lfg_step": (None, [u32, u32, u32, u32, u32, u32p, u32, u64, u32p, u32p]),
            "lfg_draws_many": (None, [u32, u32, u32, u32, u32, u64, u32p, u64, u32p, u64, u32p]),
            "lfg_jump_many": (None, [u32, u32, u32, u32, u32, u64, u32p, u64p, u64p, u32p]),
            "lfg_xpow_many": (None, [u32, u32, u32, u64, u64p, u64p, u32p]),
            "lfg_apply": (None, [u32, u32, u32, u32p, u32p, u32p]),
            "lfg_c_jump": (u32, [u32, u32, u32, u64, u64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _u32(a):
    return _p(a, ctypes.c_uint32)


def split_u128(J: int):
    if J < 0 or J >= 1 << 128:
        raise ValueError("jump length must be in [0, 2^128)")
    return J & ((1 << 64) - 1), J >> 64


# --- Appendix A / Algorithm 3 --------------------------------------------
def seed_setup(seed: int):
    """Start values (i, j, k, l) of the initialisation's two small generators."""
    out = np.zeros(4, np.int32)
    if lib().orc_seed_setup(seed, _p(out, ctypes.c_int32)):
        raise ValueError("seed out of range")
    return tuple(int(v) for v in out)


def seed_sequences(start, count: int):
    """(m_1..m_count, l_1..l_count): the lag-3 product generator mod 179 and
    the congruential generator mod 169 from start values (i, j, k, l)."""
    st = np.ascontiguousarray(np.asarray(start, np.int32))
    m = np.zeros(count, np.int32)
    l = np.zeros(count, np.int32)
    lib().orc_seed_sequences(_p(st, ctypes.c_int32), count, _p(m, ctypes.c_int32), _p(l, ctypes.c_int32))
    return m, l


def seed_real(seed: int) -> np.ndarray:
    """u_1..u_97 from the real-arithmetic initialisation (index 0 unused)."""
    u = np.zeros(98, np.float64)
    if lib().orc_seed_real(seed, _p(u, ctypes.c_double)):
        raise ValueError("seed out of range")
    return u


def seed_int(seed: int) -> np.ndarray:
    """u_1..u_97 from Algorithm 3 with w = 32 (index 0 unused)."""
    u = np.zeros(98, np.uint32)
    if lib().orc_seed_int(seed, _u32(u)):
        raise ValueError("seed out of range")
    return u


# --- Algorithms 1 and 2 ---------------------------------------------------
def real_draws(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.float64)
    if lib().orc_real_draws(seed, n, _p(out, ctypes.c_double)):
        raise ValueError("seed out of range")
    return out


def int_draws(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.uint32)
    if lib().orc_int_draws(seed, n, _u32(out)):
        raise ValueError("seed out of range")
    return out


# --- automaton state ------------------------------------------------------
def state_from_seed(seed: int) -> np.ndarray:
    """98-word record: W[0..96] = (u_1..u_97), u_1 oldest, then c'."""
    st = np.zeros(98, np.uint32)
    c = np.zeros(1, np.uint32)
    if lib().orc_state_from_seed(seed, _u32(st), _u32(c)):
        raise ValueError("seed out of range")
    st[97] = c[0]
    return st


def state_draws(state: np.ndarray, n: int):
    """(draws, state after the draws) for n steps of the generator (Sec. 2)."""
    state = np.ascontiguousarray(state, np.uint32)
    out = np.zeros(n, np.uint32)
    W = np.zeros(97, np.uint32)
    c = np.zeros(1, np.uint32)
    lib().orc_state_draws(_u32(state), int(state[97]), n, _u32(out), _u32(W), _u32(c))
    return out, np.concatenate([W, c])


def step(state: np.ndarray, J: int) -> np.ndarray:
    """f^J applied literally, one transition at a time (Sec. 2)."""
    state = np.ascontiguousarray(state, np.uint32)
    W = np.zeros(97, np.uint32)
    c = np.zeros(1, np.uint32)
    lib().orc_step(_u32(state), int(state[97]), J, _u32(W), _u32(c))
    return np.concatenate([W, c])


# --- Sec. 3.1 / 3.2 -------------------------------------------------------
def poly_mulmod(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    out = np.zeros(97, np.uint32)
    lib().orc_poly_mulmod(_u32(a), _u32(b), _u32(out))
    return out


def xpow(J: int) -> np.ndarray:
    """P_J = t^J mod phi(t) over Z/2^24, coefficients b_0..b_96."""
    lo, hi = split_u128(J)
    P = np.zeros(97, np.uint32)
    lib().orc_xpow(lo, hi, _u32(P))
    return P


def apply(state_W: np.ndarray, P: np.ndarray) -> np.ndarray:
    """u P(A) by Horner's rule (97 words in, 97 words out)."""
    W = np.ascontiguousarray(state_W[:97], np.uint32)
    P = np.ascontiguousarray(P, np.uint32)
    out = np.zeros(97, np.uint32)
    lib().orc_apply(_u32(W), _u32(P), _u32(out))
    return out


def c_jump(c: int, J: int) -> int:
    lo, hi = split_u128(J)
    return int(lib().orc_c_jump(c, lo, hi))


def jump(state: np.ndarray, J: int) -> np.ndarray:
    state = np.ascontiguousarray(state, np.uint32)
    lo, hi = split_u128(J)
    W = np.zeros(97, np.uint32)
    c = np.zeros(1, np.uint32)
    lib().orc_jump(_u32(state), int(state[97]), lo, hi, _u32(W), _u32(c))
    return np.concatenate([W, c])


# --- batch helpers ----------------------------------------------------------
def seed_jump_many(seeds, jumps) -> np.ndarray:
    """State records (n, 98) for seed[r] jumped by jumps[r]."""
    seeds = np.ascontiguousarray(np.asarray(seeds, np.int64))
    n = seeds.shape[0]
    lo = np.zeros(n, np.uint64)
    hi = np.zeros(n, np.uint64)
    for r, J in enumerate(jumps):
        lo[r], hi[r] = split_u128(int(J))
    out = np.zeros((n, 98), np.uint32)
    rc = lib().orc_seed_jump_many(n, _p(seeds, ctypes.c_int64), _p(lo, ctypes.c_uint64),
                                  _p(hi, ctypes.c_uint64), _u32(out))
    if rc:
        raise ValueError("seed out of range")
    return out


def draws_many(states: np.ndarray, count: int, want_states: bool = True):
    """(out[n, count], states after) for n independent streams."""
    states = np.ascontiguousarray(states, np.uint32).reshape(-1, 98)
    n = states.shape[0]
    out = np.zeros((n, count), np.uint32)
    st = np.zeros((n, 98), np.uint32) if want_states else None
    lib().orc_draws_many(n, _u32(states), count, _u32(out), count, _u32(st))
    return out, st


def xpow_many(jumps) -> np.ndarray:
    n = len(jumps)
    lo = np.zeros(n, np.uint64)
    hi = np.zeros(n, np.uint64)
    for r, J in enumerate(jumps):
        lo[r], hi[r] = split_u128(int(J))
    P = np.zeros((n, 97), np.uint32)
    lib().orc_xpow_many(n, _p(lo, ctypes.c_uint64), _p(hi, ctypes.c_uint64), _u32(P))
    return P


# --- general generator of Sec. 2 (arbitrary r, s, e, m, d) ------------------
class LFG:
    """Oracle for the combined generator with lags (r, s), precision e and the
    arithmetic sequence (m, d) of Sec. 2; state records are r + 1 words
    (u_1..u_r, u_1 oldest, then c).  Wraps ``lfg_oracle.c``."""

    def __init__(self, r: int, s: int, e: int, m: int, d: int):
        if lib().lfg_check(r, s, e, m, d):
            raise ValueError("invalid generator parameters (r=%d s=%d e=%d m=%d d=%d)" % (r, s, e, m, d))
        self.r, self.s, self.e, self.m, self.d = r, s, e, m, d
        self.mask = (1 << e) - 1

    @property
    def args(self):
        return (self.r, self.s, self.e, self.m, self.d)

    def _states(self, states):
        return np.ascontiguousarray(states, np.uint32).reshape(-1, self.r + 1)

    def step(self, state, J: int) -> np.ndarray:
        """f^J applied one transition at a time (Sec. 2)."""
        state = np.ascontiguousarray(state, np.uint32)
        W = np.zeros(self.r, np.uint32)
        c = np.zeros(1, np.uint32)
        lib().lfg_step(*self.args, _u32(state), int(state[self.r]), J, _u32(W), _u32(c))
        return np.concatenate([W, c])

    def draws_many(self, states, count: int, want_states: bool = True):
        """(out[n, count], states after) for n independent streams."""
        states = self._states(states)
        n = states.shape[0]
        out = np.zeros((n, count), np.uint32)
        st = np.zeros((n, self.r + 1), np.uint32) if want_states else None
        lib().lfg_draws_many(*self.args, n, _u32(states), count, _u32(out), count, _u32(st))
        return out, st

    def xpow_many(self, jumps) -> np.ndarray:
        """P_J = t^J mod (t^r + t^(r-s) - 1) over Z/2^e, one row per J."""
        n = len(jumps)
        lo = np.zeros(n, np.uint64)
        hi = np.zeros(n, np.uint64)
        for q, J in enumerate(jumps):
            lo[q], hi[q] = split_u128(int(J))
        P = np.zeros((n, self.r), np.uint32)
        lib().lfg_xpow_many(self.r, self.s, self.e, n, _p(lo, ctypes.c_uint64), _p(hi, ctypes.c_uint64), _u32(P))
        return P

    def xpow(self, J: int) -> np.ndarray:
        return self.xpow_many([J])[0]

    def apply(self, W, P) -> np.ndarray:
        W = np.ascontiguousarray(np.asarray(W)[: self.r], np.uint32)
        P = np.ascontiguousarray(P, np.uint32)
        out = np.zeros(self.r, np.uint32)
        lib().lfg_apply(self.r, self.s, self.e, _u32(W), _u32(P), _u32(out))
        return out

    def c_jump(self, c: int, J: int) -> int:
        lo, hi = split_u128(J)
        return int(lib().lfg_c_jump(self.m, self.d, c, lo, hi))

    def jump_many(self, states, jumps) -> np.ndarray:
        """f^J by the polynomial route (Sec. 3.1 and 3.2), one J per state."""
        states = self._states(states)
        n = states.shape[0]
        lo = np.zeros(n, np.uint64)
        hi = np.zeros(n, np.uint64)
        for q, J in enumerate(jumps):
            lo[q], hi[q] = split_u128(int(J))
        out = np.zeros_like(states)
        lib().lfg_jump_many(*self.args, n, _u32(states), _p(lo, ctypes.c_uint64), _p(hi, ctypes.c_uint64),
                            _u32(out))
        return out


RANMAR_PARAMS = (R, S, E, MOD, D)
