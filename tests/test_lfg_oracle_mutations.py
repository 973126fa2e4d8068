"""The general-generator oracle's pins catch plausible mistakes.

Each case builds a copy of ``oracle/lfg_oracle.c`` with one planted error (a
sign in the reduction by phi, a lag index, the shift by t, the Horner start,
the c step, the c jump, the output sign) and checks that at least one of the
independent pins fails for it: reduction to the RANMAR oracle (separate code,
pinned to the paper), the closed forms of t^J from phi alone, and the order of
t for a primitive trinomial.  The unmodified file must pass all of them.
Everything runs on the CPU; nothing here touches the GPU library."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "lfg_oracle.c")

MUTATIONS = {
    "fold_sign_s": ("prod[k - s] = (prod[k - s] - q) & mask;", "prod[k - s] = (prod[k - s] + q) & mask;"),
    "fold_sign_r": ("prod[k - r] = (prod[k - r] + q) & mask;", "prod[k - r] = (prod[k - r] - q) & mask;"),
    "lag_index": ("uint32_t nw = (u[0] - u[r - s]) & mask;", "uint32_t nw = (u[0] - u[r - s - 1]) & mask;"),
    "shift_by_t": ("for (uint32_t i = 0; i < r; ++i) prod[i + 1] = P[i];",
                   "for (uint32_t i = 1; i < r; ++i) prod[i + 1] = P[i];"),
    "horner_start": ("v[k] = (P[r - 1] * W[k]) & mask;", "v[k] = (P[r - 2] * W[k]) & mask;"),
    "c_step": ("return c >= d ? c - d : (uint32_t)((uint64_t)c + m - d);",
               "return c > d ? c - d : (uint32_t)((uint64_t)c + m - d);"),
    "c_jump": ("uint64_t sub = (jm * (uint64_t)d) % m;", "uint64_t sub = ((jm + 1) * (uint64_t)d) % m;"),
    "output_sign": ("if (out) out[q] = (u[r - 1] - c) & mask;", "if (out) out[q] = (u[r - 1] + c) & mask;"),
}


def _build(tmp_path, name, text):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(text)
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-shared", "-fPIC", str(c), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    u32p, u64p = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    L.lfg_draws_many.argtypes = [u32] * 5 + [u64, u32p, u64, u32p, u64, u32p]
    L.lfg_jump_many.argtypes = [u32] * 5 + [u64, u32p, u64p, u64p, u32p]
    L.lfg_xpow_many.argtypes = [u32] * 3 + [u64, u64p, u64p, u32p]
    return L


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _xpow(L, r, s, e, Js):
    lo = np.array([J & ((1 << 64) - 1) for J in Js], np.uint64)
    hi = np.array([J >> 64 for J in Js], np.uint64)
    P = np.zeros((len(Js), r), np.uint32)
    L.lfg_xpow_many(r, s, e, len(Js), _p(lo, ctypes.c_uint64), _p(hi, ctypes.c_uint64), _p(P, ctypes.c_uint32))
    return P


def _failures(L, orc):
    """Names of the pins the library fails."""
    fails = []
    R, S, E, M, D = orc.RANMAR_PARAMS
    # Reduction to the RANMAR oracle: draws, states after them, and jumps.
    st = np.stack([orc.state_from_seed(x) for x in (1, 12345)])
    out = np.zeros((2, 500), np.uint32)
    after = np.zeros((2, 98), np.uint32)
    L.lfg_draws_many(R, S, E, M, D, 2, _p(st, ctypes.c_uint32), 500, _p(out, ctypes.c_uint32), 500,
                     _p(after, ctypes.c_uint32))
    ref, ref_after = orc.draws_many(st, 500)
    if not (np.array_equal(out, ref) and np.array_equal(after, ref_after)):
        fails.append("ranmar_draws")
    # The same from a state whose c equals d (the step's boundary).
    st_b = st[:1].copy()
    st_b[0, 97] = D
    out_b = np.zeros((1, 3), np.uint32)
    L.lfg_draws_many(R, S, E, M, D, 1, _p(st_b, ctypes.c_uint32), 3, _p(out_b, ctypes.c_uint32), 3, None)
    if not np.array_equal(out_b, orc.draws_many(st_b, 3)[0]):
        fails.append("ranmar_draws_c_boundary")
    Js = [0, 1, 97, 130, (1 << 100) + 3]
    lo = np.array([J & ((1 << 64) - 1) for J in Js], np.uint64)
    hi = np.array([J >> 64 for J in Js], np.uint64)
    sj = np.repeat(st[1:2], len(Js), 0)
    got = np.zeros_like(sj)
    L.lfg_jump_many(R, S, E, M, D, len(Js), _p(sj, ctypes.c_uint32), _p(lo, ctypes.c_uint64),
                    _p(hi, ctypes.c_uint64), _p(got, ctypes.c_uint32))
    if not all(np.array_equal(got[q], orc.jump(st[1], J)) for q, J in enumerate(Js)):
        fails.append("ranmar_jump")
    # Closed forms of t^J from phi alone (r = 7, s = 3, e = 8).
    r, s, e = 7, 3, 8
    mask = (1 << e) - 1
    P = _xpow(L, r, s, e, [3, r, r + 1, r + s]).astype(np.int64)
    want = np.zeros((4, r), np.int64)
    want[0, 3] = 1
    want[1, 0], want[1, r - s] = 1, -1
    want[2, 1], want[2, r - s + 1] = 1, -1
    want[3, s] += 1
    want[3, 0] -= 1
    want[3, r - s] += 1
    if not np.array_equal(P, want & mask):
        fails.append("closed_forms")
    # Order of t for the primitive trinomial t^7 + t^4 + 1 over GF(2): 2^7 (2^7 - 1) over Z/2^8.
    L_ord = (2 ** 7 - 1) << (e - 1)
    one = np.zeros(r, np.uint32)
    one[0] = 1
    P = _xpow(L, r, s, e, [L_ord, L_ord // 2])
    if not (np.array_equal(P[0], one) and not np.array_equal(P[1], one)):
        fails.append("order_of_t")
    return fails


def test_unmodified_oracle_passes_every_pin(orc, tmp_path):
    L = _build(tmp_path, "orig", open(SRC).read())
    assert _failures(L, orc) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(orc, tmp_path, name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found once: {name}"
    L = _build(tmp_path, name, text.replace(old, new))
    assert _failures(L, orc), f"no pin catches the planted mistake {name}"
