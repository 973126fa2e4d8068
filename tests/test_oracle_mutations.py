"""The RANMAR oracle's pins catch plausible mistakes.

Each case builds a copy of ``oracle/ranmar_oracle.c`` with one planted error
and checks that at least one pin fails for it.  The pins are:
- Algorithm 1 == Algorithm 2 (real and integer forms, Sec. 4);
- the draws satisfy x_n = x_{n-97} - x_{n-33} once the closed form of c is
  removed (Sec. 2);
- the jump equals literal stepping (Sec. 3);
- the closed forms of t^J (Sec. 3.1) and the order of t modulo phi (the period,
  Sec. 2);
- the closed-form c jump (Sec. 3.2);
- agreement with the separate general-generator oracle at RANMAR's parameters.

The planted errors: phi's middle exponent or a coefficient sign, the lag index
and the word shift of F_1, the c step of the literal transition, the Horner
bound, the c-jump constant, and Algorithm 2's j pointer and c step.  The
unmodified file passes every pin.  CPU only."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "ranmar_oracle.c")
MASK = (1 << 24) - 1
MOD, D, C0 = 16777213, 7654321, 362436

MUTATIONS = {
    "phi_exponent": ("static const int PHI_EXP[3] = {0, 64, 97};", "static const int PHI_EXP[3] = {0, 63, 97};"),
    "phi_sign": ("static const int PHI_COEF[3] = {-1, 1, 1};", "static const int PHI_COEF[3] = {1, 1, 1};"),
    "f1_lag": ("uint32_t nw = (u[0] - u[ORC_R - ORC_S]) & ORC_MASK;",
               "uint32_t nw = (u[0] - u[ORC_R - ORC_S + 1]) & ORC_MASK;"),
    "f1_shift": ("memmove(u, u + 1, 96 * sizeof(uint32_t));", "memmove(u, u + 1, 95 * sizeof(uint32_t));"),
    "step_c": ("c = (c >= ORC_D) ? c - ORC_D : c + ORC_MOD - ORC_D;",
               "c = (c >= ORC_D) ? c - ORC_D : c + ORC_MOD - ORC_D + 1;"),
    "horner_bound": ("for (int i = 95; i >= 0; --i) {", "for (int i = 95; i >= 1; --i) {"),
    "cjump_const": ("uint64_t sub = (jm * ORC_D) % ORC_MOD;", "uint64_t sub = (jm * (ORC_D + 1)) % ORC_MOD;"),
    "alg2_j": ("    if (st->j == 0) st->j = 97;", "    if (st->j == 0) st->j = 96;"),
    "alg2_c": ("st->v = st->v + (ORC_MOD - ORC_D);", "st->v = st->v + (ORC_MOD - ORC_D + 1);"),
}


def _build(tmp_path, name, text):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(text)
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-shared", "-fPIC", str(c), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    u32p, dblp = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)
    i64, u64, u32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
    L.orc_real_draws.argtypes = [i64, u64, dblp]
    L.orc_int_draws.argtypes = [i64, u64, u32p]
    L.orc_state_from_seed.argtypes = [i64, u32p, u32p]
    L.orc_state_draws.argtypes = [u32p, u32, u64, u32p, u32p, u32p]
    L.orc_step.argtypes = [u32p, u32, u64, u32p, u32p]
    L.orc_xpow.argtypes = [u64, u64, u32p]
    L.orc_jump.argtypes = [u32p, u32, u64, u64, u32p, u32p]
    L.orc_c_jump.argtypes = [u32, u64, u64]
    L.orc_c_jump.restype = u32
    return L


def _u(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _state(L, seed):
    W = np.zeros(97, np.uint32)
    c = np.zeros(1, np.uint32)
    assert L.orc_state_from_seed(seed, _u(W), _u(c)) == 0
    return W, int(c[0])


def _xpow(L, J):
    P = np.zeros(97, np.uint32)
    L.orc_xpow(J & ((1 << 64) - 1), J >> 64, _u(P))
    return P


def _failures(L, orc):
    fails = []
    # Algorithm 1 (real) == Algorithm 2 (integer), scaled by 2^24.
    for seed in (1, 12345):
        n = 20000
        real = np.zeros(n, np.float64)
        ints = np.zeros(n, np.uint32)
        L.orc_real_draws(seed, n, real.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        L.orc_int_draws(seed, n, _u(ints))
        if not np.array_equal(real * 2.0 ** 24, ints.astype(np.float64)):
            fails.append("real_vs_int")
            break
    # The recurrence, with c removed by its closed form.
    n = 3000
    ints = np.zeros(n, np.uint32)
    L.orc_int_draws(4711, n, _u(ints))
    c = [(C0 - (q + 1) * D) % MOD for q in range(n)]
    x = [(int(ints[q]) + c[q]) & MASK for q in range(n)]
    if any(x[q] != (x[q - 97] - x[q - 33]) & MASK for q in range(97, n)):
        fails.append("recurrence")
    # Jump == stepping.
    W, c0 = _state(L, 12345)
    for J in (1, 33, 97, 98, 200, 1000):
        Wa, ca, Wb, cb = (np.zeros(97, np.uint32), np.zeros(1, np.uint32), np.zeros(97, np.uint32),
                          np.zeros(1, np.uint32))
        L.orc_jump(_u(W), c0, J, 0, _u(Wa), _u(ca))
        L.orc_step(_u(W), c0, J, _u(Wb), _u(cb))
        if not (np.array_equal(Wa, Wb) and ca[0] == cb[0]):
            fails.append("jump_vs_step")
            break
    # Closed forms: t^5, t^97 = 1 - t^64, t^98 = t - t^65.
    want = {5: {5: 1}, 97: {0: 1, 64: MASK}, 98: {1: 1, 65: MASK}}
    for J, terms in want.items():
        w = np.zeros(97, np.uint32)
        for k, v in terms.items():
            w[k] = v
        if not np.array_equal(_xpow(L, J), w):
            fails.append("closed_forms")
            break
    # Order of t: (2^97 - 1) 2^23.
    one = np.zeros(97, np.uint32)
    one[0] = 1
    Lo = ((1 << 97) - 1) << 23
    if not (np.array_equal(_xpow(L, Lo), one) and not np.array_equal(_xpow(L, Lo // 2), one)):
        fails.append("order_of_t")
    # Closed-form c jump.
    for J in (1, 12345, (1 << 100) + 7):
        if L.orc_c_jump(C0, J & ((1 << 64) - 1), J >> 64) != (C0 - J * D) % MOD:
            fails.append("c_jump")
            break
    # The separate general-generator oracle at RANMAR's parameters.
    g = orc.LFG(*orc.RANMAR_PARAMS)
    st = np.concatenate([W, [c0]]).astype(np.uint32)
    out = np.zeros(500, np.uint32)
    L.orc_state_draws(_u(W), c0, 500, _u(out), None, None)
    if not np.array_equal(out, g.draws_many(st, 500)[0][0]):
        fails.append("general_oracle_draws")
    Wj, cj = np.zeros(97, np.uint32), np.zeros(1, np.uint32)
    J = (1 << 90) + 5
    L.orc_jump(_u(W), c0, J & ((1 << 64) - 1), J >> 64, _u(Wj), _u(cj))
    if not np.array_equal(np.concatenate([Wj, cj]), g.jump_many(st, [J])[0]):
        fails.append("general_oracle_jump")
    return fails


def test_unmodified_oracle_passes_every_pin(orc, tmp_path):
    assert _failures(_build(tmp_path, "orig", open(SRC).read()), orc) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(orc, tmp_path, name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found once: {name}"
    assert _failures(_build(tmp_path, name, text.replace(old, new)), orc), f"no pin catches {name}"
