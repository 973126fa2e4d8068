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

- the initialisation's set-up, product generator, congruential generator and
  first draws (``seed_pins``: bijection and injectivity of the index
  arithmetic, the exponent form mod 179, the closed form and full period
  mod 169, the words read top down).

The planted errors: phi's middle exponent or a coefficient sign, the lag index
and the word shift of F_1, the c step of the literal transition, the Horner
bound, the c-jump constant, the sequence form's lag, c closed form and c
index, the real route's lag and c step; and in the initialisation every
constant of the index set-up (30082, 177, 178, 169, both +2 offsets and the
+1), the product generator's modulus and shift order, the congruential
generator's multiplier, increment and modulus, the bit's threshold, modulus
and order, and the orientation of the words, in both routes.  The unmodified
file passes every pin.  CPU only."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import seed_pins

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "ranmar_oracle.c")
MASK = (1 << 24) - 1
MOD, D, C0 = 16777213, 7654321, 362436

MUTATIONS = {
    # Sec. 3.1 and the literal transition of Sec. 2.
    "phi_exponent": ("static const int PHI_EXP[3] = {0, 64, 97};", "static const int PHI_EXP[3] = {0, 63, 97};"),
    "phi_sign": ("static const int PHI_COEF[3] = {-1, 1, 1};", "static const int PHI_COEF[3] = {1, 1, 1};"),
    "f1_lag": ("uint32_t nw = (u[0] - u[ORC_R - ORC_S]) & ORC_MASK;",
               "uint32_t nw = (u[0] - u[ORC_R - ORC_S + 1]) & ORC_MASK;"),
    "f1_shift": ("memmove(u, u + 1, 96 * sizeof(uint32_t));", "memmove(u, u + 1, 95 * sizeof(uint32_t));"),
    "step_c": ("c = (c >= ORC_D) ? c - ORC_D : c + ORC_MOD - ORC_D;",
               "c = (c >= ORC_D) ? c - ORC_D : c + ORC_MOD - ORC_D + 1;"),
    "horner_bound": ("for (int i = 95; i >= 0; --i) {", "for (int i = 95; i >= 1; --i) {"),
    "cjump_const": ("uint64_t sub = (jm * ORC_D) % ORC_MOD;", "uint64_t sub = (jm * (ORC_D + 1)) % ORC_MOD;"),
    # The generator as a sequence (Sec. 2), integer and real routes.
    "seq_lag": ("uint32_t x_mid = ring[(t - 33 - 1) % 97];", "uint32_t x_mid = ring[(t - 32 - 1) % 97];"),
    "seq_c_closed_form": ("uint64_t sub = (n % ORC_MOD) * ORC_D % ORC_MOD;",
                          "uint64_t sub = (n % ORC_MOD) * (ORC_D - 1) % ORC_MOD;"),
    "seq_c_index": ("if (out) out[q - 1] = (x_new - c_after(c, q)) & ORC_MASK;",
                    "if (out) out[q - 1] = (x_new - c_after(c, q - 1)) & ORC_MASK;"),
    "real_lag": ("double nw = x[0] - x[64];", "double nw = x[0] - x[63];"),
    "real_c_step": ("if (c < 0.0) c += mreal;", "if (c <= 0.0) c += mreal;"),
    # Appendix A: the index set-up (integer route).  The outer "mod 177" of i
    # is not among them: the quotient a / 177 stays below 170 for every seed
    # up to 9e8, so that reduction never changes a value and no test can see it.
    "setup_split": ("int64_t a = q / 30082, b = q % 30082;", "int64_t a = q / 30081, b = q % 30081;"),
    "setup_i_divisor": ("out[0] = (int32_t)((a / 177) % 177 + 2);", "out[0] = (int32_t)((a / 178) % 177 + 2);"),
    "setup_i_offset": ("out[0] = (int32_t)((a / 177) % 177 + 2);", "out[0] = (int32_t)((a / 177) % 177 + 1);"),
    "setup_j_modulus": ("out[1] = (int32_t)(a % 177 + 2);", "out[1] = (int32_t)(a % 178 + 2);"),
    "setup_j_offset": ("out[1] = (int32_t)(a % 177 + 2);", "out[1] = (int32_t)(a % 177 + 1);"),
    "setup_k_modulus": ("out[2] = (int32_t)((b / 169) % 178 + 1);", "out[2] = (int32_t)((b / 169) % 177 + 1);"),
    "setup_k_offset": ("out[2] = (int32_t)((b / 169) % 178 + 1);", "out[2] = (int32_t)((b / 169) % 178 + 2);"),
    "setup_k_divisor": ("out[2] = (int32_t)((b / 169) % 178 + 1);", "out[2] = (int32_t)((b / 168) % 178 + 1);"),
    "setup_l_modulus": ("out[3] = (int32_t)(b % 169);", "out[3] = (int32_t)(b % 168);"),
    # Appendix A: the two small generators, the bits and the words.
    "product_modulus": ("int32_t m_n = (int32_t)(((int64_t)m_prev[0] * m_prev[1] % 179) * m_prev[2] % 179);",
                        "int32_t m_n = (int32_t)(((int64_t)m_prev[0] * m_prev[1] % 179) * m_prev[2] % 178);"),
    "product_shift_order": ("        m_prev[0] = m_prev[1];\n        m_prev[1] = m_prev[2];\n",
                            "        m_prev[1] = m_prev[2];\n        m_prev[0] = m_prev[1];\n"),
    "lcg_multiplier": ("int32_t l_n = (53 * l_prev + 1) % 169;", "int32_t l_n = (35 * l_prev + 1) % 169;"),
    "lcg_increment": ("int32_t l_n = (53 * l_prev + 1) % 169;", "int32_t l_n = (53 * l_prev + 2) % 169;"),
    "lcg_modulus": ("int32_t l_n = (53 * l_prev + 1) % 169;", "int32_t l_n = (53 * l_prev + 1) % 168;"),
    "bit_threshold": ("return (l_n * m_n) % 64 >= 32;", "return (l_n * m_n) % 64 > 32;"),
    "bit_modulus": ("return (l_n * m_n) % 64 >= 32;", "return (l_n * m_n) % 128 >= 64;"),
    "bit_order": ("word = 2 * word + (uint32_t)seed_bit_of(mseq[n], lseq[n]);",
                  "word = word + ((uint32_t)seed_bit_of(mseq[n], lseq[n]) << p);"),
    "word_orientation": ("for (int k = 0; k < 97; ++k) W[k] = u[97 - k] & ORC_MASK;",
                         "for (int k = 0; k < 97; ++k) W[k] = u[k + 1] & ORC_MASK;"),
    # Appendix A: the real route's own set-up and stepping.
    "real_setup_i": ("g.p0 = 2 + (q / (30082L * 177)) % 177;", "g.p0 = 2 + (q / (30082L * 178)) % 177;"),
    "real_setup_k": ("g.p2 = 1 + (lo / 169) % 178;", "g.p2 = 1 + (lo / 169) % 177;"),
    "real_lcg": ("g->lc = (g->lc * 53 + 1) % 169;", "g->lc = (g->lc * 53 + 1) % 168;"),
    "real_bit": ("return (int)((prod * g->lc) % 64 / 32);", "return (int)((prod * g->lc) % 64 / 33);"),
    "real_weight": ("for (int h = 0; h < p; ++h) weight *= 0.5;", "for (int h = 1; h < p; ++h) weight *= 0.5;"),
    "real_orientation": ("for (int k = 0; k < 97; ++k) x[k] = u[97 - k];",
                         "for (int k = 0; k < 97; ++k) x[k] = u[k + 1];"),
}

# Seeds that reach every part of the set-up: both ends of the low part (the
# top one has k = 178), the second block, the first i step (high part 177), a large and the largest seed.
SEEDS = (1, 12345, 30082, 30083, 5324515, 777777777, 900000000)


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
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.orc_seed_setup.argtypes = [i64, i32p]
    L.orc_seed_sequences.argtypes = [i32p, ctypes.c_int32, i32p, i32p]
    L.orc_seed_int.argtypes = [i64, u32p]
    return L


class _Seeding:
    """The oracle's initialisation routines from one built copy."""

    def __init__(self, L):
        self.L = L

    def setup(self, seed):
        out = np.zeros(4, np.int32)
        assert self.L.orc_seed_setup(seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))) == 0
        return tuple(int(v) for v in out)

    def sequences(self, start, count):
        st = np.ascontiguousarray(np.asarray(start, np.int32))
        m, l = np.zeros(count, np.int32), np.zeros(count, np.int32)
        p = ctypes.POINTER(ctypes.c_int32)
        self.L.orc_seed_sequences(st.ctypes.data_as(p), count, m.ctypes.data_as(p), l.ctypes.data_as(p))
        return m, l

    def seed_int(self, seed):
        u = np.zeros(98, np.uint32)
        assert self.L.orc_seed_int(seed, _u(u)) == 0
        return u

    def int_draws(self, seed, n):
        out = np.zeros(n, np.uint32)
        assert self.L.orc_int_draws(seed, n, _u(out)) == 0
        return out


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
    # The real route == the integer route, scaled by 2^24 (Sec. 3.1, sigma;
    # Appendix A), on seeds that reach every part of the set-up.
    for seed in SEEDS:
        n = 3000
        real = np.zeros(n, np.float64)
        ints = np.zeros(n, np.uint32)
        L.orc_real_draws(seed, n, real.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        L.orc_int_draws(seed, n, _u(ints))
        if not np.array_equal(real * 2.0 ** 24, ints.astype(np.float64)):
            fails.append("real_vs_int")
            break
    # Appendix A: what the printed constants fix about the initialisation.
    sd = _Seeding(L)
    fails += seed_pins.check_setup_low_part(sd.setup)
    fails += seed_pins.check_setup_high_part(sd.setup)
    fails += seed_pins.check_product_generator(sd.setup, sd.sequences, SEEDS, steps=300)
    fails += seed_pins.check_congruential_generator(sd.sequences)
    fails += seed_pins.check_first_draws(sd.seed_int, sd.int_draws, SEEDS)
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
    if not fails:
        # The only costly pin: real == integer through the draw at which c
        # passes exactly through 0 (c_n = 0 for n = c_0 / d mod m).
        n0 = C0 * pow(D, -1, MOD) % MOD
        n = n0 + 200
        real = np.zeros(n, np.float64)
        ints = np.zeros(n, np.uint32)
        L.orc_real_draws(12345, n, real.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        L.orc_int_draws(12345, n, _u(ints))
        if not np.array_equal(real[n0 - 200:] * 2.0 ** 24, ints[n0 - 200:].astype(np.float64)):
            fails.append("real_vs_int_through_c_zero")
    return fails


def test_unmodified_oracle_passes_every_pin(orc, tmp_path):
    assert _failures(_build(tmp_path, "orig", open(SRC).read()), orc) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(orc, tmp_path, name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found once: {name}"
    assert _failures(_build(tmp_path, name, text.replace(old, new)), orc), f"no pin catches {name}"
