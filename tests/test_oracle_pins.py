"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper prints no sample draws, so every pin here is a closed form, an
identity between two formulations the paper asserts are equal, a group law,
brute force on small inputs, or a number-theoretic fact (the order of t modulo
phi).  Each test names the passage it rests on.  None of them retypes an
oracle formula: they compare the oracle against a different route to the same
value.
"""
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MASK = (1 << 24) - 1


def _golden_params():
    out = {}
    with open(os.path.join(GOLDEN, "paper_parameters.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split(None, 1)
                out[k] = v.strip()
    return out


def test_oracle_constants_match_paper(orc):
    """Sec. 2 and Algorithm 3 constants as printed."""
    g = _golden_params()
    assert (orc.R, orc.S, orc.E) == (int(g["r"]), int(g["s"]), int(g["e"]))
    assert orc.MOD == int(g["m"]) == int(g["M"]) - 3
    assert orc.D == int(g["d_num"]) and orc.C0 == int(g["c_num"])
    # P_97 = t^97 mod phi encodes phi's low terms: t^97 = 1 - t^64 (Sec. 3.1).
    phi = dict((int(a), int(b)) for a, b in (t.split(":") for t in g["phi_terms"].split(",")))
    P97 = orc.xpow(97)
    expect = np.zeros(97, np.int64)
    for e_, c_ in phi.items():
        if e_ < 97:
            expect[e_] = (-c_) & MASK
    assert np.array_equal(P97.astype(np.int64), expect)


SEEDS = [1, 2, 12345, 4711, 900000, 900000000, 31328, 777777777]


@pytest.mark.parametrize("seed", SEEDS)
def test_real_equals_integer_draws(orc, seed):
    """Sec. 3.1 isomorphism sigma and Sec. 4: Algorithm 2 equals Algorithm 1.

    The real-arithmetic generator (Algorithm 1, seeded in real arithmetic) and
    the integer generator (Algorithm 2, seeded by Algorithm 3) must agree
    exactly after scaling by 2^24."""
    n = 1_000_000 if seed == 12345 else 100_000
    real = orc.real_draws(seed, n)
    ints = orc.int_draws(seed, n)
    scaled = real * float(1 << 24)
    assert np.all(scaled == np.floor(scaled))
    assert np.array_equal(scaled.astype(np.uint32), ints)
    assert ints.max() <= MASK


def test_real_equals_integer_through_c_zero(orc):
    """c_n = 0 is a legal value reached once every m draws, at n = c_0 / d
    mod m (15,418,204 from the initial c); both routes must agree through it
    (the real route steps c in real numbers with a wrap below zero, the
    integer route takes c_n from its closed form)."""
    n0 = orc.C0 * pow(orc.D, -1, orc.MOD) % orc.MOD
    assert (orc.C0 - n0 * orc.D) % orc.MOD == 0
    n = n0 + 1000
    real = orc.real_draws(12345, n)[n0 - 1000:]
    ints = orc.int_draws(12345, n)[n0 - 1000:]
    assert np.array_equal(real * float(1 << 24), ints.astype(np.float64))


@pytest.mark.parametrize("seed", SEEDS)
def test_real_equals_integer_seeding(orc, seed):
    """Appendix A: Algorithm 3 reproduces the real-arithmetic initialisation."""
    ur = orc.seed_real(seed)[1:]
    ui = orc.seed_int(seed)[1:]
    assert np.array_equal((ur * float(1 << 24)).astype(np.uint32), ui)
    assert ui.max() <= MASK


def test_seed_range(orc):
    """Algorithm 3 accepts seeds up to 9e8; seed 0 has no defined Quotient of -1."""
    for bad in (0, -5, 900000001):
        with pytest.raises(ValueError):
            orc.state_from_seed(bad)
    orc.state_from_seed(900000000)


# --- Appendix A: the initialisation's set-up and small generators -------------
import seed_pins  # noqa: E402


def test_seed_setup_low_part_is_a_bijection(orc):
    """30082 = 178 * 169: inside a block of 30082 seeds, (k, l) runs once over
    [1, 178] x [0, 168] while (i, j) stays fixed (Algorithm 3's set-up)."""
    assert seed_pins.check_setup_low_part(orc.seed_setup) == []


def test_seed_setup_is_injective_and_non_degenerate(orc):
    """The high part of s - 1 is below 177^2, so (i, j) differs for every
    block; every start value is a non-zero residue mod 179 and the three
    product-generator values are never all 1."""
    assert seed_pins.check_setup_high_part(orc.seed_setup) == []


def test_product_generator_exponent_form(orc):
    """m_n = g^(e_n) mod 179 with e_n = e_(n-1) + e_(n-2) + e_(n-3) mod 178:
    the lag-3 product generator computed through discrete logarithms."""
    seeds = [1, 2, 170, 12345, 30083, 5324515, 777777777, 900000000]
    assert seed_pins.check_product_generator(orc.seed_setup, orc.seed_sequences, seeds) == []


def test_congruential_generator_closed_form_and_period(orc):
    """l_n = 53^n l_0 + (53^n - 1)/52 mod 169, and full period 169 from every
    start (Hull-Dobell)."""
    assert seed_pins.check_congruential_generator(orc.seed_sequences) == []


def test_first_draws_read_the_seeded_words_top_down(orc):
    """The generator starts its pointers at 97 and 33: draw q <= 33 is
    u_(98-q) - u_(34-q) - c_q mod 2^24, straight from the seeded array."""
    seeds = [1, 12345, 4711, 900000, 900000000]
    assert seed_pins.check_first_draws(orc.seed_int, orc.int_draws, seeds) == []


def test_real_and_integer_seeding_agree_across_the_seed_range(orc):
    """The two independent routes of the initialisation (real: words as sums
    of 2^-p, its own index arithmetic; integer: 24-bit words from the bit
    sequence) agree exactly on seeds spread over every part of the set-up."""
    g = synth.rng(106)
    seeds = [1, 2, 169, 170, 30082, 30083, 5324514, 5324515, 899993277, 900000000]
    seeds += [int(v) for v in g.integers(1, 900_000_001, size=300)]
    for s in seeds:
        ur = orc.seed_real(s)[1:]
        ui = orc.seed_int(s)[1:]
        assert np.array_equal(ur * float(1 << 24), ui.astype(np.float64)), s


def _literal_quotient_words(seed, words=97):
    """Algorithm 3 with the printed Quotient(i*j, 179) taken literally."""
    ij = (seed - 1) // 30082
    kl = (seed - 1) - 30082 * ij
    i, j = (ij // 177) % 177 + 2, ij % 177 + 2
    k, l = (kl // 169) % 178 + 1, kl % 169
    out = []
    for _ in range(words):
        s, t = 0, 1 << 31
        for _ in range(24):
            m = ((i * j) // 179) * k % 179
            i, j, k = j, k, m
            l = (53 * l + 1) % 169
            if (l * m) % 64 >= 32:
                s += t
            t //= 2
        out.append(s >> 8)
    return out


def test_remainder_reading_of_algorithm3(orc):
    """Appendix A, Algorithm 3: read Quotient(i*j,179) as Remainder.

    Taken literally, seed 1 gives i*j = 4 < 179, the quotient 0, and from then
    on m = 0 for ever: all 97 words are zero and the generator degenerates,
    which contradicts the claim that the integer initialisation matches the
    real one.  The Remainder reading keeps m in [1, 178] (179 is prime)."""
    assert all(w == 0 for w in _literal_quotient_words(1))
    u = orc.seed_int(1)[1:]
    assert np.count_nonzero(u) > 80
    # 179 prime: the product of non-zero residues never vanishes.
    assert all(179 % p for p in range(2, 14))


def test_draws_follow_the_recurrence_definition(orc):
    """Sec. 2 definition: x_n = x_{n-97} - x_{n-33} mod 1 and c_n = c_{n-1} - d.

    Recover x from each output y_n = x - c_n using the closed form of c_n
    (Sec. 3.2) and check the lagged recurrence from the seeded words on."""
    seed, n = 4711, 20000
    y = orc.int_draws(seed, n).astype(np.int64)
    idx = np.arange(1, n + 1, dtype=np.int64)
    c = (orc.C0 - (idx % orc.MOD) * orc.D) % orc.MOD
    xnew = (y + c) & MASK
    W = orc.state_from_seed(seed)[:97].astype(np.int64)
    x = np.concatenate([W, xnew])           # x_1 .. x_{97+n}
    lhs = x[97:]
    rhs = (x[:-97] - x[64:-33]) & MASK
    assert np.array_equal(lhs, rhs)


def test_canonical_state_roundtrip(orc):
    """Running Algorithm 2 from the automaton state equals running it from
    the seed, and a split run equals one long run (state export is exact)."""
    for seed in (1, 12345, 900000000):
        st = orc.state_from_seed(seed)
        ref = orc.int_draws(seed, 5000)
        out, st2 = orc.state_draws(st, 5000)
        assert np.array_equal(out, ref)
        a, sa = orc.state_draws(st, 1234)
        b, sb = orc.state_draws(sa, 5000 - 1234)
        assert np.array_equal(np.concatenate([a, b]), ref)
        assert np.array_equal(sb, st2)
        assert st2[:97].max() <= MASK and st2[97] < orc.MOD


# --- Sec. 3.1: P_J = t^J mod phi --------------------------------------------
def test_small_powers_are_monomials(orc):
    """t^J has degree < 97 for J < 97, so P_J = t^J exactly."""
    for J in list(range(0, 97)):
        P = orc.xpow(J)
        e = np.zeros(97, np.uint32)
        e[J] = 1
        assert np.array_equal(P, e), J


def test_powers_just_above_the_degree(orc):
    """phi = t^97 + t^64 - 1 gives t^(97+j) = t^j - t^(64+j) for j <= 32 and,
    reducing t^(64+j) again, t^j - t^(j-33) + t^(j+31) for 33 <= j <= 65."""
    for j in range(0, 33):
        P = orc.xpow(97 + j).astype(np.int64)
        e = np.zeros(97, np.int64)
        e[j] += 1
        e[64 + j] -= 1
        assert np.array_equal(P, e & MASK), j
    for j in range(33, 66):
        P = orc.xpow(97 + j).astype(np.int64)
        e = np.zeros(97, np.int64)
        e[j] += 1
        e[j - 33] -= 1
        e[j + 31] += 1
        assert np.array_equal(P, e & MASK), j


def test_power_law(orc):
    """P_a P_b = P_(a+b) mod phi for 120-bit exponents (t^a t^b = t^(a+b))."""
    g = synth.rng(101)
    lo, hi = synth.u128_uniform(g, 12, 120)
    Js = synth.u128_to_int(lo, hi)
    for a, b in zip(Js[0::2], Js[1::2]):
        assert np.array_equal(orc.poly_mulmod(orc.xpow(a), orc.xpow(b)), orc.xpow(a + b))
        assert np.array_equal(orc.poly_mulmod(orc.xpow(a), orc.xpow(a)), orc.xpow(2 * a))


def _is_probable_prime(n):
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71]
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_order_of_t_modulo_phi(orc):
    """The lagged Fibonacci part has period (2^97 - 1) 2^23 (the stated period
    of about 2^144 is this times m): t^L = 1 mod phi over Z/2^24 for
    L = (2^97-1) 2^23, and t^(L/p) != 1 for each prime p dividing L.

    A wrong reduction polynomial, a sign error or a dropped carry in the
    powering would change this order."""
    p1, p2 = 11447, 13842607235828485645766393
    assert p1 * p2 == (1 << 97) - 1
    assert _is_probable_prime(p1) and _is_probable_prime(p2)
    L = ((1 << 97) - 1) << 23
    one = np.zeros(97, np.uint32)
    one[0] = 1
    assert np.array_equal(orc.xpow(L), one)
    for p in (2, p1, p2):
        assert not np.array_equal(orc.xpow(L // p), one), p


def test_period_statement(orc):
    """Sec. 2: the full period is about 2^144; L * m with gcd(L, m) = 1."""
    L = ((1 << 97) - 1) << 23
    g = _golden_params()
    assert math.gcd(L, orc.MOD) == 1
    assert abs(math.log2(L * orc.MOD) - int(g["period_log2"])) < 0.5
    # c has period exactly m: jumping c by m is the identity (Sec. 3.2).
    for c in (0, 1, orc.C0, orc.MOD - 1):
        assert orc.c_jump(c, orc.MOD) == c
        assert orc.c_jump(c, 5 * orc.MOD + 17) == orc.c_jump(c, 17)


# --- jump-ahead ---------------------------------------------------------------
JUMPS_SMALL = [0, 1, 2, 32, 33, 34, 63, 64, 65, 96, 97, 98, 99, 129, 130, 193, 194, 1000, 4097]


@pytest.mark.parametrize("seed", [1, 12345, 900000000])
def test_jump_equals_stepping(orc, seed):
    """Sec. 3.1 (Cayley-Hamilton) and Sec. 3.2: the jump reaches exactly the
    state of J single transitions (brute force)."""
    st = orc.state_from_seed(seed)
    g = synth.rng(102 + seed % 7)
    Js = JUMPS_SMALL + [int(v) for v in g.integers(0, 100_000, size=8)]
    for J in Js:
        assert np.array_equal(orc.jump(st, J), orc.step(st, J)), J


def test_jump_equals_stepping_large(orc):
    """Config-1 size: J = 2^20 and J = 10^6 against brute force."""
    st = orc.state_from_seed(12345)
    for J in (1 << 20, 1_000_000):
        assert np.array_equal(orc.jump(st, J), orc.step(st, J))


def test_jump_then_draw_matches_offset(orc):
    """Offset J means the first draw of the jumped stream is draw J+1."""
    seed = 31328
    ref = orc.int_draws(seed, 3000)
    st = orc.state_from_seed(seed)
    for J in (0, 1, 97, 1000, 2000):
        out, _ = orc.state_draws(orc.jump(st, J), 1000)
        assert np.array_equal(out, ref[J:J + 1000]), J


def test_jump_composition(orc):
    """f^a o f^b = f^(a+b) for 120-bit a, b."""
    g = synth.rng(103)
    lo, hi = synth.u128_uniform(g, 8, 120)
    Js = synth.u128_to_int(lo, hi)
    st = orc.state_from_seed(4711)
    for a, b in zip(Js[0::2], Js[1::2]):
        assert np.array_equal(orc.jump(orc.jump(st, a), b), orc.jump(st, a + b))


def test_apply_is_linear(orc):
    """uP(A) is linear in u over Z/2^24."""
    g = synth.rng(104)
    P = orc.xpow(123456789012345)
    for _ in range(4):
        u = g.integers(0, 1 << 24, size=97, dtype=np.int64)
        v = g.integers(0, 1 << 24, size=97, dtype=np.int64)
        al, be = (int(x) for x in g.integers(0, 1 << 24, size=2))
        lhs = orc.apply(((al * u + be * v) & MASK).astype(np.uint32), P).astype(np.int64)
        rhs = (al * orc.apply(u.astype(np.uint32), P).astype(np.int64)
               + be * orc.apply(v.astype(np.uint32), P).astype(np.int64)) & MASK
        assert np.array_equal(lhs, rhs)


def test_apply_equals_sequence_form(orc):
    """Since t^J = P_J mod phi and the sequence obeys phi, every later term is
    x_(n+J) = sum_i b_i x_(n+i): the new window is a Hankel product of P_J
    with the window extended by 96 steps of the recurrence."""
    g = synth.rng(105)
    for J in (5, 1000, (1 << 100) + 12345):
        P = orc.xpow(J).astype(object)
        W = [int(v) for v in g.integers(0, 1 << 24, size=97)]
        X = list(W)
        for n in range(96):
            X.append((X[n] - X[n + 64]) & MASK)
        expect = [sum(P[i] * X[i + l] for i in range(97)) & MASK for l in range(97)]
        got = orc.apply(np.array(W, np.uint32), orc.xpow(J))
        assert [int(v) for v in got] == expect


def test_config1_single_stream(orc):
    """Config 1: seed 12345, 10^6 draws, one jump of 2^20 against 2^20 steps."""
    p = synth.SINGLE_STREAM
    ints = orc.int_draws(p["seed"], p["draws"])
    real = orc.real_draws(p["seed"], p["draws"])
    assert np.array_equal((real * float(1 << 24)).astype(np.uint32), ints)
    st = orc.state_from_seed(p["seed"])
    assert np.array_equal(orc.jump(st, p["jump"]), orc.step(st, p["jump"]))
    # The continued stream after the jump is the tail of the long run.
    out, _ = orc.state_draws(orc.jump(st, 999_000), 1000)
    assert np.array_equal(out, ints[999_000:])
