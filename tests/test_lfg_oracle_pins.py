"""Pins of the general-generator oracle (arbitrary r, s, e, m, d; Sec. 2 and
Sec. 5) against what the paper and the mathematics fix.

- Reduction: with RANMAR's parameters it must reproduce the RANMAR oracle,
  which the paper's algorithms pin (Algorithm 1 == Algorithm 2, closed forms,
  the order of t).
- Brute force: the polynomial jump (Sec. 3.1, 3.2) must reach the state of J
  literal transitions, for small generators of every shape (s = 1, s = r - 1,
  s > r/2, e = 1, e = 32, m = 1).
- Closed forms: t^J mod phi for J <= r + s follows from phi = t^r + t^(r-s) - 1
  alone (Sec. 3.1).
- Number theory: when t^r + t^(r-s) + 1 is primitive over GF(2) (checked here
  with independent GF(2) arithmetic), the order of t modulo phi over Z/2^e is
  2^(e-1) (2^r - 1) (Brent, "On the periods of generalized Fibonacci
  recurrences", Math. Comp. 63, 1994); for RANMAR this is the period behind
  the paper's figure of about 2^144 (Sec. 2).
"""
import numpy as np
import pytest

import synth

LFG_CASES = synth.LFG_CASES


def _one(r):
    v = np.zeros(r, np.uint32)
    v[0] = 1
    return v


# --- validation ----------------------------------------------------------------
@pytest.mark.parametrize("bad", [(1, 1, 24, 3, 1), (5, 0, 8, 7, 1), (5, 5, 8, 7, 1), (5, 2, 0, 1, 0),
                                 (5, 2, 33, 7, 1), (5, 2, 8, 0, 0), (5, 2, 8, 256, 1), (5, 2, 8, 7, 7)])
def test_rejects_invalid_parameters(orc, bad):
    with pytest.raises(ValueError):
        orc.LFG(*bad)


# --- reduction to RANMAR ---------------------------------------------------------
def test_ranmar_parameters_reduce_to_ranmar(orc):
    """With (97, 33, 24, 2^24 - 3, 7654321) every routine equals the RANMAR
    oracle's (a separate implementation pinned to the paper)."""
    g = orc.LFG(*orc.RANMAR_PARAMS)
    states = np.stack([orc.state_from_seed(s) for s in (1, 12345, 900000000)])
    a, sa = g.draws_many(states, 3000)
    b, sb = orc.draws_many(states, 3000)
    assert np.array_equal(a, b) and np.array_equal(sa, sb)
    Js = [0, 1, 96, 97, 98, 130, 10**6, (1 << 64) - 1, (1 << 120) - 1, 3 * 10**35]
    assert np.array_equal(g.xpow_many(Js), orc.xpow_many(Js))
    for J in Js[:6] + Js[-2:]:
        assert np.array_equal(g.jump_many(states[1:2], [J])[0], orc.jump(states[1], J))
        assert g.c_jump(orc.C0, J) == orc.c_jump(orc.C0, J)


# --- brute force -----------------------------------------------------------------
SMALL = ["r2s1e3", "r5s1e8", "r5s4e8", "r7s3e8", "r7s6e1", "r10s7e16", "r17s3e32", "r33s32e24", "r55s24e32"]


@pytest.mark.parametrize("name", SMALL)
def test_jump_equals_stepping(orc, name):
    """Sec. 3.1 (Cayley-Hamilton) and Sec. 3.2 for general (r, s, e, m, d):
    the polynomial jump equals J literal transitions."""
    g = orc.LFG(*LFG_CASES[name])
    r, s = g.r, g.s
    st = synth.lfg_states(g.r, g.e, g.m, 3, offset=11)
    Js = sorted({0, 1, s - 1, s, s + 1, r - 1, r, r + 1, r + s, 2 * r - 1, 2 * r, 3 * r + 5, 1000, 4097})
    Js = [J for J in Js if J >= 0]
    for q in range(3):
        got = g.jump_many(np.repeat(st[q:q + 1], len(Js), 0), Js)
        for k, J in enumerate(Js):
            assert np.array_equal(got[k], g.step(st[q], J)), (name, q, J)


@pytest.mark.parametrize("name", SMALL)
def test_draws_equal_stepping(orc, name):
    """Draw q is (newest word - c) mod 2^e of the state after q + 1 transitions."""
    g = orc.LFG(*LFG_CASES[name])
    st = synth.lfg_states(g.r, g.e, g.m, 1, offset=12)[0]
    out, after = g.draws_many(st, 200)
    for q in (0, 1, g.s, g.r, 199):
        w = g.step(st, q + 1)
        assert out[0, q] == (int(w[g.r - 1]) - int(w[g.r])) & g.mask
    assert np.array_equal(after[0], g.step(st, 200))


def test_jump_composition_large_r(orc):
    """P_{a+b} route: jump(a) then jump(b) equals jump(a + b), at r = 1279."""
    g = orc.LFG(*LFG_CASES["r1279s418e32"])
    st = synth.lfg_states(g.r, g.e, g.m, 1, offset=13)
    a, b = (1 << 70) + 12345, (1 << 33) + 7
    ab = g.jump_many(g.jump_many(st, [a]), [b])
    assert np.array_equal(ab, g.jump_many(st, [a + b]))
    # and a short jump against literal stepping at this size
    assert np.array_equal(g.jump_many(st, [3000])[0], g.step(st[0], 3000))


# --- closed forms ------------------------------------------------------------------
@pytest.mark.parametrize("name", SMALL + ["ranmar", "r97s64e24", "r607s273e24"])
def test_small_powers(orc, name):
    """t^J for J < r is a monomial; t^r = 1 - t^(r-s); t^(r+k) = t^k - t^(r-s+k)
    for 0 < k < s; t^(r+s) = t^s - 1 + t^(r-s)."""
    g = orc.LFG(*LFG_CASES[name])
    r, s, M = g.r, g.s, g.mask
    Js = list(range(0, r + s + 1))
    if r > 100:  # keep the oracle's cost small at large r
        Js = sorted({0, 1, s, r - 1, r, r + 1, r + s - 1, r + s})
    P = g.xpow_many(Js).astype(np.int64)
    for row, J in enumerate(Js):
        expect = np.zeros(r, np.int64)
        if J < r:
            expect[J] = 1
        elif J < r + s:
            k = J - r
            expect[k] += 1
            expect[r - s + k] -= 1
        else:
            expect[s] += 1
            expect[0] -= 1
            expect[r - s] += 1
        assert np.array_equal(P[row], expect & M), (name, J)


# --- order of t (number theory) ------------------------------------------------------
def _gf2_mulmod(a, b, f, deg):
    out = 0
    while b:
        if b & 1:
            out ^= a
        b >>= 1
        a <<= 1
        if (a >> deg) & 1:
            a ^= f
    return out


def _gf2_powt(J, f, deg):
    """t^J mod f over GF(2), polynomials as bit masks."""
    res, base = 1, 2
    while J:
        if J & 1:
            res = _gf2_mulmod(res, base, f, deg)
        base = _gf2_mulmod(base, base, f, deg)
        J >>= 1
    return res


def _factor(n):
    out, p = [], 2
    while p * p <= n and p < 300000:
        while n % p == 0:
            out.append(p)
            n //= p
        p += 1
    if n > 1:
        out.append(n)  # remaining cofactor: checked prime below
    return sorted(set(out))


def _probable_prime(n):
    if n < 2:
        return False
    d, k = n - 1, 0
    while d % 2 == 0:
        d //= 2
        k += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if a % n == 0:
            continue
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(k - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _primitive_mod2(r, s):
    """t^r + t^(r-s) + 1 primitive over GF(2): order of t is exactly 2^r - 1."""
    f = (1 << r) | (1 << (r - s)) | 1
    N = (1 << r) - 1
    primes = _factor(N)
    assert all(_probable_prime(p) for p in primes)
    if _gf2_powt(N, f, r) != 1:
        return False
    return all(_gf2_powt(N // p, f, r) != 1 for p in primes)


@pytest.mark.parametrize("name", ["r7s3e8", "r17s3e32", "r31s28e16", "r55s24e32", "ranmar", "r97s64e24"])
def test_order_of_t(orc, name):
    g = orc.LFG(*LFG_CASES[name])
    r, s, e = g.r, g.s, g.e
    assert _primitive_mod2(r, s), "test case must use a primitive trinomial"
    N = (1 << r) - 1
    L = N << (e - 1)
    one = _one(r)
    assert np.array_equal(g.xpow(L), one)
    for p in _factor(N) + [2]:
        if L % p == 0:
            assert not np.array_equal(g.xpow(L // p), one), (name, p)


def test_non_primitive_trinomial_detected():
    """Guard on the helper itself: t^4 + t^2 + 1 = (t^2 + t + 1)^2 over GF(2)."""
    assert not _primitive_mod2(4, 2)
    assert _primitive_mod2(7, 3)


# --- arithmetic sequence -------------------------------------------------------------
@pytest.mark.parametrize("name", ["r5s1e8", "r17s3e32", "ranmar", "r55s24e32"])
def test_c_jump(orc, name):
    """Sec. 3.2: c_J = (c - J d) mod m; c has period m."""
    g = orc.LFG(*LFG_CASES[name])
    st = synth.lfg_states(g.r, g.e, g.m, 1, offset=14)[0]
    c = int(st[g.r])
    for J in (0, 1, 2, 17, 1000):
        assert g.c_jump(c, J) == int(g.step(st, J)[g.r])
    assert g.c_jump(c, g.m) == c
    big = (1 << 127) + 12345
    assert g.c_jump(c, big) == g.c_jump(c, big % g.m)


@pytest.mark.parametrize("name", ["r2s1e3", "r5s1e8", "r10s7e16"])
def test_c_sequence_every_start(orc, name):
    """Sec. 2 (f_2): from every c_0 in [0, m), k transitions give
    (c_0 - k d) mod m, always below m (the boundary c = d included)."""
    g = orc.LFG(*synth.LFG_CASES[name])
    u = np.zeros(g.r + 1, np.uint32)
    for c0 in sorted(set(range(min(g.m, 40))) | {g.d, (g.d + 1) % g.m, g.m - 1}):
        u[g.r] = c0
        for k in (1, 2, g.m - 1, g.m, 2 * g.m + 3):
            c = int(g.step(u, k)[g.r])
            assert c == (c0 - k * g.d) % g.m and c < g.m, (name, c0, k)

