"""The algebra behind the product form of stream families, checked on the CPU
against the oracle's jumps (Sec. 3.1: a jump by J is the matrix P_J(A_c)
acting on the row vector of the window).

The GPU path forms start j*A + i of a family as x_i times one factor matrix
Q_j shared by A starts, reads Q_j from a single extended sequence instead of
97 jumped unit windows, and multiplies in signed 8-bit digits.  Each identity
is compared with a different route to the same value: unit windows jumped by
the oracle, states jumped directly, exact integer products.
"""
import numpy as np
import pytest

import synth

MASK = (1 << 24) - 1


def _unit(r):
    e = np.zeros(97, np.uint32)
    e[r] = 1
    return e


def _factor_rows(orc, J):
    """Rows of P_J(A_c) mod 2^24: unit window e_r jumped by J."""
    P = orc.xpow(J)
    return np.stack([orc.apply(_unit(r), P) for r in range(97)]).astype(np.int64)


def _h(orc, J):
    """Terms J .. J+192 of the sequence started from e_96, by two jumps."""
    a = orc.apply(_unit(96), orc.xpow(J)).astype(np.int64)
    b = orc.apply(_unit(96), orc.xpow(J + 96)).astype(np.int64)
    return np.concatenate([a, b[1:]])


@pytest.mark.parametrize("J", [0, 1, 33, 97, 4096, (7 << 48) + 5, (1 << 119) + 12345])
def test_factor_rows_from_one_sequence(orc, J):
    """Q_J[r][l] = h[l + 96 - r] + (r <= 63 ? h[l + 63 - r] : 0) mod 2^24."""
    Q = _factor_rows(orc, J)
    h = _h(orc, J)
    for r in range(97):
        for l in range(97):
            v = h[l + 96 - r] + (h[l + 63 - r] if r <= 63 else 0)
            assert Q[r, l] == v & MASK, (J, r, l)


def test_factor_rows_are_two_toeplitz_bands(orc):
    """Entries depend only on l - r within rows 0..63 and within rows 64..96."""
    Q = _factor_rows(orc, 123456789)
    for r0, r1 in ((0, 63), (64, 96)):
        for r in range(r0, r1):
            assert np.array_equal(Q[r, :-1], Q[r + 1, 1:])


def test_family_start_is_source_times_shared_factor(orc):
    """x_(jA+i) = x_i Q_j with Q_j the factor of j*A*delta (mod 2^24)."""
    base = orc.state_from_seed(4711)
    delta, A = (1 << 40) + 7, 48
    g = synth.rng(301)
    for _ in range(3):
        i, j = int(g.integers(0, A)), int(g.integers(1, 40))
        xi = orc.jump(base, i * delta)[:97].astype(np.int64)
        Q = _factor_rows(orc, j * A * delta)
        got = (xi @ Q) & MASK
        expect = orc.jump(base, (j * A + i) * delta)[:97].astype(np.int64)
        assert np.array_equal(got, expect)


def _digits(v):
    """Signed 8-bit digits from the bytes of (v + 0x808080) xor 0x808080."""
    e = ((v + 0x808080) ^ 0x808080) & 0xFFFFFF
    return [(((e >> (8 * k)) & 0xFF) ^ 0x80) - 0x80 for k in range(3)]


def test_signed_digits_reconstruct():
    g = synth.rng(302)
    vals = np.concatenate([g.integers(0, 1 << 24, size=20000), [0, 1, 127, 128, 255, 256, 0x7F7F7F, 0x808080,
                                                                   MASK - 1, MASK]])
    for v in vals.tolist():
        d = _digits(v)
        assert all(-128 <= x <= 127 for x in d)
        assert (d[0] + 256 * d[1] + 65536 * d[2]) & MASK == v


def test_six_digit_products_give_the_product_mod_2_24():
    """W Q mod 2^24 from the six digit products of weight below 2^24, with
    each partial sum inside int32 (97 terms of magnitude <= 2^14 each)."""
    g = synth.rng(303)
    W = g.integers(0, 1 << 24, size=(16, 97), dtype=np.int64)
    Q = g.integers(0, 1 << 24, size=(97, 97), dtype=np.int64)
    Wd = [np.vectorize(lambda v, k=k: _digits(int(v))[k])(W) for k in range(3)]
    Qd = [np.vectorize(lambda v, k=k: _digits(int(v))[k])(Q) for k in range(3)]
    parts = {}
    for a in range(3):
        for b in range(3 - a):
            p = Wd[a] @ Qd[b]
            assert np.abs(p).max() <= 97 * 128 * 128 < 2 ** 31
            parts[(a, b)] = p
    y = (parts[(0, 0)] + ((parts[(0, 1)] + parts[(1, 0)]) << 8)
         + ((parts[(0, 2)] + parts[(1, 1)] + parts[(2, 0)]) << 16)) & MASK
    exact = np.array([[sum(int(W[m, k]) * int(Q[k, o]) for k in range(97)) & MASK for o in range(97)]
                      for m in range(16)])
    assert np.array_equal(y, exact)
