"""Index simulation of the matrix-core family kernels (CPU only).

The product-form family (start s = j A + i is x_i P_j(A_c), Sec. 3.1; c by the
closed form of Sec. 3.2) runs as two launches, `k_family_l1` (direct starts
and the factors' sequences h) and `k_family_gemm` / `k_family_gemm32` (int8
MFMA products in 16- or 32-row tiles).  This test re-derives, from the host
launcher and the kernels' own index expressions, every global and LDS address
the two launches touch, for the family sizes the library and its tests use and
for every tiles-per-wave value the launcher can pick (1..8), and checks that
  - every read and write stays inside its buffer (the output [n][98], the
    factor buffer [(B-1)][196], the base record, each LDS array), and
  - every output word of rows [0, n) is written exactly once (row 0 not at all
    when the family is built in place), rows [0, A) by the first launch and
    rows [A, n) by the second.
It simulates addresses only, not values; the GPU tests check the values.
"""
import math

import numpy as np
import pytest

KW = 98          # words per state record
KH = 196         # words per factor sequence h (193 used)
SEQ = 240        # bytes per limb sequence
COPY = 6 * SEQ + 16   # bytes per shifted copy (16 copies)
TQ_BYTES = 16 * COPY
TB_BYTES = 6 * 256
L1_WORDS = 193 + 97


def _tally(count, rows, cols):
    """count[rows[k], cols[k]] += 1 for every k (repeats counted)."""
    count += np.bincount(np.asarray(rows, np.int64) * KW + cols, minlength=count.size).reshape(count.shape)


def launch_shape(n, tr, slots):
    """The host launcher's decisions: (A, B, tpw, gx), or None when the
    product form does not apply (the radix rounds then serve)."""
    A = math.ceil(math.sqrt(n) / tr) * tr
    A = max(A, tr)
    if 2 * A > n:
        return None
    B = (n + A - 1) // A
    all_tiles = (B - 1) * (A // tr)
    want = (all_tiles + 4 * slots - 1) // (4 * slots)
    tpw = min(8, max(1, want))
    return A, B, tpw


def sim_l1(n, A, B, in_place, seeded, count):
    """k_family_l1: grid (njobs + 7) / 8 workgroups of 256 threads, a job per
    half-wave (t = 8 block + half), lane l < 32."""
    njobs = A + B - 1
    blocks = (njobs + 7) // 8
    t = np.arange(blocks * 8, dtype=np.int64)
    block = t // 8
    hw = t % 8
    l = np.arange(32, dtype=np.int64)
    # LDS: the half-wave's window X (193 words) and polynomial Bp (97) in
    # lds[8 * 290]; the extension loop writes X[97 + s0 + l], reads X[s0 + l]
    # and X[s0 + l + 64] for s0 in {0, 32, 64}; h is read back as X[o], o < 193.
    lds_hi = hw[:, None] * L1_WORDS + np.maximum(96 + 64 + l, 193 + 96)[None, :]
    assert lds_hi.max() < 8 * L1_WORDS
    for s0 in (0, 32, 64):
        assert (97 + s0 + l).max() < 193 and (s0 + l + 64).max() < 193
    # Workgroups seeding together: seeded[96 - thread] for thread < 97.
    wg_seeds = seeded and ((block + 1) * 8 <= A)
    if np.any(wg_seeds):
        assert 96 - 0 < 97 and 96 - 96 >= 0
    active = t < njobs
    start = t < A
    if not seeded:  # base record: words l, l+32, l+64, 96 and c (97)
        assert max((l + 64).max(), 97) < KW
    # Direct starts: out[t][...] for active starts, except t = 0 in place.
    st = t[active & start & ~((t == 0) & in_place)]
    words = np.concatenate([l, l + 32, l + 64, [96, 97]])
    rows = np.repeat(st, words.size)
    cols = np.tile(words, st.size)
    assert rows.size == 0 or rows.max() < n
    _tally(count, rows, cols)
    # Factor sequences: H[(t - A) * 196 + o], o = l, l + 32, ... < 193.
    ft = t[active & ~start]
    o = np.arange(193)
    idx = ((ft - A)[:, None] * KH + o[None, :]).ravel()
    assert idx.size == 0 or (idx.min() >= 0 and idx.max() < (B - 1) * KH)
    assert ft.size == B - 1


def _lds_common(tr):
    """The limb-sequence set-up shared by both product kernels: hl reads,
    tb writes (entry m = thread < 256) and the shifted copies."""
    m = np.arange(256)
    i1, i2 = 208 - m, 175 - m
    assert np.all(((i1 >= 0) & (i1 <= 192)) <= ((i1 >= 0) & (i1 < 196)))
    assert (5 * 256 + m).max() < TB_BYTES
    if tr == 32:  # qcol[m] for m < 128 reads hl[192 - m] and hl[159 - m] for m < 97 / m <= 63
        mm = np.arange(97)
        assert (192 - mm).min() >= 0 and (159 - mm[mm <= 63]).min() >= 0
    # Shifted copies: wave w0 < 4, k < 24, it = w0 + 4k: copy c = it / 6,
    # sequence cb = it % 6; lane < 60 writes 4 bytes at c * COPY + cb * SEQ + 4 lane
    # and reads base words wi, wi + 1 with wi = cb * 64 + (c >> 2) + lane.
    it = (np.arange(4)[:, None] + 4 * np.arange(24)[None, :]).ravel()
    assert sorted(it.tolist()) == list(range(96))  # every (copy, sequence) once
    c, cb = it // 6, it % 6
    lane = np.arange(SEQ // 4)
    wr = (c * COPY + cb * SEQ)[:, None] + 4 * lane[None, :]
    assert wr.min() >= 0 and (wr + 4).max() <= TQ_BYTES
    wi = (cb * 64 + (c >> 2))[:, None] + lane[None, :]
    assert (wi + 1).max() < TB_BYTES // 4


def _tiles(A, tr, tpw):
    """Source tiles of every wave: workgroup x < gx, wave w < 4, tt < tpw
    take tile (4 x + w) tpw + tt; together they cover [0, A / tr) once."""
    tiles = A // tr
    gx = (tiles + 4 * tpw - 1) // (4 * tpw)
    t = ((np.arange(gx)[:, None, None] * 4 + np.arange(4)[None, :, None]) * tpw +
         np.arange(tpw)[None, None, :]).ravel()
    assert np.unique(t).size == t.size and set(range(tiles)) <= set(t.tolist())
    return t, tiles


def factor_stores(n, A, tpw, jq, tr):
    """(rows, columns) of every output word the product kernel stores for
    factor j = jq + 1, after checking the tile's source-record reads.  A
    wave stops at its first tile that is not ok (beyond A / tr tiles, or
    starting at or beyond row n); the later ones are not ok either."""
    t, tiles = _tiles(A, tr, tpw)
    j = jq + 1
    tl = t[(t < tiles) & (j * A + t * tr < n)]
    lane = np.arange(64)
    if tl.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if tr == 16:
        mrow, kg = lane & 15, lane >> 4
        # load_tile: words kk*64 + kg*16 + 4d + e (< 128) and 97 of record tile*16 + mrow.
        rec = tl[:, None] * 16 + mrow[None, :]
        assert rec.max() < A and rec.max() * KW + 127 < n * KW
        s0 = j * A + tl * 16
        rows = np.minimum(n - s0, 16)
        # Accumulator (lane, i) of column tile nt: row kg*4 + i, column nt*16 +
        # mrow; stored when (nt < 6 or mrow == 0) and the row is < rows.
        i, nt = np.arange(4), np.arange(7)
        r = kg[None, :, None, None] * 4 + i[None, None, None, :]
        col = nt[None, None, :, None] * 16 + mrow[None, :, None, None]
        keep = ((nt[None, None, :, None] < 6) | (mrow[None, :, None, None] == 0)) & (r < rows[:, None, None, None])
        keep = np.broadcast_to(keep, (tl.size, 64, 7, 4))
        # c: dst[lane * 98 + 97] for lane < rows.
        cl = np.broadcast_to(lane[None, :], (tl.size, 64))
        kc = cl < rows[:, None]
        extra_r = [(s0[:, None] + cl)[kc]]
        extra_c = [np.full(int(kc.sum()), 97)]
    else:
        mrow, kg = lane & 31, lane >> 5
        # load_tile32: words 32 kk + 16 kg + 4 d + e (< 96), 96 and 97 of record tile*32 + mrow.
        rec = tl[:, None] * 32 + mrow[None, :]
        assert rec.max() < A
        s0 = j * A + tl * 32
        rows = np.minimum(n - s0, 32)
        # Accumulator i of lane l: row 8 (i / 4) + 4 kg + i mod 4, column 32 nt + mrow.
        i, nt = np.arange(16), np.arange(3)
        r = 8 * (i // 4)[None, None, None, :] + 4 * kg[None, :, None, None] + (i % 4)[None, None, None, :]
        col = 32 * nt[None, None, :, None] + mrow[None, :, None, None]
        keep = np.broadcast_to(r < rows[:, None, None, None], (tl.size, 64, 3, 16))
        # Column 96 and c: lanes kg == 0 with mrow < rows.
        k0 = (kg[None, :] == 0) & (mrow[None, :] < rows[:, None])
        rr = (s0[:, None] + mrow[None, :])[k0]
        extra_r = [rr, rr]
        extra_c = [np.full(rr.size, 96), np.full(rr.size, 97)]
    R_ = np.broadcast_to(s0[:, None, None, None] + r, keep.shape)[keep]
    C_ = np.broadcast_to(col, keep.shape)[keep]
    R_ = np.concatenate([R_] + extra_r)
    C_ = np.concatenate([C_] + extra_c)
    assert R_.min() >= j * A and R_.max() < min(n, (j + 1) * A) and C_.min() >= 0 and C_.max() <= 97
    return R_, C_


def sim_product(n, A, B, tpw, tr, count):
    """k_family_gemm (tr = 16) or k_family_gemm32 (tr = 32): grid (gx, B - 1)
    of 4 waves x 64 lanes."""
    _lds_common(tr)
    lane = np.arange(64)
    if tr == 16:
        # B operand: qb = cq * COPY + (mrow == 0 ? 16 : 0) + 16 kg, then
        # (6 - nt) * 16 + kk * (3 * SEQ + 64) + b * SEQ, 16 bytes.
        mrow, kg = lane & 15, lane >> 4
        qb = ((16 - mrow) & 15) * COPY + np.where(mrow == 0, 16, 0) + 16 * kg
        offs = [qb + (6 - nt) * 16 + kk * (3 * SEQ + 64) + b * SEQ
                for nt in range(7) for kk in range(2) for b in range(3)]
    else:
        # B operand: qb = cq * COPY + qbase, then (kk < 2 ? 0 : 3 SEQ) + b SEQ
        # + (2 - nt) 32 + 32 kk; qcol[kk * 32 + kg * 16 + e] and qcol[96] of
        # 128; per-wave w96w[8 (i / 4) + 4 kg + i mod 4] of 32.
        mrow, kg = lane & 31, lane >> 5
        qbase = np.where((mrow & 15) == 0, 112, 96) - 16 * ((mrow >> 4) & 1) + 16 * kg - 64
        qb = ((16 - (mrow & 15)) & 15) * COPY + qbase
        offs = [qb + (0 if kk < 2 else 3 * SEQ) + b * SEQ + (2 - nt) * 32 + kk * 32
                for nt in range(3) for kk in range(3) for b in range(3)]
        assert 2 * 32 + 16 + 15 < 128
        i = np.arange(16)
        assert (8 * (i // 4)[None, :] + 4 * kg[:, None] + (i % 4)[None, :]).max() < 32
    for off in offs:
        assert off.min() >= 0 and (off + 16).max() <= TQ_BYTES
    # Factor sequences: H[jq * 196 + thread] for thread < 193, jq < B - 1.
    assert (B - 2) * KH + 192 < (B - 1) * KH
    rs, cs = zip(*(factor_stores(n, A, tpw, jq, tr) for jq in range(B - 1)))
    _tally(count, np.concatenate(rs), np.concatenate(cs))


SIZES = [33, 64, 600, 4097, 32768, 40001, 65536, 70001, 131071]


@pytest.mark.parametrize("tr", [16, 32])
@pytest.mark.parametrize("n", SIZES)
def test_family_product_indices(n, tr):
    if launch_shape(n, tr, 768) is None:  # too small: the radix rounds serve
        assert 2 * max(tr, math.ceil(math.sqrt(n) / tr) * tr) > n
        return
    A, B, _ = launch_shape(n, tr, 768)
    assert A % tr == 0 and A * B >= n and (B - 1) * A < n and B - 1 <= 65535
    # The launcher's pick for any device size is one of 1..8; check them all.
    assert {launch_shape(n, tr, s)[2] for s in (1, 256, 768, 1 << 20)} <= set(range(1, 9))
    firsts = {}
    for in_place, seeded in ((False, False), (True, False), (False, True)):
        c1 = np.zeros((n, KW), np.int64)
        sim_l1(n, A, B, in_place, seeded, c1)
        firsts[(in_place, seeded)] = c1
    for tpw in range(1, 9):
        c2 = np.zeros((n, KW), np.int64)
        sim_product(n, A, B, tpw, tr, c2)
        assert not c2[:A].any() and np.all(c2[A:] == 1), (n, tr, tpw)
        for (in_place, seeded), c1 in firsts.items():
            want = np.ones((n, KW), np.int64)
            if in_place:
                want[0] = 0
            assert np.array_equal(c1 + c2, want), (n, tr, tpw, in_place, seeded)


def test_family_indices_at_the_largest_no_alloc_size():
    """The no-allocation entry point's limit, n = 2^24: A = B = 4096, so the
    factors fit its fixed array of 4096 sequences; the largest factor buffer
    index and the largest source record stay inside their buffers."""
    n = 1 << 24
    for tr in (16, 32):
        A, B, tpw = launch_shape(n, tr, 768)
        assert (A, B) == (4096, 4096) and B - 1 <= 4096
        assert (B - 1) * KH <= 4096 * KH
        assert (A - 1) * KW + 127 < n * KW


def test_family_indices_large_boundary_factors():
    """2^20 starts (the bulk family): the first and the last factor's tiles,
    for every tiles-per-wave value, write their rows exactly once."""
    n = 1 << 20
    for tr in (16, 32):
        A, B, _ = launch_shape(n, tr, 768)
        for tpw in range(1, 9):
            for jq in (0, B - 2):
                j = jq + 1
                lo, hi = j * A, min(n, (j + 1) * A)
                R_, C_ = factor_stores(n, A, tpw, jq, tr)
                count = np.zeros((hi - lo, KW), np.int64)
                _tally(count, R_ - lo, C_)
                assert np.all(count == 1), (tr, tpw, j)
