"""GPU parity: every entry point of the HIP library against the CPU oracle,
bit for bit (all arithmetic is integer; the float32 output k * 2^-24 is exact).

Small cases are compared element by element at sizes that span several
workgroups and ragged tails; the full workload sizes are compared on sampled
streams the oracle computes one by one, and on whole-array identities between
two GPU routes that must agree exactly (independent jumps vs. prefix-doubled
families)."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import dev, f32_words, jumps_t, limbs_t, say, seeds_t, states_t, u32

pytestmark = pytest.mark.gpu

R = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    global R
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_00093_amd as pkg
    pkg.ranmar_init()
    R = pkg
    yield
    torch.cuda.synchronize()


MASK = (1 << 24) - 1
TABLE2 = [(1 << 64) - 1, (1 << 120) - 1]


def _rand_states(orc, n, seed=7):
    g = synth.rng(200 + seed)
    W = g.integers(0, 1 << 24, size=(n, 97), dtype=np.uint64).astype(np.uint32)
    c = g.integers(0, orc.MOD, size=(n, 1), dtype=np.uint64).astype(np.uint32)
    return np.concatenate([W, c], 1)


# --- a1: seeding --------------------------------------------------------------
def test_seed_batch(orc):
    seeds = [1, 2, 3, 12345, 4711, 900000, 900000000, 30082, 30083, 177 * 30082 + 5] + \
        [int(s) for s in synth.seeds(300, offset=11)]
    say(f"seed_batch n={len(seeds)}")
    out = R.ranmar_seed_batch(seeds_t(seeds))
    torch.cuda.synchronize()
    got = u32(out)
    for r, s in enumerate(seeds):
        assert np.array_equal(got[r], orc.state_from_seed(s)), s


def test_seed_batch_invalid_marks_record():
    say("seed_batch invalid seeds")
    out = R.ranmar_seed_batch(seeds_t([0, -3, 900000001, 5]))
    got = u32(out)
    for r in range(3):
        assert not got[r, :97].any() and got[r, 97] == 0xFFFFFFFF
    assert got[3, 97] == 362436


# --- a3: t^J mod phi ------------------------------------------------------------
@pytest.fixture(params=[0, 1], ids=["lane_square_multiply", "window_products"])
def poly_variant(request):
    R.ranmar_tune_set(R.RANMAR_K_POLY, request.param)
    yield request.param
    R.ranmar_tune_set(R.RANMAR_K_POLY, -1)


def test_jump_poly(orc, poly_variant):
    g = synth.rng(210)
    lo, hi = synth.u128_uniform(g, 120, 120)
    Js = [0, 1, 2, 5, 63, 64, 65, 96, 97, 98, 129, 130, 193, 255, 256, 257, 1 << 20, 10 ** 6, (1 << 128) - 1,
          ((1 << 8) - 1) << 120, (1 << 127) + 1] + TABLE2 + \
        synth.u128_to_int(lo, hi) + [int(v) for v in g.integers(0, 1 << 40, size=20)]
    say(f"jump_poly n={len(Js)} variant={poly_variant}")
    P = u32(R.ranmar_jump_poly(jumps_t(Js)))
    ref = orc.xpow_many(Js)
    bad = [Js[r] for r in range(len(Js)) if not np.array_equal(P[r], ref[r])]
    assert not bad, bad[:5]


def test_jump_poly_waves_of_mixed_length(orc, poly_variant):
    """Lanes of one wave with very different exponent lengths (the lane
    variant's loop runs over the wave's longest; short exponents carry leading
    zeros), and a count that leaves the last workgroup's waves partly idle."""
    Js = [(1 << (k % 128)) + k for k in range(203)]
    say(f"jump_poly mixed lengths n=203 variant={poly_variant}")
    P = u32(R.ranmar_jump_poly(jumps_t(Js)))
    ref = orc.xpow_many(Js)
    assert np.array_equal(P, ref)


def test_jump_poly_variants_agree_at_scale():
    """The two t^J mod phi variants on 20,000 uniform 120-bit exponents
    (with the 20-bit table built, the window products take it)."""
    s, lo, hi = synth.batch_jumps(20000, 120, offset=33)
    J = limbs_t(lo, hi)
    R.ranmar_seed_jump(seeds_t(s), J)   # 20,000 requests: builds the 20-bit window table
    try:
        R.ranmar_tune_set(R.RANMAR_K_POLY, 0)
        a = R.ranmar_jump_poly(J)
        R.ranmar_tune_set(R.RANMAR_K_POLY, 1)
        b = R.ranmar_jump_poly(J)
    finally:
        R.ranmar_tune_set(R.RANMAR_K_POLY, -1)
    assert torch.equal(a, b)


# --- a4: apply ----------------------------------------------------------------
def test_apply_poly(orc):
    n = 150
    st = _rand_states(orc, n, 1)
    g = synth.rng(211)
    P = g.integers(0, 1 << 24, size=(n, 97), dtype=np.uint64).astype(np.uint32)
    P[:, :3] |= np.uint32(0xFF000000)   # high bits must be ignored
    say(f"apply_poly n={n}")
    d = states_t(st)
    R.ranmar_apply_poly(d, torch.from_numpy(P.view(np.int32).copy()).to(dev()))
    got = u32(d)
    for r in range(n):
        assert np.array_equal(got[r, :97], orc.apply(st[r, :97], P[r] & MASK)), r
        assert got[r, 97] == st[r, 97]


# --- a2-a4: jump ---------------------------------------------------------------
def test_jump_in_place(orc):
    n = 130
    st = _rand_states(orc, n, 2)
    g = synth.rng(212)
    lo, hi = synth.u128_uniform(g, n, 120)
    Js = synth.u128_to_int(lo, hi)
    Js[:6] = [0, 1, 97, (1 << 128) - 1, orc.MOD, ((1 << 97) - 1) << 23]
    say(f"jump in place n={n}")
    d = states_t(st)
    R.ranmar_jump(d, jumps_t(Js))
    got = u32(d)
    for r in range(n):
        assert np.array_equal(got[r], orc.jump(st[r], Js[r])), (r, Js[r])


def test_jump_small_equals_stepping(orc):
    st0 = orc.state_from_seed(12345)
    Js = [0, 1, 2, 31, 32, 33, 64, 96, 97, 98, 1000, 4097, 65536]
    say("jump vs stepping")
    d = states_t(np.tile(st0, (len(Js), 1)))
    R.ranmar_jump(d, jumps_t(Js))
    got = u32(d)
    for r, J in enumerate(Js):
        assert np.array_equal(got[r], orc.step(st0, J)), J


def test_seed_jump(orc):
    s, lo, hi = synth.batch_jumps(200, 120, offset=13)
    s = s.copy()
    s[:3] = [1, 900000000, 12345]
    Js = synth.u128_to_int(lo, hi)
    say("seed_jump n=200")
    got = u32(R.ranmar_seed_jump(seeds_t(s), limbs_t(lo, hi)))
    ref = orc.seed_jump_many(s, Js)
    assert np.array_equal(got, ref)
    # NULL offsets: offset 0 == seeding
    got0 = u32(R.ranmar_seed_jump(seeds_t(s[:70])))
    assert np.array_equal(got0, np.stack([orc.state_from_seed(int(x)) for x in s[:70]]))


def test_seed_jump_invalid_seed_leaves_marker():
    say("seed_jump invalid seed")
    got = u32(R.ranmar_seed_jump(seeds_t([0, 7]), jumps_t([5, 5])))
    assert not got[0, :97].any() and got[0, 97] == 0xFFFFFFFF
    assert got[1, 97] != 0xFFFFFFFF


# --- a5: generation ------------------------------------------------------------
@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_generate_ragged(orc, fmt, n):
    st = np.stack([orc.state_from_seed(1000 + 7 * k) for k in range(n)])
    for count in (1, 5, 31, 32, 33, 63, 64, 65, 96, 97, 98, 100, 193, 1000, 4097):
        say(f"generate n={n} count={count} fmt={fmt}")
        ld = count + 3
        d_in = states_t(st)
        d_st = torch.full_like(d_in, -1)
        dt = torch.float32 if fmt else torch.int32
        out = torch.full((n, ld), -7, dtype=dt, device=dev())
        R.ranmar_generate(d_in, count, fmt, out=out, states_out=d_st, ld=ld)
        ref, ref_st = orc.draws_many(st, count)
        got = u32(out)
        want = f32_words(ref) if fmt else ref
        assert np.array_equal(got[:, :count], want), (n, count, fmt)
        pad = u32(torch.full((1, 1), -7, dtype=dt))[0, 0]
        assert (got[:, count:] == pad).all()
        assert np.array_equal(u32(d_st), ref_st), (n, count)


def test_generate_in_place_continues_stream(orc):
    n = 9
    st = np.stack([orc.state_from_seed(77 + k) for k in range(n)])
    d = states_t(st)
    outs = []
    for count in (40, 1, 31, 100):
        say(f"generate in-place count={count}")
        outs.append(u32(R.ranmar_generate(d, count, 0, states_out=d)))
    total = sum(o.shape[1] for o in outs)
    ref, ref_st = orc.draws_many(st, total)
    assert np.array_equal(np.concatenate(outs, 1), ref)
    assert np.array_equal(u32(d), ref_st)


def test_generate_count_zero_copies():
    st = np.arange(98 * 3, dtype=np.uint32).reshape(3, 98) % 1000
    d_in = states_t(st)
    d_out = torch.zeros_like(d_in)
    say("generate count=0")
    R.ranmar_generate(d_in, 0, 0, states_out=d_out)
    assert np.array_equal(u32(d_out), st)


@pytest.mark.parametrize("n,count,ld", [(1, 1, 1), (3, 33, 40), (17, 1000, 1000), (64, 4097, 4100)])
def test_generate_both_formats(orc, n, count, ld):
    """RANMAR_U24_F32: every draw as uint32 k in plane 0 and as the float
    k * 2^-24 in plane 1, in one pass, with every generation variant; the
    state after the draws as with one format."""
    st = np.stack([orc.state_from_seed(40 + k) for k in range(n)])
    ref, ref_st = orc.draws_many(st, count)
    nv = R.ranmar_tune_variants(R.RANMAR_K_GENERATE)
    try:
        for v in range(nv):
            R.ranmar_tune_set(R.RANMAR_K_GENERATE, v)
            say(f"generate both n={n} count={count} ld={ld} variant={v}")
            out = torch.full((2, n, ld), -5, dtype=torch.int32, device=dev())
            so = torch.zeros((n, 98), dtype=torch.int32, device=dev())
            R.ranmar_generate(states_t(st), count, R.RANMAR_U24_F32, out=out, states_out=so, ld=ld)
            w = u32(out)
            assert np.array_equal(w[0, :, :count], ref), v
            assert np.array_equal(w[1, :, :count], f32_words(ref)), v
            assert (w[:, :, count:] == np.uint32(0xFFFFFFFB)).all(), v   # padding untouched
            assert np.array_equal(u32(so), ref_st), v
    finally:
        R.ranmar_tune_set(R.RANMAR_K_GENERATE, -1)


@pytest.mark.parametrize("variant", [0, 1, 2], ids=["radix_valu", "product_mfma", "product_mfma32"])
@pytest.mark.parametrize("n,delta", [(8192, 1 << 40), (9999, (1 << 40) + 12345), (70_001, 1 << 40),
                                     (5000, (1 << 115) + 12345), (300, 1 << 40), (33, (1 << 40) + 5),
                                     (31, 12345), (32_768, 1 << 40), (131_071, 3)])
def test_family_variants(orc, variant, n, delta):
    """Every family variant against independent jumps: radix rounds on the
    VALU, and the matrix product (about sqrt(n) direct starts and as many
    shared factors, the rest as int8 MFMA products of signed digits, in
    16- or 32-row tiles).  The product forms cover ragged last blocks
    (70,001; 131,071; 33, whose last factor holds one start), 15-digit
    factors (2^115 spacing) and the default switch-over size (32,768); below
    two blocks of tile height (n = 31, and n = 33 for 32-row tiles) they
    fall back to the radix rounds."""
    base = orc.state_from_seed(4711)
    R.ranmar_tune_set(R.RANMAR_K_FAMILY, variant)
    try:
        say(f"jump_family variant={variant} n={n} delta={delta}")
        fam = R.ranmar_jump_family(states_t(base), delta, n)
    finally:
        R.ranmar_tune_set(R.RANMAR_K_FAMILY, -1)
    ind = R.ranmar_seed_jump(seeds_t([4711] * n), jumps_t([k * delta for k in range(n)]))
    assert torch.equal(fam, ind)
    for k in sorted({0, 1, n // 3, n - 1}):
        assert np.array_equal(u32(fam[k]), orc.jump(base, k * delta)), k


@pytest.mark.parametrize("variant,n", [(0, 600), (1, 600), (1, 40_000), (2, 600), (2, 40_000)])
def test_family_in_place(orc, variant, n):
    """d_base == d_out: the family is built around its own first record."""
    delta = (1 << 40) + 7
    base = orc.state_from_seed(31)
    fam = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    fam[0] = states_t(base)[0]
    say(f"jump_family in place variant={variant} n={n}")
    R.ranmar_tune_set(R.RANMAR_K_FAMILY, variant)
    try:
        R.ranmar_jump_family(fam[:1], delta, n, out=fam)
    finally:
        R.ranmar_tune_set(R.RANMAR_K_FAMILY, -1)
    ind = R.ranmar_seed_jump(seeds_t([31] * n), jumps_t([k * delta for k in range(n)]))
    assert torch.equal(fam, ind)


def test_generate_variants_bit_identical(orc):
    n, count = 64, 777
    st = np.stack([orc.state_from_seed(5 + k) for k in range(n)])
    ref, _ = orc.draws_many(st, count)
    nv = R.ranmar_tune_variants(R.RANMAR_K_GENERATE)
    try:
        for v in range(nv):
            say(f"generate variant {v} {R.ranmar_tune_variant_name(0, v)}")
            R.ranmar_tune_set(R.RANMAR_K_GENERATE, v)
            for fmt in (0, 1):
                got = u32(R.ranmar_generate(states_t(st), count, fmt))
                assert np.array_equal(got, f32_words(ref) if fmt else ref), (v, fmt)
    finally:
        R.ranmar_tune_set(R.RANMAR_K_GENERATE, -1)


@pytest.mark.parametrize("n,count,ld", [(1, 33, 36), (131, 2048, 2048), (131, 1000, 1003), (257, 64, 68),
                                        (2053, 160, 160)])
def test_generate_variants_ragged_grids_and_pitches(orc, n, count, ld):
    """Every generation variant on stream counts that leave workgroups (of 8
    or 16 half-waves, in groups of 8 workgroups) partly empty, with row
    pitches that allow 16-byte stores (ld a multiple of 4) or not (the wide
    forms then fall back to 4-byte stores): draws, untouched padding and the
    states written back, bit for bit."""
    st = np.stack([orc.state_from_seed(900 + 7 * k) for k in range(n)])
    ref, ref_st = orc.draws_many(st, count)
    nv = R.ranmar_tune_variants(R.RANMAR_K_GENERATE)
    try:
        for v in range(nv):
            R.ranmar_tune_set(R.RANMAR_K_GENERATE, v)
            say(f"generate ragged n={n} count={count} ld={ld} variant={v}")
            out = torch.full((n, ld), -5, dtype=torch.float32, device=dev())
            so = torch.zeros((n, 98), dtype=torch.int32, device=dev())
            R.ranmar_generate(states_t(st), count, R.RANMAR_F32, out=out, states_out=so, ld=ld)
            w = u32(out)
            assert np.array_equal(w[:, :count], f32_words(ref)), v
            assert (w[:, count:] == u32(torch.full((1,), -5, dtype=torch.float32))[0]).all(), v
            assert np.array_equal(u32(so), ref_st), v
    finally:
        R.ranmar_tune_set(R.RANMAR_K_GENERATE, -1)


# --- stream families -----------------------------------------------------------
@pytest.mark.parametrize("n,delta", [(1, (1 << 40) + 12345), (2, (1 << 40) + 12345), (3, (1 << 40) + 12345),
                                     (64, (1 << 40) + 12345), (100, (1 << 40) + 12345),
                                     (5000, (1 << 40) + 12345), (70_000, 1 << 40), (200, (1 << 120) + 3)])
def test_family_equals_independent_jumps(orc, n, delta):
    """Families are built in radix-256 rounds (1, 2 and 3 rounds here; the
    last case has 16-digit exponents up to 199 (2^120 + 3) < 2^128)."""
    base = orc.state_from_seed(4711)
    say(f"jump_family n={n} delta={delta}")
    fam = R.ranmar_jump_family(states_t(base), delta, n)
    ind = R.ranmar_seed_jump(seeds_t([4711] * n), jumps_t([k * delta for k in range(n)]))
    assert torch.equal(fam, ind)
    for k in sorted({0, n - 1, n // 2, min(n - 1, 63)}):
        assert np.array_equal(u32(fam[k]), orc.jump(base, k * delta)), k


# --- per-rank streams -------------------------------------------------------------
@pytest.mark.parametrize("seed,J,first,n,discard", [
    (4711, 1 << 40, 0, 1, 0), (4711, 1 << 40, 0, 7, 1), (12345, (1 << 100) + 77, 3, 130, 0),
    (900000000, 999_999, 1000, 5000, 1), (1, 1 << 60, 0, 40_000, 0), (77, (1 << 50) + 3, 5, 33_000, 1)])
def test_rank_streams(orc, seed, J, first, n, discard):
    """Rank first+k starts at offset (first+k) J (+1 with the warm-up discard);
    the last two cases take the matrix-core family path with the seeding
    inside its first launch."""
    say(f"rank_streams seed={seed} J={J} first={first} n={n} discard={discard}")
    got = R.ranmar_rank_streams(seed, J, first, n, discard_first=bool(discard), device=dev())
    torch.cuda.synchronize()
    base = orc.state_from_seed(seed)
    for k in sorted({0, 1 % n, n // 2, n - 1}):
        assert np.array_equal(u32(got[k]), orc.jump(base, (first + k) * J + discard)), k
    if n <= 200:
        ind = R.ranmar_seed_jump(seeds_t([seed] * n), jumps_t([(first + k) * J + discard for k in range(n)]))
        assert torch.equal(got, ind)


def test_shards_concatenate_to_single_run(orc):
    """Multi-GPU sharding evidence on one GPU: the 2^20-stream bulk family
    (seed 900000, starts k 2^100, 1,024 float32 draws) run once, and run as 8
    shards of 131,072 streams (each started with first_rank = g * 131,072, as
    GPU g of 8 would), give identical arrays; rows are also checked against the
    oracle."""
    cfg = synth.BULK_1M
    n, shards, L = cfg["streams"], 8, cfg["draws"]
    per = n // shards
    say(f"shards: {n} streams as {shards} x {per}, {L} draws")
    st = R.ranmar_rank_streams(cfg["seed"], cfg["spacing"], 0, n, device=dev())
    whole = R.ranmar_generate(st, L, R.RANMAR_F32)
    del st
    parts = []
    for g in range(shards):
        stg = R.ranmar_rank_streams(cfg["seed"], cfg["spacing"], g * per, per, device=dev())
        parts.append(R.ranmar_generate(stg, L, R.RANMAR_F32))
        del stg
    cat = torch.cat(parts, 0)
    torch.cuda.synchronize()
    assert torch.equal(whole.view(torch.int32), cat.view(torch.int32))
    del parts, cat
    base = orc.state_from_seed(cfg["seed"])
    for k in (0, per - 1, per, 5 * per + 17, n - 1):
        ref, _ = orc.state_draws(orc.jump(base, k * cfg["spacing"]), L)
        assert np.array_equal(u32(whole[k]), f32_words(ref)), k


def test_rank_streams_discard_is_one_draw(orc):
    """With the discard, rank 0's first draw is the undiscarded stream's second."""
    say("rank_streams discard = one draw")
    a = R.ranmar_rank_streams(4711, 1 << 30, 0, 2, discard_first=False, device=dev())
    b = R.ranmar_rank_streams(4711, 1 << 30, 0, 2, discard_first=True, device=dev())
    da = u32(R.ranmar_generate(a, 8, 0))
    db = u32(R.ranmar_generate(b, 7, 0))
    assert np.array_equal(da[0, 1:], db[0]) and np.array_equal(da[1, 1:], db[1])


def test_rank_streams_rejects_bad_arguments():
    """Bad seeds, an offset beyond 2^128 and a discard flag other than 0/1
    are refused on the host (RANMAR_EINVAL, nothing launched)."""
    say("rank_streams invalid arguments")
    out = torch.empty((4, 98), dtype=torch.int32, device=dev())
    st = torch.cuda.current_stream().cuda_stream
    for seed, J, first, discard in ((0, 1, 0, 0), (900000001, 1, 0, 0), (5, 1 << 127, 2, 0), (5, 1, 0, 2)):
        rc = R.lib().ranmar_rank_streams(seed, R._binding._u128(J), first, 4, discard, out.data_ptr(), st)
        assert rc == -1, (seed, J, first, discard)


# --- one stream by block splitting -------------------------------------------------
@pytest.mark.parametrize("K,L", [(64, 16384), (40_000, 25), (1000, 1000)])
def test_single_stream_by_block_splitting(orc, K, L):
    """Sec. 1's block splitting: K segments of L draws, segment k started at
    offset k L and written to row k of a [K][L] array, give the single
    stream's first K L draws in order (40,000 segments take the matrix-core
    family path)."""
    seed = 12345
    say(f"single stream by splitting K={K} L={L}")
    st = R.ranmar_rank_streams(seed, L, 0, K, device=dev())
    out = R.ranmar_generate(st, L, R.RANMAR_U24)
    torch.cuda.synchronize()
    assert np.array_equal(u32(out).reshape(-1), orc.int_draws(seed, K * L))


# --- configurations at full size -------------------------------------------------
def test_config1_single_stream(orc):
    p = synth.SINGLE_STREAM
    say("config1: seed 12345, 1e6 draws, jump 2^20")
    st = states_t(orc.state_from_seed(p["seed"]))
    got = u32(R.ranmar_generate(st, p["draws"], 0))[0]
    assert np.array_equal(got, orc.int_draws(p["seed"], p["draws"]))
    d = states_t(orc.state_from_seed(p["seed"]))
    R.ranmar_jump(d, jumps_t([p["jump"]]))
    assert np.array_equal(u32(d)[0], orc.step(orc.state_from_seed(p["seed"]), p["jump"]))


def test_config2_family_65k(orc):
    p = synth.FAMILY_65K
    n, cnt = p["streams"], p["draws"]
    say(f"config2: {n} streams x {cnt}, offsets k*2^40")
    lo, hi = synth.family_offsets(n, p["spacing"])
    st = R.ranmar_seed_jump(seeds_t([p["seed"]] * n), limbs_t(lo, hi))
    fam = R.ranmar_jump_family(states_t(orc.state_from_seed(p["seed"])), p["spacing"], n)
    assert torch.equal(st, fam)
    st_copy = st.clone()
    out_u = R.ranmar_generate(st, cnt, 0)
    out_f = R.ranmar_generate(st_copy, cnt, 1, states_out=st_copy)
    torch.cuda.synchronize()
    sample = synth.family_sample(n, 64)
    base = orc.state_from_seed(p["seed"])
    for k in sample:
        s_k = orc.jump(base, int(k) * p["spacing"])
        assert np.array_equal(u32(st[k]), s_k), k
        ref, ref_st = orc.draws_many(s_k[None], cnt)
        assert np.array_equal(u32(out_u[k]), ref[0]), k
        assert np.array_equal(u32(out_f[k]), f32_words(ref[0])), k
        assert np.array_equal(u32(st_copy[k]), ref_st[0]), k
    # Properties over every stream: range of the words and exact float values.
    assert int(out_u.min()) >= 0 and int(out_u.max()) <= MASK
    assert torch.equal(out_u.to(torch.float64) * 2.0 ** -24, out_f.to(torch.float64))


def test_config3_bulk_states_and_sample(orc):
    p = synth.BULK_1M
    n, cnt = p["streams"], p["draws"]
    say(f"config3: {n} streams at k*2^100, {cnt} f32 draws")
    base = orc.state_from_seed(p["seed"])
    fam = R.ranmar_jump_family(states_t(base), p["spacing"], n)
    lo, hi = synth.family_offsets(n, p["spacing"])
    ind = R.ranmar_seed_jump(seeds_t(np.full(n, p["seed"], np.int32)), limbs_t(lo, hi))
    assert torch.equal(fam, ind)
    del ind
    out = R.ranmar_generate(fam, cnt, 1)
    torch.cuda.synchronize()
    for k in synth.family_sample(n, 32, offset=3):
        s_k = orc.jump(base, int(k) * p["spacing"])
        assert np.array_equal(u32(fam[k]), s_k), k
        ref, _ = orc.draws_many(s_k[None], cnt)
        assert np.array_equal(u32(out[k]), f32_words(ref[0])), k
    # every value is a multiple of 2^-24 in [0, 1)
    assert float(out.min()) >= 0.0 and float(out.max()) < 1.0
    assert torch.equal(torch.floor(out.double() * 2 ** 24), out.double() * 2 ** 24)


def test_config4_batched_jumps_sample(orc):
    n = synth.BATCH_JUMPS["requests"]
    s, lo, hi = synth.batch_jumps(n, 120, offset=4)
    say(f"config4: {n} seed+jump requests, 120-bit J")
    out = R.ranmar_seed_jump(seeds_t(s), limbs_t(lo, hi))
    torch.cuda.synchronize()
    g = synth.rng(214)
    idx = np.unique(np.concatenate([[0, n - 1], g.choice(n, 200, replace=False)]))
    Js = synth.u128_to_int(lo[idx], hi[idx])
    ref = orc.seed_jump_many(s[idx], Js)
    assert np.array_equal(u32(out[torch.from_numpy(idx).to(dev())]), ref)
    w = u32(out)
    assert w[:, :97].max() <= MASK and w[:, 97].max() < orc.MOD


def test_repeatable(orc):
    s, lo, hi = synth.batch_jumps(1000, 120, offset=15)
    say("repeatability")
    a = R.ranmar_seed_jump(seeds_t(s), limbs_t(lo, hi))
    b = R.ranmar_seed_jump(seeds_t(s), limbs_t(lo, hi))
    assert torch.equal(a, b)
    assert torch.equal(R.ranmar_generate(a, 333, 1), R.ranmar_generate(b, 333, 1))


# --- jump variants: per-lane square-and-multiply; 32, 16 or 8 lanes with 8-, 16-, 20- or 24-bit windows ---
@pytest.fixture(params=[0, 1, 2, 3, 4, 5, 6], ids=["lane_sqmul", "half_window", "lanes16_window", "lanes8_window",
                                                   "lanes8_window16", "lanes8_window20", "lanes8_window24"])
def jump_variant(request):
    R.ranmar_tune_set(R.RANMAR_K_JUMP, request.param)
    yield request.param
    R.ranmar_tune_set(R.RANMAR_K_JUMP, -1)


def test_jump_variant_seeding(orc, jump_variant):
    """J = 0: pure seeding (the half-wave variant seeds the 97 words in
    parallel from closed-form jumps of the two small generators)."""
    seeds = [1, 2, 3, 12345, 4711, 900000, 900000000, 30082, 30083] + \
        [int(s) for s in synth.seeds(400, offset=17)]
    say(f"seed via seed_jump variant={jump_variant}")
    got = u32(R.ranmar_seed_jump(seeds_t(seeds), jumps_t([0] * len(seeds))))
    assert np.array_equal(got, np.stack([orc.state_from_seed(s) for s in seeds]))


def _edge_jumps():
    g = synth.rng(220)
    lo, hi = synth.u128_uniform(g, 60, 120)
    return [0, 1, 2, 255, 256, 257, 65535, 1 << 64, (1 << 64) - 1, (1 << 120) - 1, (1 << 128) - 1,
            ((1 << 97) - 1) << 23, (1 << 20) - 1, 1 << 20, ((1 << 20) - 1) << 20, 1 << 60, (1 << 120) + 255,
            ((1 << 8) - 1) << 120, (1 << 24) - 1, 1 << 24, ((1 << 24) - 1) << 24, ((1 << 24) - 1) << 96,
            (1 << 72) + (1 << 71), ((1 << 48) - 1) << 40] + synth.u128_to_int(lo, hi)


def test_jump_variant_edges(orc, jump_variant):
    Js = _edge_jumps()
    seeds = [int(s) for s in synth.seeds(len(Js), offset=18)]
    seeds[:3] = [0, 900000001, -7]       # invalid seeds leave the marker record
    say(f"seed_jump edges variant={jump_variant}")
    got = u32(R.ranmar_seed_jump(seeds_t(seeds), jumps_t(Js)))
    for r in range(3):
        assert not got[r, :97].any() and got[r, 97] == 0xFFFFFFFF
    ref = orc.seed_jump_many(seeds[3:], Js[3:])
    assert np.array_equal(got[3:], ref)
    # in-place jump of arbitrary states
    st = _rand_states(orc, len(Js), 9)
    d = states_t(st)
    R.ranmar_jump(d, jumps_t(Js))
    w = u32(d)
    for r in range(0, len(Js), 5):
        assert np.array_equal(w[r], orc.jump(st[r], Js[r])), (r, Js[r])


def test_jump_variants_agree_at_scale(jump_variant):
    n = 20000
    s, lo, hi = synth.batch_jumps(n, 120, offset=19)
    say(f"jump variants at n={n}")
    a = R.ranmar_seed_jump(seeds_t(s), limbs_t(lo, hi))
    for other in range(R.ranmar_tune_variants(R.RANMAR_K_JUMP)):
        if other == jump_variant:
            continue
        R.ranmar_tune_set(R.RANMAR_K_JUMP, other)
        b = R.ranmar_seed_jump(seeds_t(s), limbs_t(lo, hi))
        assert torch.equal(a, b), other


_HALF_WINDOW_FRESH = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_2512_00093_amd as R
from tests.gpu_util import jumps_t, seeds_t, u32
from tests.test_gpu_parity import _edge_jumps
torch.cuda.set_device(0)
R.ranmar_init()
R.ranmar_tune_set(R.RANMAR_K_JUMP, 1)
Js = _edge_jumps()
seeds = [4711 + 1000 * k for k in range(len(Js))]
np.save(sys.argv[2], u32(R.ranmar_seed_jump(seeds_t(seeds), jumps_t(Js))))
"""


def test_half_window_jump_with_either_table(orc, tmp_path):
    """The half-wave jump multiplies the 20-bit table's factors once that
    table exists and the 8-bit table's before. A fresh process, in which
    nothing has built the 20-bit table (few requests never do), checks the
    8-bit route; this process checks the 20-bit route after a forced 20-bit
    jump has built the table."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    Js = _edge_jumps()
    seeds = [4711 + 1000 * k for k in range(len(Js))]
    ref = orc.seed_jump_many(seeds, Js)
    out = tmp_path / "fresh.npy"
    say("half-window jump in a fresh process (8-bit table)")
    subprocess.run([sys.executable, "-c", _HALF_WINDOW_FRESH, root, str(out)], cwd=root, check=True,
                   timeout=300)
    assert np.array_equal(np.load(out), ref)
    try:
        R.ranmar_tune_set(R.RANMAR_K_JUMP, 5)
        R.ranmar_seed_jump(seeds_t(seeds[:8]), jumps_t(Js[:8]))       # builds the 20-bit table
        R.ranmar_tune_set(R.RANMAR_K_JUMP, 1)
        say("half-window jump with the 20-bit table")
        got = u32(R.ranmar_seed_jump(seeds_t(seeds), jumps_t(Js)))
    finally:
        R.ranmar_tune_set(R.RANMAR_K_JUMP, -1)
    assert np.array_equal(got, ref)


def test_tune_run_jump_and_generate():
    best, ms = R.ranmar_tune_run(R.RANMAR_K_JUMP, 4096, 120)
    assert 0 <= best < R.ranmar_tune_variants(R.RANMAR_K_JUMP) and all(m > 0 for m in ms)
    try:
        best, ms = R.ranmar_tune_run(R.RANMAR_K_POLY, 4096, 120)
        assert 0 <= best < 2 and len(ms) == 2 and all(m > 0 for m in ms)
    finally:
        R.ranmar_tune_clear(R.RANMAR_K_POLY)
    best, ms = R.ranmar_tune_run(R.RANMAR_K_GENERATE, 4096, 4096)
    assert 0 <= best < R.ranmar_tune_variants(R.RANMAR_K_GENERATE) and all(m > 0 for m in ms)
    best, ms = R.ranmar_tune_run(R.RANMAR_K_FAMILY, 20000, 40)
    assert 0 <= best < R.ranmar_tune_variants(R.RANMAR_K_FAMILY) and all(m > 0 for m in ms)


def test_seed_batch_both_paths(orc):
    """< 4096 seeds: 32 lanes per seed; >= 4096: one lane per seed."""
    seeds = [int(s) for s in synth.seeds(5000, offset=23)]
    say("seed_batch n=5000 (lane path) and n=100 (half-wave path)")
    big = u32(R.ranmar_seed_batch(seeds_t(seeds)))
    small = u32(R.ranmar_seed_batch(seeds_t(seeds[:100])))
    assert np.array_equal(big[:100], small)
    for r in (0, 1, 99, 2500, 4999):
        assert np.array_equal(big[r], orc.state_from_seed(seeds[r])), r


def test_family_polynomial_path(orc):
    """Exponents 2^b delta above 128 bits take the squaring-chain path."""
    delta = (1 << 121) + 1
    n = 129
    base = orc.state_from_seed(777)
    say("jump_family wide exponents n=129")
    fam = u32(R.ranmar_jump_family(states_t(base), delta, n))
    for k in (0, 1, 2, 64, 100, 127):      # k * delta < 2^128 for the oracle
        assert np.array_equal(fam[k], orc.jump(base, k * delta)), k
    # stream 128 (exponent above 2^128) by the group law: 128 delta = 127 delta + delta
    assert np.array_equal(fam[128], orc.jump(orc.jump(base, 127 * delta), delta))
