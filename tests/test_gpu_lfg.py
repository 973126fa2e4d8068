"""GPU parity of the general lagged-Fibonacci path (any r, s, e, m, d; Sec. 2,
Sec. 3.1, 3.2, Sec. 5) against the general oracle, through the C ABI.

Integer work: every comparison is bit-exact.  Inputs are seeded synthetic
states (uniform words below 2^e, c below m) and jump lengths with edge values
around the lags plus uniform 120-bit lengths."""
import numpy as np
import pytest
import torch

import paper_2512_00093_amd as R
import synth
from gpu_util import dev, jumps_t, say, u32

pytestmark = pytest.mark.gpu

CASES = list(synth.LFG_CASES)
BIG = {"r607s273e24", "r1279s418e32", "r4423s2098e24", "r1000s3e16", "r1279s418e24", "r5120s2000e24"}


def _jumps(r, s, n_rand, offset, bits=120):
    edge = sorted({0, 1, s - 1, s, s + 1, r - 1, r, r + 1, r + s, 2 * r - 1, 2 * r, 12345,
                   (1 << 64) - 1, (1 << 64), (1 << bits) - 1})
    g = synth.rng(offset)
    rand = [int(x) for x in synth.u128_to_int(*synth.u128_uniform(g, n_rand, bits))]
    return [J for J in edge if J >= 0] + rand


def _states_t(arr):
    return torch.from_numpy(np.ascontiguousarray(arr, np.uint32).view(np.int32).copy()).to(dev())


def _params(name):
    return R.lfg_params(*synth.LFG_CASES[name])


@pytest.mark.parametrize("name", CASES)
def test_lfg_jump_poly(orc, name):
    g = orc.LFG(*synth.LFG_CASES[name])
    Js = _jumps(g.r, g.s, 2 if name in BIG else 12, offset=21)
    if g.r >= 4000:  # keep the oracle's cost to seconds
        Js = [0, 1, g.r, g.r + g.s, (1 << 64) - 1, (1 << 100) + 3]
    say(f"lfg_jump_poly {name} n={len(Js)}")
    got = u32(R.ranmar_lfg_jump_poly(_params(name), jumps_t(Js)))
    assert np.array_equal(got, g.xpow_many(Js)), name


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("in_place", [False, True])
def test_lfg_jump(orc, name, in_place):
    g = orc.LFG(*synth.LFG_CASES[name])
    Js = _jumps(g.r, g.s, 2 if name in BIG else 10, offset=22)
    if g.r >= 4000:
        Js = [0, g.r + 1, (1 << 90) + 17]
    st = synth.lfg_states(g.r, g.e, g.m, len(Js), offset=23)
    say(f"lfg_jump {name} n={len(Js)} in_place={in_place}")
    d_in = _states_t(st)
    if in_place:
        R.ranmar_lfg_jump(_params(name), d_in, jumps_t(Js))
        got = u32(d_in)
    else:
        d_out = torch.full_like(d_in, -1)
        R.ranmar_lfg_jump(_params(name), d_in, jumps_t(Js), out=d_out)
        got = u32(d_out)
        assert np.array_equal(u32(d_in), st)
    assert np.array_equal(got, g.jump_many(st, Js)), name


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("fmt", [R.RANMAR_U24, R.RANMAR_F32])
def test_lfg_generate(orc, name, fmt):
    g = orc.LFG(*synth.LFG_CASES[name])
    if fmt == R.RANMAR_F32 and g.e > 24:
        pytest.skip("float output needs e <= 24")
    n = 37 if g.r < 2000 else 5  # ragged: not a multiple of the streams per wave
    st = synth.lfg_states(g.r, g.e, g.m, n, offset=24)
    p = _params(name)
    # Row pitches of count + 5 and of count rounded up to a multiple of 4,
    # plus 4 (every row start 16-byte aligned).
    for count, pad in [(c, pad) for c in (0, 1, 3, g.s, g.r + 1, 1000, 4097) for pad in (5, None)]:
        ld = count + pad if pad is not None else (count + 3) // 4 * 4 + 4
        say(f"lfg_generate {name} n={n} count={count} ld={ld} fmt={fmt}")
        d_in = _states_t(st)
        d_st = torch.full_like(d_in, -1)
        dt = torch.float32 if fmt else torch.int32
        out = torch.full((n, max(ld, 1)), -7, dtype=dt, device=dev())
        R.ranmar_lfg_generate(p, d_in, count, fmt, out=out, states_out=d_st, ld=ld)
        ref, ref_st = g.draws_many(st, count)
        got = u32(out)
        want = (ref.astype(np.float64) * 2.0 ** -g.e).astype(np.float32).view(np.uint32) if fmt else ref
        assert np.array_equal(got[:, :count], want), (name, count)
        pad = u32(torch.full((1, 1), -7, dtype=dt))[0, 0]
        assert (got[:, count:ld] == pad).all()
        assert np.array_equal(u32(d_st), ref_st), (name, count)


@pytest.mark.parametrize("name", ["r5s1e8", "ranmar", "r1279s418e32", "r1000s3e16"])
def test_lfg_generate_in_place_continues(orc, name):
    g = orc.LFG(*synth.LFG_CASES[name])
    st = synth.lfg_states(g.r, g.e, g.m, 11, offset=25)
    d = _states_t(st)
    p = _params(name)
    outs = []
    for count in (40, 1, 63, 700):
        say(f"lfg_generate in place {name} count={count}")
        outs.append(u32(R.ranmar_lfg_generate(p, d, count, R.RANMAR_U24, states_out=d)))
    ref, ref_st = g.draws_many(st, sum(o.shape[1] for o in outs))
    assert np.array_equal(np.concatenate(outs, 1), ref)
    assert np.array_equal(u32(d), ref_st)


def test_lfg_ranmar_matches_specialised_path(orc):
    """With RANMAR's parameters the general kernels equal the RANMAR kernels
    (jump and generate) on seeded states."""
    seeds = [1, 12345, 900000000, 4711]
    st = np.stack([orc.state_from_seed(s) for s in seeds])
    Js = [0, 97, (1 << 120) - 1, 10**30]
    p = R.lfg_params(*orc.RANMAR_PARAMS)
    say("lfg vs ranmar jump/generate")
    d_gen = _states_t(st)
    R.ranmar_lfg_jump(p, d_gen, jumps_t(Js))
    d_spec = _states_t(st)
    R.ranmar_jump(d_spec, jumps_t(Js))
    assert np.array_equal(u32(d_gen), u32(d_spec))
    a = u32(R.ranmar_lfg_generate(p, d_gen, 5000, R.RANMAR_U24))
    b = u32(R.ranmar_generate(d_spec, 5000, R.RANMAR_U24))
    assert np.array_equal(a, b)


def test_lfg_full_size_sampled(orc):
    """The benchmark's generation shape (65,536 streams of the r = 1279
    generator, 4,096 draws) and jump shape (4,096 jumps of 120 bits), checked
    on sampled rows against the oracle."""
    cfg = synth.LFG_GEN
    g = orc.LFG(*synth.LFG_CASES[cfg["case"]])
    n, count = cfg["streams"], cfg["draws"]
    st = synth.lfg_states(g.r, g.e, g.m, n, offset=26)
    p = _params(cfg["case"])
    say(f"lfg_generate full size n={n} count={count}")
    d = _states_t(st)
    out = R.ranmar_lfg_generate(p, d, count, R.RANMAR_U24, states_out=d)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, 1, 31, 32, 63, n - 1], synth.rng(27).integers(0, n, 10)]))
    ref, ref_st = g.draws_many(st[rows], count)
    assert np.array_equal(u32(out[torch.from_numpy(rows).to(dev())]), ref)
    assert np.array_equal(u32(d)[rows], ref_st)
    jc = synth.LFG_JUMPS
    Js = [int(x) for x in synth.u128_to_int(*synth.u128_uniform(synth.rng(28), jc["jumps"], jc["jump_bits"]))]
    say(f"lfg_jump full size n={len(Js)}")
    st2 = synth.lfg_states(g.r, g.e, g.m, len(Js), offset=29)
    d2 = _states_t(st2)
    R.ranmar_lfg_jump(p, d2, jumps_t(Js))
    pick = [0, 1, 2047, len(Js) - 1]
    assert np.array_equal(u32(d2)[pick], g.jump_many(st2[pick], [Js[i] for i in pick]))


def test_lfg_rejects_bad_arguments():
    with pytest.raises(R.RanmarError):
        R.lfg_params(5, 5, 8, 7, 1)
    with pytest.raises(R.RanmarError):
        R.lfg_params(R.RANMAR_LFG_MAX_R + 1, 3, 24, 5, 1)
    p = R.lfg_params(55, 24, 32, 4294967291, 2654435761)
    st = torch.zeros((2, 56), dtype=torch.int32, device=dev())
    with pytest.raises(R.RanmarError):
        R.ranmar_lfg_generate(p, st, 10, R.RANMAR_F32)  # float output needs e <= 24


@pytest.mark.parametrize("name", ["r5s1e8", "r17s3e32", "ranmar", "r607s273e24", "r1000s3e16"])
@pytest.mark.parametrize("n,delta", [(1, 5), (2, 1), (3, 97), (17, 1 << 40), (100, 12345), (1000, (1 << 100) + 7)])
def test_lfg_family(orc, name, n, delta):
    """Family starts out[k] = f^(k delta)(base) against the oracle's jumps."""
    g = orc.LFG(*synth.LFG_CASES[name])
    base = synth.lfg_states(g.r, g.e, g.m, 1, offset=33)
    say(f"lfg_jump_family {name} n={n} delta={delta}")
    got = u32(R.ranmar_lfg_jump_family(_params(name), _states_t(base), delta, n))
    rows = sorted({0, 1, n // 2, n - 1} | set(int(x) for x in synth.rng(34).integers(0, n, 6))) if n > 8 else range(n)
    rows = [k for k in rows if k < n]
    want = g.jump_many(np.repeat(base, len(rows), 0), [k * delta for k in rows])
    assert np.array_equal(got[rows], want), (name, n, delta)


def test_lfg_family_equals_jumps_whole_array():
    """Every start of a 4,100-stream family at r = 1279 equals the per-stream
    jump to k delta (two independent GPU routes, whole array)."""
    name = "r1279s418e24"
    r, s, e, m, d = synth.LFG_CASES[name]
    base = synth.lfg_states(r, e, m, 1, offset=35)
    n, delta = 4100, (1 << 90) + 3
    say(f"lfg family vs jumps n={n}")
    p = _params(name)
    fam = u32(R.ranmar_lfg_jump_family(p, _states_t(base), delta, n))
    d = _states_t(np.repeat(base, n, 0))
    R.ranmar_lfg_jump(p, d, jumps_t([k * delta for k in range(n)]))
    assert np.array_equal(fam, u32(d))


def test_lfg_family_in_place_and_full_size(orc):
    """base == out[0] (in place), at the benchmark's family shape: 65,536
    starts of the r = 1279 generator spaced 2^40 apart, sampled rows against
    the oracle."""
    name = synth.LFG_GEN["case"]
    g = orc.LFG(*synth.LFG_CASES[name])
    n, delta = 65_536, 1 << 40
    base = synth.lfg_states(g.r, g.e, g.m, 1, offset=36)
    say(f"lfg family in place n={n}")
    out = torch.zeros((n, g.r + 1), dtype=torch.int32, device=dev())
    out[0] = _states_t(base)[0]
    R.ranmar_lfg_jump_family(_params(name), out[0:1], delta, n, out=out)
    torch.cuda.synchronize()
    rows = [0, 1, 255, 256, 257, 65_535] + [int(x) for x in synth.rng(37).integers(0, n, 6)]
    want = g.jump_many(np.repeat(base, len(rows), 0), [k * delta for k in rows])
    assert np.array_equal(u32(out)[rows], want)


def test_lfg_family_rejects_overflow():
    p = R.lfg_params(*synth.LFG_CASES["ranmar"])
    base = torch.zeros((1, 98), dtype=torch.int32, device=dev())
    with pytest.raises(R.RanmarError):
        R.ranmar_lfg_jump_family(p, base, 1 << 127, 3)


def test_lfg_family_large_equals_ranmar_family(orc):
    """At RANMAR's parameters, a 2^20-start general family (1,023 shared
    polynomials) equals, whole array, the RANMAR family of the same base
    (int8 matrix-core products: an independent route), and sampled rows
    equal the oracle."""
    n, delta = 1 << 20, (1 << 40) + 9
    base = orc.state_from_seed(4711)
    say(f"lfg family vs ranmar family n={n}")
    p = R.lfg_params(*orc.RANMAR_PARAMS)
    d_base = _states_t(base[None, :])
    gen = R.ranmar_lfg_jump_family(p, d_base, delta, n)
    spec = torch.empty_like(gen)
    R.ranmar_jump_family(d_base, delta, n, out=spec)
    torch.cuda.synchronize()
    assert torch.equal(gen, spec)
    rows = [0, 1, 1023, 1024, 1025, n - 1] + [int(x) for x in synth.rng(40).integers(0, n, 4)]
    for k in rows:
        assert np.array_equal(u32(gen[k]), orc.jump(base, k * delta)), k


def test_lfg_full_size_equals_ranmar_kernels(orc):
    """At RANMAR's parameters and full size, whole arrays: 16,384 general
    jumps (uniform 120-bit J) equal the windowed RANMAR jump, and 65,536
    streams x 4,096 general draws equal the RANMAR generator."""
    p = R.lfg_params(*orc.RANMAR_PARAMS)
    n = 16384
    seeds = synth.seeds(n, offset=41)
    lo, hi = synth.u128_uniform(synth.rng(42), n, 120)
    jt = jumps_t(synth.u128_to_int(lo, hi))
    say(f"lfg vs ranmar jump n={n}")
    st = R.ranmar_seed_batch(torch.from_numpy(seeds.copy()).to(dev()))
    gen = st.clone()
    R.ranmar_lfg_jump(p, gen, jt)
    R.ranmar_jump(st, jt)
    torch.cuda.synchronize()
    assert torch.equal(gen, st)
    fam = synth.FAMILY_65K
    say(f"lfg vs ranmar generate {fam['streams']} x {fam['draws']}")
    starts = R.ranmar_rank_streams(fam["seed"], fam["spacing"], 0, fam["streams"], device=dev())
    a = R.ranmar_lfg_generate(p, starts, fam["draws"], R.RANMAR_U24)
    b = R.ranmar_generate(starts, fam["draws"], R.RANMAR_U24)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
