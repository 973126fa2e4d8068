"""Batched execution (one persistent, graph-launched kernel for uneven
requests) and serving (continuous batching under an HBM budget), bit for bit
against the oracle and against the same requests run alone."""
import time

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import dev, f32_words, say, states_t, u32

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


def _mixed_requests(k, seed_off, max_count=120_000, with_zero=True):
    g = synth.rng(300 + seed_off)
    seeds = g.integers(1, 900_000_001, size=k)
    lo, hi = synth.u128_uniform(g, k, 120)
    counts = np.floor(10 ** g.uniform(0, np.log10(max_count), size=k)).astype(np.int64)
    counts[:6] = [1, 31, 16384, 16385, 32768 + 5, 100_000][:min(6, k)]
    if with_zero and k > 7:
        counts[7] = 0
    fmts = g.integers(0, 2, size=k)
    return [dict(seed=int(seeds[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=int(counts[i]),
                 fmt=int(fmts[i])) for i in range(k)]


def _alloc(items):
    for it in items:
        dt = torch.float32 if it["fmt"] else torch.int32
        it["out"] = torch.full((max(it["count"], 1),), -3, dtype=dt, device=dev())
        it["state"] = torch.zeros(98, dtype=torch.int32, device=dev())
    return items


def _check(orc, items, sample=None):
    idx = range(len(items)) if sample is None else sample
    for r in idx:
        it = items[r]
        st0 = orc.seed_jump_many([it["seed"]], [it["offset"]])[0]
        ref, ref_st = orc.draws_many(st0[None], it["count"])
        got = u32(it["out"])[:it["count"]]
        want = f32_words(ref[0]) if it["fmt"] else ref[0]
        assert np.array_equal(got, want), (r, it["count"], it["fmt"])
        assert np.array_equal(u32(it["state"]), ref_st[0]), (r, it["count"])


def test_batch_outputs_at_every_alignment(orc):
    """Outputs that start 0, 4, 8 or 12 bytes past a 16-byte boundary: the
    aligned chunks are written 16 bytes per lane, the others 4 bytes per lane
    (both kinds can share a wave); every draw and final state is the oracle's."""
    items = _mixed_requests(24, 7, max_count=60_000)
    for k, it in enumerate(items):
        dt = torch.float32 if it["fmt"] else torch.int32
        shift = k % 4
        it["buf"] = torch.full((max(it["count"], 1) + 4,), -3, dtype=dt, device=dev())
        it["out"] = it["buf"][shift:shift + max(it["count"], 1)]
        it["state"] = torch.zeros(98, dtype=torch.int32, device=dev())
    b = R.ranmar_batch_create(64, 4096, 8192)
    try:
        say(f"batch outputs at every alignment n={len(items)}")
        R.ranmar_batch_run(b, R.make_requests(items))
        torch.cuda.synchronize()
        _check(orc, items)
        for k, it in enumerate(items):   # nothing written outside the output
            shift, n = k % 4, max(it["count"], 1)
            outside = torch.cat([it["buf"][:shift], it["buf"][shift + n:]])
            assert bool((u32(outside) == u32(torch.full_like(outside, -3))).all()), k
    finally:
        R.ranmar_batch_destroy(b)


def test_batch_matches_oracle(orc):
    items = _alloc(_mixed_requests(40, 1))
    b = R.ranmar_batch_create(64, 4096)
    try:
        say(f"batch_run n={len(items)} draws={sum(i['count'] for i in items)}")
        R.ranmar_batch_run(b, R.make_requests(items))
        torch.cuda.synchronize()
        _check(orc, items)
    finally:
        R.ranmar_batch_destroy(b)


def test_batch_graph_replays_with_eager_work_between(orc):
    """The captured graph is replayed several times, with the program's own
    eager launches and synchronisations in between; every replay is checked."""
    b = R.ranmar_batch_create(200, 2048, 4096)
    try:
        for rep in range(4):
            items = _alloc(_mixed_requests(30 + 40 * (rep % 2), 10 + rep, max_count=40_000))
            say(f"graph replay {rep}: n={len(items)}")
            R.ranmar_batch_run(b, R.make_requests(items))
            # eager work between replays
            st = states_t(np.stack([orc.state_from_seed(99 + rep)]))
            eager = R.ranmar_generate(st, 1000, 0)
            torch.cuda.synchronize()
            assert np.array_equal(u32(eager)[0], orc.int_draws(99 + rep, 1000))
            _check(orc, items)
    finally:
        R.ranmar_batch_destroy(b)


def test_batch_many_jumps_one_launch(orc):
    """Jump-only requests (count 0, state out): the batched-jump workload."""
    n = 5000
    s, lo, hi = synth.batch_jumps(n, 120, offset=21)
    out = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                  state=out[i]) for i in range(n)]
    b = R.ranmar_batch_create(n, 1)
    try:
        say(f"batch jumps n={n}")
        R.ranmar_batch_run(b, R.make_requests(items))
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)
    direct = R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev()))
    assert torch.equal(out, direct)
    idx = [0, 1, 77, n - 1]
    ref = orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx]))
    assert np.array_equal(u32(out)[idx], ref)


def test_unbatched_matches_batched(orc):
    items_a = _alloc(_mixed_requests(20, 2))
    items_b = _alloc([{k: v for k, v in it.items() if k in ("seed", "offset", "count", "fmt")} for it in items_a])
    b = R.ranmar_batch_create(32, 1024)
    try:
        say("batched vs one launch per request")
        R.ranmar_batch_run(b, R.make_requests(items_a))
        R.ranmar_run_unbatched(R.make_requests(items_b))
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)
    for x, y in zip(items_a, items_b):
        assert torch.equal(x["out"], y["out"]) and torch.equal(x["state"], y["state"])
    _check(orc, items_b, sample=[0, 3, 5, 7])


def test_batch_capacity_and_argument_errors():
    b = R.ranmar_batch_create(4, 8, 1024)
    try:
        out = torch.zeros(10_000, dtype=torch.int32, device=dev())
        ok = dict(seed=5, offset=0, count=100, fmt=0, out=out, state=None)
        with pytest.raises(R.RanmarError) as e:
            R.ranmar_batch_run(b, R.make_requests([ok] * 5))           # more requests than capacity
        assert e.value.status == R.RANMAR_ENOMEM
        with pytest.raises(R.RanmarError) as e:
            R.ranmar_batch_run(b, R.make_requests([dict(ok, count=9 * 1024)]))   # more chunks than capacity
        assert e.value.status == R.RANMAR_ENOMEM
        for bad in (dict(ok, seed=0), dict(ok, fmt=3), dict(ok, out=None)):
            with pytest.raises(R.RanmarError) as e:
                R.ranmar_batch_run(b, R.make_requests([bad]))
            assert e.value.status == R.RANMAR_EINVAL
        R.ranmar_batch_run(b, R.make_requests([ok]))
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)


# --- serving -----------------------------------------------------------------
def _server(arena_bytes, **cfg):
    arena = torch.empty(arena_bytes // 4, dtype=torch.int32, device=dev())
    c = R.ranmar_serve_cfg()
    for k, v in cfg.items():
        setattr(c, k, v)
    return R.ranmar_serve_create(arena, c), arena


def _result(server, arena, ticket, fmt):
    ptr, cnt = R.ranmar_serve_result(server, ticket)
    off = (ptr - arena.data_ptr()) // 4
    words = u32(arena[off:off + cnt])
    return words


def test_serve_results_match_oracle_and_alone(orc):
    reqs = _mixed_requests(60, 3, max_count=300_000)
    srv, arena = _server(256 << 20, max_tick_chunks=16, chunk_draws=4096, lanes=3, queue_when_full=1)
    outs = {}
    try:
        say(f"serve mix n={len(reqs)}")
        tickets = []
        for it in reqs:
            st, t = R.ranmar_serve_submit(srv, it["seed"], it["offset"], it["count"], it["fmt"])
            assert st == 0
            tickets.append(t)
        for r, t in enumerate(tickets):
            assert R.ranmar_serve_wait(srv, t, 30_000_000_000) == 0
            outs[r] = _result(srv, arena, t, reqs[r]["fmt"])
            R.ranmar_serve_release(srv, t)
        s = R.ranmar_serve_stats_get(srv)
        assert s.completed == len(reqs) and s.released == len(reqs) and s.bytes_in_use == 0
        assert s.ticks > 1 and s.p99_ns >= s.p50_ns > 0
    finally:
        R.ranmar_serve_destroy(srv)
    # each result equals the oracle ...
    for r in range(0, len(reqs), 3):
        it = reqs[r]
        st0 = orc.seed_jump_many([it["seed"]], [it["offset"]])[0]
        ref, _ = orc.draws_many(st0[None], it["count"])
        assert np.array_equal(outs[r], f32_words(ref[0]) if it["fmt"] else ref[0]), r
    # ... and the same request served alone gives the same bits.
    srv2, arena2 = _server(64 << 20, lanes=1)
    try:
        for r in (0, 4, 5, 11, 30):
            it = reqs[r]
            st, t = R.ranmar_serve_submit(srv2, it["seed"], it["offset"], it["count"], it["fmt"])
            assert st == 0
            assert R.ranmar_serve_wait(srv2, t) == 0
            assert np.array_equal(_result(srv2, arena2, t, it["fmt"]), outs[r]), r
            R.ranmar_serve_release(srv2, t)
    finally:
        R.ranmar_serve_destroy(srv2)


def test_serve_budget_admission():
    srv, arena = _server(1 << 20, queue_when_full=0, lanes=1)
    try:
        st, _ = R.ranmar_serve_submit(srv, 7, 0, (1 << 20) // 4 + 1, 1)
        assert st == R.RANMAR_ENOMEM                       # never fits the budget
        st, t1 = R.ranmar_serve_submit(srv, 7, 0, 200_000, 1)
        assert st == 0
        R.ranmar_serve_wait(srv, t1)
        st, _ = R.ranmar_serve_submit(srv, 8, 0, 100_000, 1)
        assert st == R.RANMAR_EAGAIN                       # budget held by t1 until released
        R.ranmar_serve_release(srv, t1)
        st, t2 = R.ranmar_serve_submit(srv, 8, 0, 100_000, 1)
        assert st == 0
        R.ranmar_serve_wait(srv, t2)
        R.ranmar_serve_release(srv, t2)
        assert R.ranmar_serve_stats_get(srv).rejected == 2
    finally:
        R.ranmar_serve_destroy(srv)
    # With queueing, over-budget requests wait for releases and then run.
    srv, arena = _server(1 << 20, queue_when_full=1, lanes=2)
    try:
        sub = [R.ranmar_serve_submit(srv, 9 + i, i, 150_000, 0) for i in range(4)]
        assert all(st == 0 for st, _ in sub)
        ts = [t for _, t in sub]
        R.ranmar_serve_wait(srv, ts[0])
        assert not R.ranmar_serve_poll(srv, ts[3])     # 4 x 600 KB cannot all fit 1 MiB
        for t in ts:
            R.ranmar_serve_wait(srv, t)
            R.ranmar_serve_release(srv, t)
        s = R.ranmar_serve_stats_get(srv)
        assert s.bytes_peak <= 1 << 20 and s.completed == 4
    finally:
        R.ranmar_serve_destroy(srv)


def test_serve_unbatched_same_bits(orc):
    reqs = _mixed_requests(12, 4, max_count=80_000, with_zero=False)
    res = []
    for unb in (0, 1):
        srv, arena = _server(64 << 20, unbatched=unb, lanes=2)
        outs = []
        try:
            sub = [R.ranmar_serve_submit(srv, it["seed"], it["offset"], it["count"], it["fmt"]) for it in reqs]
            assert all(st == 0 for st, _ in sub)
            ts = [t for _, t in sub]
            for it, t in zip(reqs, ts):
                R.ranmar_serve_wait(srv, t)
                outs.append(_result(srv, arena, t, it["fmt"]))
                R.ranmar_serve_release(srv, t)
        finally:
            R.ranmar_serve_destroy(srv)
        res.append(outs)
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_serve_replay_driver():
    n = 400
    tr = synth.serve_requests(n, qps=20_000, offset=31, count_log10=(2.0, 5.0))
    srv, arena = _server(512 << 20, lanes=2)
    try:
        say(f"replay n={n}")
        t0 = time.time()
        lat = R.ranmar_serve_replay(srv, tr["arrival"], tr["seeds"], tr["off_lo"], tr["off_hi"], tr["counts"])
        wall = time.time() - t0
        s = R.ranmar_serve_stats_get(srv)
    finally:
        R.ranmar_serve_destroy(srv)
    assert s.completed == n and s.released == n and s.bytes_in_use == 0
    assert (lat > 0).all() and wall < 30
    assert s.draws == int(tr["counts"].sum())


def test_batch_prepare_then_launch(orc):
    items = _alloc(_mixed_requests(10, 6, max_count=50_000))
    b = R.ranmar_batch_create(16, 256)
    try:
        with pytest.raises(R.RanmarError) as e:
            R.ranmar_batch_launch(b)                     # nothing prepared
        assert e.value.status == R.RANMAR_EINVAL
        R.ranmar_batch_prepare(b, R.make_requests(items))
        say("batch prepare + launch")
        R.ranmar_batch_launch(b)
        with pytest.raises(R.RanmarError):
            R.ranmar_batch_launch(b)                     # a preparation is launched once
        torch.cuda.synchronize()
        _check(orc, items)
    finally:
        R.ranmar_batch_destroy(b)


def test_batch_splits_requests_across_bins(orc):
    """One long request among short and jump-only ones: the work is spread
    over many bins, so the long request is cut into parts with their own
    jumps; every draw and the final state must still be those of the single
    stream.  Run twice on one batch (the second run with fewer requests, so
    fewer bins and a smaller grid)."""
    b = R.ranmar_batch_create(64, 1024)
    try:
        for rep, k in enumerate((24, 5)):
            items = _mixed_requests(k, 40 + rep, max_count=50_000)
            items[1]["count"] = 3_000_017          # 184 chunks of 16384: split over many bins
            if k > 3:
                items[3]["count"] = 0
            _alloc(items)
            say(f"bins rep {rep}: n={k} draws={sum(i['count'] for i in items)}")
            R.ranmar_batch_run(b, R.make_requests(items))
            torch.cuda.synchronize()
            _check(orc, items)
    finally:
        R.ranmar_batch_destroy(b)


def test_batch_jump_octets_and_pairs(orc):
    """From 16384 requests without draws the batch jumps them eight per wave
    with 20-bit windows (octet items), after the slices with draws.  Same bits
    as ranmar_seed_jump and the oracle; the requests with draws in the same
    batch match too."""
    n = 20000
    s, lo, hi = synth.batch_jumps(n, 120, offset=23)
    states = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                  state=states[i]) for i in range(n)]
    drawn = _alloc(_mixed_requests(6, 60, max_count=70_000, with_zero=False))
    mixed = items[:10000] + drawn + items[10000:]
    b = R.ranmar_batch_create(len(mixed), 64)
    try:
        say(f"batch octets n={len(mixed)}")
        R.ranmar_batch_run(b, R.make_requests(mixed))
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)
    w = u32(states)
    direct = u32(R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                    torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev())))
    assert np.array_equal(w, direct)
    idx = [0, 1, 4999, 10000, n - 1]
    ref = orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx]))
    assert np.array_equal(w[idx], ref)
    _check(orc, drawn)


def test_batch_large_prepare_in_parts(orc):
    """From 65,536 requests the host validates and places them on several
    threads; requests with draws scattered among 100,000 jumps keep their
    order and bits."""
    n = 100_000
    s, lo, hi = synth.batch_jumps(n, 120, offset=29)
    states = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                  state=states[i]) for i in range(n)]
    drawn = _alloc(_mixed_requests(4, 61, max_count=50_000, with_zero=False))
    mixed = [drawn[0]] + items[:30_000] + [drawn[1]] + items[30_000:70_001] + [drawn[2]] + items[70_001:] + [drawn[3]]
    b = R.ranmar_batch_create(len(mixed), 64)
    try:
        for rep in range(2):
            states.zero_()
            say(f"batch prepare in parts n={len(mixed)} rep={rep}")
            R.ranmar_batch_run(b, R.make_requests(mixed))
            torch.cuda.synchronize()
            w = u32(states)
            direct = u32(R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                            torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev())))
            assert np.array_equal(w, direct)
    finally:
        R.ranmar_batch_destroy(b)
    idx = [0, 29_999, 30_000, 70_000, 70_001, n - 1]
    assert np.array_equal(w[idx], orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx])))
    _check(orc, drawn)


def test_batch_jumps_only_then_mixed_on_one_object(orc):
    """A batch whose first request has no draws has its jump records staged
    while it is validated; they are kept when every request is a jump and
    staged again when one is not.  One batch object runs a batch of jumps
    only, a batch that starts with jumps and holds draws, and jumps only
    again: every jump equals ranmar_seed_jump, the draws the oracle."""
    n = 70_000
    s, lo, hi = synth.batch_jumps(n, 120, offset=31)
    direct = u32(R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                    torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev())))
    b = R.ranmar_batch_create(n + 3, 64)
    try:
        for rep, with_draws in enumerate((False, True, False)):
            states = torch.zeros((n, 98), dtype=torch.int32, device=dev())
            items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                          state=states[i]) for i in range(n)]
            drawn = _alloc(_mixed_requests(3, 62 + rep, max_count=40_000, with_zero=False)) if with_draws else []
            mixed = items[:20_000] + drawn[:1] + items[20_000:50_000] + drawn[1:] + items[50_000:]
            say(f"batch jumps first rep={rep} draws={with_draws} n={len(mixed)}")
            R.ranmar_batch_run(b, R.make_requests(mixed))
            torch.cuda.synchronize()
            assert np.array_equal(u32(states), direct), rep
            _check(orc, drawn)
    finally:
        R.ranmar_batch_destroy(b)
    idx = [0, 19_999, 20_000, n - 1]
    assert np.array_equal(direct[idx], orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx])))


# --- tuner over the batch executor --------------------------------------------
@pytest.mark.parametrize("variant", range(9))
def test_batch_every_mapping_bit_identical(orc, variant):
    """Every mapping the batch tuner can pick (bins, jump items per dequeue,
    8- or 32-lane jumps for requests without draws, the direct mapping, which
    falls back to the default on a batch with draws) on one batch that mixes
    20,000 jump-only requests (octet items from 16,384 on), requests with
    draws and one long request split over bins: the same bits as
    ranmar_seed_jump and the oracle."""
    n = 20000
    s, lo, hi = synth.batch_jumps(n, 120, offset=24)
    states = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                  state=states[i]) for i in range(n)]
    drawn = _mixed_requests(12, 70 + variant, max_count=70_000, with_zero=False)
    drawn[2]["count"] = 1_500_007
    _alloc(drawn)
    mixed = items[:7000] + drawn + items[7000:]
    R.ranmar_tune_set(R.RANMAR_K_BATCH, variant)
    b = R.ranmar_batch_create(len(mixed), 256)
    try:
        say(f"batch mapping {R.ranmar_tune_variant_name(R.RANMAR_K_BATCH, variant)} n={len(mixed)}")
        R.ranmar_batch_run(b, R.make_requests(mixed))
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)
        R.ranmar_tune_set(R.RANMAR_K_BATCH, -1)
    direct = R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev()))
    assert torch.equal(states, direct)
    idx = [0, 6999, 7000, n - 1]
    assert np.array_equal(u32(states)[idx], orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx])))
    _check(orc, drawn)


@pytest.mark.parametrize("n,window", [(16384, 20), (20003, 20), (65541, 20), (20003, 24)])
def test_batch_direct_mapping_jumps_only(orc, n, window):
    """The direct mapping (one octet of requests per worker, no queue) on
    batches of jumps only, the last octet ragged, some requests without a
    state record, with the 20-bit table or (the jump kernel's pick forced to
    it) the 24-bit one: the same bits as ranmar_seed_jump and the oracle; the
    records left out stay untouched."""
    s, lo, hi = synth.batch_jumps(n, 120, offset=31)
    states = torch.full((n, 98), -7, dtype=torch.int32, device=dev())
    skip = set(range(5, n, 997))
    items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                  state=None if i in skip else states[i]) for i in range(n)]
    R.ranmar_tune_set(R.RANMAR_K_BATCH, 8)
    R.ranmar_tune_set(R.RANMAR_K_JUMP, 6 if window == 24 else 5)
    b = R.ranmar_batch_create(n, 1)
    try:
        say(f"direct mapping n={n} window={window}")
        R.ranmar_batch_run(b, R.make_requests(items))
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)
        R.ranmar_tune_set(R.RANMAR_K_BATCH, -1)
        R.ranmar_tune_set(R.RANMAR_K_JUMP, -1)
    direct = R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev()))
    keep = np.array([i not in skip for i in range(n)])
    kt = torch.from_numpy(keep).to(dev())
    assert torch.equal(states[kt], direct[kt])
    assert bool((states[~kt] == -7).all())
    idx = [0, 7, 8, n - 2, n - 1]
    assert np.array_equal(u32(states)[idx], orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx])))


@pytest.mark.parametrize("variant", [0, 4, 5])
def test_batch_mappings_with_the_24_bit_table(orc, variant):
    """With the jump kernel's pick forced to the 24-bit table, a batch's
    octets (and, once the table is set, its jump pairs) take it: a batch that
    mixes 20,000 jump-only requests with requests with draws gives the same
    bits as ranmar_seed_jump and the oracle under queue mappings with octets
    and with pairs only."""
    n = 20000
    s, lo, hi = synth.batch_jumps(n, 120, offset=25)
    states = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    items = [dict(seed=int(s[i]), offset=(int(hi[i]) << 64) | int(lo[i]), count=0, fmt=0, out=None,
                  state=states[i]) for i in range(n)]
    drawn = _alloc(_mixed_requests(12, 90 + variant, max_count=70_000, with_zero=False))
    mixed = items[:9000] + drawn + items[9000:]
    R.ranmar_tune_set(R.RANMAR_K_BATCH, variant)
    R.ranmar_tune_set(R.RANMAR_K_JUMP, 6)
    b = R.ranmar_batch_create(len(mixed), 256)
    try:
        say(f"24-bit table, batch mapping {R.ranmar_tune_variant_name(R.RANMAR_K_BATCH, variant)}")
        R.ranmar_batch_run(b, R.make_requests(mixed))
        torch.cuda.synchronize()
        R.ranmar_batch_run(b, R.make_requests(mixed))   # the same batch again: the same bits
        torch.cuda.synchronize()
    finally:
        R.ranmar_batch_destroy(b)
        R.ranmar_tune_set(R.RANMAR_K_BATCH, -1)
        R.ranmar_tune_set(R.RANMAR_K_JUMP, -1)
    direct = R.ranmar_seed_jump(torch.from_numpy(s.copy()).to(dev()),
                                torch.from_numpy(np.stack([lo, hi], 1).view(np.int64).copy()).to(dev()))
    assert torch.equal(states, direct)
    idx = [0, 8999, 9000, n - 1]
    assert np.array_equal(u32(states)[idx], orc.seed_jump_many(s[idx], synth.u128_to_int(lo[idx], hi[idx])))
    _check(orc, drawn)


@pytest.mark.parametrize("variant", range(4))
def test_batch_every_chunk_length_bit_identical(orc, variant):
    """Every chunk length the chunk tuner can pick (4,096 << variant draws),
    taken by a batch created with chunk_draws = 0: requests whose counts
    straddle chunk boundaries give the oracle's draws and final states."""
    items = _alloc(_mixed_requests(24, 80 + variant, max_count=200_000))
    items[4]["count"] = 4096 * 5 + 1
    items[4]["out"] = torch.full((items[4]["count"],), -3, dtype=torch.float32 if items[4]["fmt"] else torch.int32,
                                 device=dev())
    R.ranmar_tune_set(R.RANMAR_K_CHUNK, variant)
    try:
        b = R.ranmar_batch_create(32, 4096, 0)
    finally:
        R.ranmar_tune_set(R.RANMAR_K_CHUNK, -1)
    try:
        say(f"batch chunk length {R.ranmar_tune_variant_name(R.RANMAR_K_CHUNK, variant)}")
        R.ranmar_batch_run(b, R.make_requests(items))
        torch.cuda.synchronize()
        _check(orc, items)
    finally:
        R.ranmar_batch_destroy(b)


def test_batch_and_chunk_tuners_pick_a_variant():
    """The tuner times every mapping and every chunk length on the device at
    a given shape and records a pick that later batches use."""
    try:
        nv = R.ranmar_tune_variants(R.RANMAR_K_BATCH)
        assert nv == 9
        best, ms = R.ranmar_tune_run(R.RANMAR_K_BATCH, 4096, 0)
        assert 0 <= best < nv and len(ms) == nv and np.all(np.asarray(ms) > 0)
        best_c, ms_c = R.ranmar_tune_run(R.RANMAR_K_CHUNK, 64, 100_000)
        assert 0 <= best_c < 4 and np.all(np.asarray(ms_c) > 0)
        best_b2, _ = R.ranmar_tune_run(R.RANMAR_K_BATCH, 64, 100_000)
        assert 0 <= best_b2 < nv
    finally:  # later tests get the built-in defaults again
        R.ranmar_tune_clear(R.RANMAR_K_BATCH)
        R.ranmar_tune_clear(R.RANMAR_K_CHUNK)


def test_requests_ending_at_the_top_of_the_offset_range(orc):
    """A request is cut into parts that start at offset + d as 128-bit
    offsets of their own, so offset + count - 1 must stay below 2^128: a
    request whose parts would pass it is refused (batch and server) instead
    of restarting near offset 0; one that ends exactly at 2^128 - 1 runs and
    gives the oracle's draws."""
    top = (1 << 128) - 5
    b = R.ranmar_batch_create(4, 64, 1024)
    srv, arena = _server(64 << 20, lanes=1, chunk_draws=1024)
    try:
        out = torch.zeros(4 * 1024, dtype=torch.int32, device=dev())
        bad = dict(seed=5, offset=top, count=3 * 1024, fmt=0, out=out, state=None)
        with pytest.raises(R.RanmarError) as e:
            R.ranmar_batch_run(b, R.make_requests([bad]))
        assert e.value.status == R.RANMAR_EINVAL
        st, _ = R.ranmar_serve_submit(srv, 5, top, 3 * 1024, 0)
        assert st == R.RANMAR_EINVAL
        items = _alloc([dict(seed=5, offset=top, count=5, fmt=0)])
        say("batch request ending at 2^128 - 1")
        R.ranmar_batch_run(b, R.make_requests(items))
        torch.cuda.synchronize()
        _check(orc, items)
        st, t = R.ranmar_serve_submit(srv, 5, top, 5, 0)
        assert st == 0 and R.ranmar_serve_wait(srv, t, 10_000_000_000) == 0
        assert np.array_equal(_result(srv, arena, t, 0), u32(items[0]["out"])[:5])
        R.ranmar_serve_release(srv, t)
    finally:
        R.ranmar_batch_destroy(b)
        R.ranmar_serve_destroy(srv)
