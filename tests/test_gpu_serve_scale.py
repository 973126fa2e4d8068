"""Serving at the scale of the 200,000-request workload (Sec. 1: a stream is
rebuilt exactly from its seed and offset, so a served result must not depend
on what else the server runs).

All 200,000 requests of the workload (seed uniform on [1, 9e8], offset uniform
on [0, 2^120), count log-uniform on [1e2, 1e7], float32 output) go through one
server with the 64 GiB budget at once.  1,000 of them, among them the 20
largest, are submitted by the test while a replay thread submits the other
199,000 and releases each as it completes, so the sampled ones are served in
the mix.  Each sampled result is then
  - compared with the oracle (the oracle's own jump to three windows of 512
    draws: the first, one in the middle and the last; whole results below
    1,537 draws), and
  - served again alone by a fresh server: bit for bit the same.
"""
import threading

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import dev, f32_words, say, u32

pytestmark = pytest.mark.gpu

N_REQ = synth.SERVE["requests"]
N_SAMPLE = 1000
WIN = 512


def _server(arena, lanes=4):
    import paper_2512_00093_amd as R
    c = R.ranmar_serve_cfg()
    c.queue_when_full = 1
    c.lanes = lanes
    return R.ranmar_serve_create(arena, c)


def _slice(arena, ptr, cnt):
    off = (ptr - arena.data_ptr()) // 4
    return arena[off:off + cnt]


def test_serve_200k_mix_sampled_against_oracle_and_alone(orc):
    import paper_2512_00093_amd as R
    R.ranmar_init()
    tr = synth.serve_requests(N_REQ, qps=1.0, offset=5)
    counts = tr["counts"].astype(np.int64)
    g = synth.rng(60)
    largest = np.argsort(counts)[-20:]
    rest = np.setdiff1d(np.arange(N_REQ), largest)
    sample = np.sort(np.concatenate([largest, g.choice(rest, size=N_SAMPLE - 20, replace=False)]))
    others = np.setdiff1d(np.arange(N_REQ), sample)
    offsets = [(int(h) << 64) | int(l) for l, h in zip(tr["off_lo"], tr["off_hi"])]

    arena = torch.empty(synth.SERVE["budget_bytes"] // 4, dtype=torch.int32, device=dev())
    srv = _server(arena)
    kept = {}
    try:
        say(f"serve mix: {len(others)} replayed + {len(sample)} sampled, {float(counts.sum()):.3g} draws")
        err = []

        def replay():
            try:
                R.ranmar_serve_replay(srv, np.zeros(len(others)), tr["seeds"][others], tr["off_lo"][others],
                                      tr["off_hi"][others], tr["counts"][others], R.RANMAR_F32)
            except Exception as e:  # reported by the main thread
                err.append(e)

        th = threading.Thread(target=replay)
        th.start()
        tickets = []
        for i in sample:
            st, t = R.ranmar_serve_submit(srv, int(tr["seeds"][i]), offsets[i], int(counts[i]), R.RANMAR_F32)
            assert st == 0, (i, st)
            tickets.append(t)
        for i, t in zip(sample, tickets):
            assert R.ranmar_serve_wait(srv, t, 120_000_000_000) == 0, i
            ptr, cnt = R.ranmar_serve_result(srv, t)
            assert cnt == counts[i]
            kept[int(i)] = _slice(arena, ptr, cnt).clone()
            # The copy runs on torch's stream: it must have read the result
            # before the release lets the server reuse those bytes.
            torch.cuda.current_stream().synchronize()
            R.ranmar_serve_release(srv, t)
        th.join(timeout=300)
        assert not th.is_alive() and not err, err
        s = R.ranmar_serve_stats_get(srv)
        assert s.completed == N_REQ and s.released == N_REQ and s.bytes_in_use == 0
        say(f"served {s.completed} requests in {s.ticks} launches, peak arena {s.bytes_peak / 2**30:.1f} GiB")
    finally:
        R.ranmar_serve_destroy(srv)
    del arena
    torch.cuda.synchronize()

    # Against the oracle: three windows per request (whole result when short).
    say("oracle windows")
    for i in sample:
        i = int(i)
        c = int(counts[i])
        got = u32(kept[i])
        starts = [0] if c <= 3 * WIN else [0, int(g.integers(WIN, c - 2 * WIN)), c - WIN]
        width = c if c <= 3 * WIN else WIN
        st0 = orc.seed_jump_many([int(tr["seeds"][i])] * len(starts), [offsets[i] + p for p in starts])
        ref, _ = orc.draws_many(st0, width)
        for k, p in enumerate(starts):
            assert np.array_equal(got[p:p + width], f32_words(ref[k])), (i, c, p)

    # The same requests alone, through a fresh server: the same bits.
    say("alone")
    arena2 = torch.empty((64 << 20) // 4 * 4, dtype=torch.int32, device=dev())
    srv2 = _server(arena2, lanes=1)
    try:
        for i in sample:
            i = int(i)
            st, t = R.ranmar_serve_submit(srv2, int(tr["seeds"][i]), offsets[i], int(counts[i]), R.RANMAR_F32)
            assert st == 0
            assert R.ranmar_serve_wait(srv2, t, 30_000_000_000) == 0
            ptr, cnt = R.ranmar_serve_result(srv2, t)
            assert torch.equal(_slice(arena2, ptr, cnt), kept[i]), i
            R.ranmar_serve_release(srv2, t)
    finally:
        R.ranmar_serve_destroy(srv2)
