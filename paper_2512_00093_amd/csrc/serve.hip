// Serving: continuous batching of (seed, offset, count) requests.
//
// Client threads submit requests into a FIFO.  A server thread
//   - admits requests in order while their output fits the arena (the HBM
//     budget the caller handed over) and the in-flight limit allows;
//   - cuts admitted requests into slices of whole chunks and packs slices into
//     ticks of at most max_tick_chunks chunks; each tick is one launch of a
//     batch executor (one graph: descriptor copy + persistent kernel) on one
//     of `lanes` HIP streams, so a new tick starts while earlier ticks still
//     run and requests that arrive meanwhile join the next tick;
//   - watches each tick's event and marks a request complete when its last
//     slice has finished.
// A slice of a request is itself a request (offset + first draw, its draw
// count, output at the right place), so the output equals that of the request
// run alone: the jumps are exact and compose (Sec. 3).
//
// With cfg.unbatched every admitted request is launched on its own (one launch
// per request, no graph, no packing): the baseline.  A batched tick that holds
// a single request is launched the same way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ranmar.h"
#include "arena.hpp"
#include "common.hpp"
#include "internal.hpp"

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

enum ReqState { QUEUED = 0, ADMITTED = 1, DONE = 2 };

struct Req {
  int32_t seed;
  int fmt;
  ranmar_u128 off;
  uint64_t count, next = 0, pending = 0;
  uint64_t aoff = 0, bytes = 0;
  uint64_t t_arr = 0, t_done = 0;
  uint64_t tag = 0;  // replay: request index + 1; 0 for ordinary submissions
  int st = QUEUED;
};

struct Lane {
  hipStream_t st = nullptr;
  ranmar_batch* b = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  std::vector<std::pair<uint64_t, uint64_t>> slices;  // (ticket, draws)
  std::vector<ranmar_request> reqbuf;
};

constexpr uint64_t kAlign = 256;

ranmar_u128 add_u128(ranmar_u128 a, uint64_t b) {
  ranmar_u128 r;
  r.lo = a.lo + b;
  r.hi = a.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

}  // namespace

struct ranmar_server {
  int dev = 0;
  uint8_t* arena = nullptr;
  uint64_t arena_bytes = 0;
  ranmar_serve_cfg cfg{};
  uint32_t L = 16384;
  uint64_t max_tick_requests = 8192;

  ranmar::ArenaAlloc arena_alloc;
  uint64_t inflight = 0;
  uint64_t queued_bytes = 0;  // output bytes of submitted, not yet admitted requests

  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;   // submitted, not admitted
  std::deque<uint64_t> active;  // admitted, draws left to schedule
  uint64_t next_ticket = 1;
  std::vector<Lane> lanes;

  std::thread th;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv_srv, cv_done;

  std::vector<double> lat;
  bool track_done = false;       // keep completed tickets in done_q (replay)
  std::vector<uint64_t> done_q;  // tickets completed since the last drain
  uint64_t submitted = 0, completed = 0, released = 0, rejected = 0, ticks = 0, draws = 0;
  uint64_t t_first = 0, t_last = 0;
  int err = 0;

  void complete(uint64_t t, Req& R, uint64_t when) {
    R.st = DONE;
    R.t_done = when;
    lat.push_back((double)(R.t_done - R.t_arr));
    ++completed;
    draws += R.count;
    t_last = when;
    if (track_done) done_q.push_back(t);
  }

  void release_locked(std::unordered_map<uint64_t, Req>::iterator it) {
    arena_alloc.release(it->second.aoff, it->second.count ? it->second.bytes : 0);
    --inflight;
    ++released;
    reqs.erase(it);
  }

  int submit_locked(int32_t seed, ranmar_u128 offset, uint64_t count, int fmt, uint64_t t_arrival_ns, uint64_t tag,
                    uint64_t* ticket);

  // Server thread body.
  void loop() {
    hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool progress = false;
      // 1. completions
      for (Lane& ln : lanes) {
        if (!ln.busy) continue;
        const hipError_t q = hipEventQuery(ln.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) err = RANMAR_EHIP;
        ln.busy = false;
        progress = true;
        const uint64_t when = now_ns();
        for (auto& sl : ln.slices) {
          auto it = reqs.find(sl.first);
          if (it == reqs.end()) continue;
          Req& R = it->second;
          if (--R.pending == 0 && R.next == R.count) complete(sl.first, R, when);
        }
        ln.slices.clear();
        cv_done.notify_all();
      }
      // 2. admission, in arrival order
      while (!queue.empty() && inflight < cfg.max_inflight) {
        const uint64_t t = queue.front();
        Req& R = reqs[t];
        uint64_t off = 0;
        if (!arena_alloc.alloc(R.bytes, &off)) break;
        R.aoff = off;
        R.st = ADMITTED;
        ++inflight;
        queued_bytes -= R.bytes;
        queue.pop_front();
        active.push_back(t);
        progress = true;
      }
      // 3. dispatch ticks on idle lanes
      for (Lane& ln : lanes) {
        if (ln.busy || active.empty()) continue;
        ln.reqbuf.clear();
        ln.slices.clear();
        uint64_t budget = cfg.max_tick_chunks;
        while (!active.empty() && budget > 0 && ln.reqbuf.size() < max_tick_requests) {
          const uint64_t t = active.front();
          Req& R = reqs[t];
          const uint64_t remaining = R.count - R.next;
          uint64_t take = remaining;
          if (!cfg.unbatched && take > budget * L) take = budget * L;
          ranmar_request q{};
          q.seed = R.seed;
          q.fmt = (uint32_t)R.fmt;
          q.offset = add_u128(R.off, R.next);
          q.count = take;
          q.d_out = arena + R.aoff + 4 * R.next;
          q.d_state = nullptr;
          ln.reqbuf.push_back(q);
          ln.slices.emplace_back(t, take);
          ++R.pending;
          R.next += take;
          const uint64_t chunks = (take + L - 1) / L;
          budget = chunks >= budget ? 0 : budget - chunks;
          if (R.next == R.count) active.pop_front();
          if (cfg.unbatched) break;  // one request per launch
        }
        if (ln.reqbuf.empty()) continue;
        ln.busy = true;  // its event (or the failure) is picked up above
        ++ticks;
        progress = true;
        // Descriptor preparation and the launch run without the lock, so
        // submissions and releases go on meanwhile (only this thread uses the
        // lane).
        lk.unlock();
        // A tick of one request is launched with the request passed by value
        // (no descriptor copy); the draws are the same either way.
        int rc = (cfg.unbatched || ln.reqbuf.size() == 1)
                     ? ranmar_run_unbatched(ln.reqbuf.data(), ln.reqbuf.size(), ln.st)
                     : ranmar_batch_run(ln.b, ln.reqbuf.data(), ln.reqbuf.size(), ln.st);
        if (rc == RANMAR_OK && hipEventRecord(ln.ev, ln.st) != hipSuccess) rc = RANMAR_EHIP;
        lk.lock();
        if (rc != RANMAR_OK) err = rc;
      }
      if (progress) continue;
      bool any_busy = false;
      for (Lane& ln : lanes) any_busy |= ln.busy;
      if (stop && !any_busy && queue.empty() && active.empty()) break;
      if (any_busy) {
        // Poll the lanes' events without sleeping: a timed sleep would add the
        // kernel's timer slack (tens of microseconds) to every completion.
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv_srv.wait_for(lk, std::chrono::milliseconds(2));
      }
    }
  }
};

int ranmar_server::submit_locked(int32_t seed, ranmar_u128 offset, uint64_t count, int fmt, uint64_t t_arrival_ns,
                                 uint64_t tag, uint64_t* ticket) {
  if (seed < 1 || seed > 900000000 || (fmt != RANMAR_U24 && fmt != RANMAR_F32)) return RANMAR_EINVAL;
  // A request is cut into slices that start at offset + d (d < count) as
  // 128-bit offsets of their own: the last one must not pass 2^128 - 1.
  const unsigned __int128 off = ((unsigned __int128)offset.hi << 64) | offset.lo;
  if (count > 0 && off > ~(unsigned __int128)0 - (count - 1)) return RANMAR_EINVAL;
  if (count > (UINT64_MAX - kAlign) / 4) return RANMAR_ENOMEM;
  const uint64_t nbytes = (4 * count + kAlign - 1) & ~(kAlign - 1);
  if (nbytes > arena_bytes) {
    ++rejected;
    return RANMAR_ENOMEM;
  }
  if (!cfg.queue_when_full &&
      (arena_alloc.in_use() + queued_bytes + nbytes > arena_bytes || inflight + queue.size() >= cfg.max_inflight)) {
    ++rejected;
    return RANMAR_EAGAIN;
  }
  const uint64_t t = next_ticket++;
  Req R{};
  R.seed = seed;
  R.fmt = fmt;
  R.off = offset;
  R.count = count;
  R.bytes = nbytes;
  R.tag = tag;
  R.t_arr = t_arrival_ns ? t_arrival_ns : now_ns();
  if (!t_first) t_first = now_ns();
  ++submitted;
  if (count == 0) {
    R.st = ADMITTED;
    ++inflight;
    auto& ref = reqs[t] = R;
    complete(t, ref, now_ns());
    cv_done.notify_all();
  } else {
    reqs[t] = R;
    queue.push_back(t);
    queued_bytes += nbytes;
    cv_srv.notify_one();
  }
  *ticket = t;
  return RANMAR_OK;
}

extern "C" {

int ranmar_serve_create(void* d_arena, uint64_t arena_bytes, const ranmar_serve_cfg* cfg, ranmar_server** out) {
  if (!out || !d_arena || arena_bytes < kAlign || ((uintptr_t)d_arena & (kAlign - 1))) return RANMAR_EINVAL;
  int rc = ranmar::ensure_init();
  if (rc) return rc;
  ranmar_server* s = new ranmar_server();
  hipGetDevice(&s->dev);
  s->arena = (uint8_t*)d_arena;
  s->arena_bytes = arena_bytes & ~(kAlign - 1);
  if (cfg) s->cfg = *cfg;
  if (!s->cfg.max_inflight) s->cfg.max_inflight = 65536;
  // 8192: measured lower p50/p99 than 16384 at 2e4 and 5e5 requests/s (more
  // chunks of a request run at once).  Longer chunks can serve more at
  // capacity (fewer chunk starts) but a large request alone then runs on fewer
  // lanes, so the server does not take the chunk tuner's pick by itself.
  if (!s->cfg.chunk_draws) s->cfg.chunk_draws = 8192;
  // A launch carries about 2^27 draws (16,384 chunks of 8,192) whatever the
  // chunk length, so that longer chunks make fewer chunks, not larger launches.
  if (!s->cfg.max_tick_chunks)
    s->cfg.max_tick_chunks = std::max<uint64_t>(1024, (16384ull * 8192ull) / std::max<uint64_t>(1, s->cfg.chunk_draws));
  if (!s->cfg.lanes) s->cfg.lanes = 2;
  if (s->cfg.lanes > 8 || s->cfg.chunk_draws > (1u << 24) || s->cfg.max_tick_chunks > (1u << 22)) {
    delete s;
    return RANMAR_EINVAL;
  }
  s->L = (uint32_t)s->cfg.chunk_draws;
  s->arena_alloc.reset(s->arena_bytes);
  s->lanes.resize(s->cfg.lanes);
  for (Lane& ln : s->lanes) {
    if (hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming) != hipSuccess)
      rc = RANMAR_EHIP;
    if (!rc && !s->cfg.unbatched) {
      rc = ranmar_batch_create(s->max_tick_requests, s->cfg.max_tick_chunks, s->L, &ln.b);
      // Every request jumps to a 120-bit offset: the 20-bit table (built here,
      // once per device, not on a request's path) takes 6 factors, not 15.
      if (!rc) ranmar::batch_use_wide_windows(ln.b);
    }
    if (rc) break;
  }
  if (rc) {
    for (Lane& ln : s->lanes) {
      if (ln.b) ranmar_batch_destroy(ln.b);
      if (ln.ev) hipEventDestroy(ln.ev);
      if (ln.st) hipStreamDestroy(ln.st);
    }
    delete s;
    return rc;
  }
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return RANMAR_OK;
}

int ranmar_serve_submit(ranmar_server* s, int32_t seed, ranmar_u128 offset, uint64_t count, int fmt,
                        uint64_t t_arrival_ns, uint64_t* ticket) {
  if (!s || !ticket) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  return s->submit_locked(seed, offset, count, fmt, t_arrival_ns, 0, ticket);
}

int ranmar_serve_poll(ranmar_server* s, uint64_t ticket, int* done) {
  if (!s || !done) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RANMAR_ENOENT;
  *done = it->second.st == DONE;
  return s->err ? s->err : RANMAR_OK;
}

int ranmar_serve_wait(ranmar_server* s, uint64_t ticket, int64_t timeout_ns) {
  if (!s) return RANMAR_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto pred = [&] {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second.st == DONE || s->err;
  };
  if (timeout_ns < 0)
    s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), pred))
    return RANMAR_ETIMEDOUT;
  if (s->reqs.find(ticket) == s->reqs.end()) return RANMAR_ENOENT;
  return s->err ? s->err : RANMAR_OK;
}

int ranmar_serve_result(ranmar_server* s, uint64_t ticket, const void** d_ptr, uint64_t* count) {
  if (!s || !d_ptr || !count) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RANMAR_ENOENT;
  if (it->second.st != DONE) return RANMAR_EAGAIN;
  *d_ptr = s->arena + it->second.aoff;
  *count = it->second.count;
  return RANMAR_OK;
}

int ranmar_serve_release(ranmar_server* s, uint64_t ticket) {
  if (!s) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return RANMAR_ENOENT;
  if (it->second.st != DONE) return RANMAR_EAGAIN;
  s->release_locked(it);
  s->cv_srv.notify_one();
  return RANMAR_OK;
}

int ranmar_serve_stats_get(ranmar_server* s, ranmar_serve_stats* out) {
  if (!s || !out) return RANMAR_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->released = s->released;
  out->rejected = s->rejected;
  out->ticks = s->ticks;
  out->draws = s->draws;
  out->bytes_in_use = s->arena_alloc.in_use();
  out->bytes_peak = s->arena_alloc.peak();
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
    out->p50_ns = pct(0.50);
    out->p99_ns = pct(0.99);
    out->max_ns = v.back();
  }
  out->busy_s = s->t_last > s->t_first ? (s->t_last - s->t_first) * 1e-9 : 0.0;
  return s->err ? s->err : RANMAR_OK;
}

int ranmar_serve_destroy(ranmar_server* s) {
  if (!s) return RANMAR_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_srv.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (Lane& ln : s->lanes) {
    if (ln.st) hipStreamSynchronize(ln.st);
    if (ln.b) ranmar_batch_destroy(ln.b);
    if (ln.ev) hipEventDestroy(ln.ev);
    if (ln.st) hipStreamDestroy(ln.st);
  }
  const int err = s->err;
  delete s;
  return err ? err : RANMAR_OK;
}

int ranmar_serve_replay(ranmar_server* s, uint64_t n, const double* t_arrival_s, const int32_t* seeds,
                        const ranmar_u128* offsets, const uint64_t* counts, int fmt, double* latency_ns) {
  if (!s || (n && (!t_arrival_s || !seeds || !offsets || !counts))) return RANMAR_EINVAL;
  if (n == 0) return RANMAR_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->track_done) return RANMAR_EINVAL;  // one replay at a time
    s->track_done = true;
    s->done_q.clear();
  }
  std::atomic<uint64_t> n_rejected{0};
  std::atomic<int> first_err{0};
  // Releaser: takes the tickets completed since its last pass (the server
  // queues them) and releases them, in completion order.
  std::thread rel([&] {
    std::vector<uint64_t> batch;
    uint64_t finished = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    while (finished + n_rejected.load(std::memory_order_acquire) < n) {
      if (s->done_q.empty()) {
        if (s->err) break;
        s->cv_done.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
      batch.swap(s->done_q);
      for (const uint64_t t : batch) {
        auto q = s->reqs.find(t);
        if (q == s->reqs.end() || q->second.tag == 0) continue;  // not ours: left to its submitter
        if (latency_ns) latency_ns[q->second.tag - 1] = (double)(q->second.t_done - q->second.t_arr);
        s->release_locked(q);
        ++finished;
      }
      batch.clear();
      s->cv_srv.notify_one();
    }
  });
  const uint64_t t0 = now_ns();
  auto due_of = [&](uint64_t r) { return t0 + (uint64_t)(t_arrival_s[r] * 1e9); };
  for (uint64_t r = 0; r < n;) {
    const uint64_t due = due_of(r);
    while (now_ns() < due) {
      const uint64_t left = due - now_ns();
      if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
    }
    // Every request that has arrived by now is handed over under one lock
    // (at most 256, so the server thread is not held off), each with its own
    // arrival time, from which its latency counts.
    const uint64_t now = now_ns();
    std::lock_guard<std::mutex> g(s->mu);
    const uint64_t end = std::min<uint64_t>(n, r + 256);
    do {
      uint64_t t = 0;
      const int rc = s->submit_locked(seeds[r], offsets[r], counts[r], fmt, due_of(r), r + 1, &t);
      if (rc != RANMAR_OK) {
        int z = 0;
        first_err.compare_exchange_strong(z, rc);
        n_rejected.fetch_add(1, std::memory_order_release);
      }
      ++r;
    } while (r < end && due_of(r) <= now);
  }
  rel.join();
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->track_done = false;
    s->done_q.clear();
  }
  if (s->err) return s->err;
  return first_err.load();
}

}  // extern "C"
