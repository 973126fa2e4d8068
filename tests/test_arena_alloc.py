"""Host check of the server's arena allocator (csrc/arena.hpp, plain C++):
random allocations and releases against a model that keeps only the live
blocks.  After every step the allocator's free blocks must be exactly the
gaps between live blocks (release coalesces completely), an allocation must
take the start of the smallest gap that holds it (best fit; the lowest such
offset on ties) and fail only when no gap does, and in-use and peak bytes
must match.  Compiled with g++; no GPU."""
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>
#include "arena.hpp"

static int fail(const char* what, long step) { std::printf("FAIL %s at step %ld\n", what, step); return 1; }

int main(int argc, char** argv) {
  const uint64_t A = std::strtoull(argv[1], nullptr, 10);
  const long steps = std::atol(argv[2]);
  std::mt19937_64 g(std::strtoull(argv[3], nullptr, 10));
  ranmar::ArenaAlloc a(A);
  std::map<uint64_t, uint64_t> live;  // offset -> size
  uint64_t used = 0, peak = 0;
  auto gaps = [&] {
    std::map<uint64_t, uint64_t> gp;
    uint64_t at = 0;
    for (auto& b : live) { if (b.first > at) gp[at] = b.first - at; at = b.first + b.second; }
    if (at < A) gp[at] = A - at;
    return gp;
  };
  for (long s = 0; s < steps; ++s) {
    const bool do_alloc = live.empty() || (g() % 100) < 55;
    if (do_alloc) {
      const uint64_t want = 1 + g() % (g() % 8 == 0 ? A / 4 : A / 200);
      const auto gp = gaps();
      uint64_t best_off = 0, best_size = 0; bool any = false;
      for (auto& x : gp)
        if (x.second >= want && (!any || x.second < best_size)) { best_off = x.first; best_size = x.second; any = true; }
      uint64_t off = 0;
      const bool ok = a.alloc(want, &off);
      if (ok != any) return fail("alloc success", s);
      if (ok) {
        if (off != best_off) return fail("best fit", s);
        live[off] = want;
        used += want;
        if (used > peak) peak = used;
      }
    } else {
      auto it = live.begin();
      std::advance(it, g() % live.size());
      a.release(it->first, it->second);
      used -= it->second;
      live.erase(it);
    }
    if (a.free_by_offset() != gaps()) return fail("free blocks", s);
    if (a.in_use() != used || a.peak() != peak) return fail("counters", s);
  }
  while (!live.empty()) { a.release(live.begin()->first, live.begin()->second); live.erase(live.begin()); }
  if (a.free_blocks() != 1 || a.free_by_offset().begin()->second != A || a.in_use() != 0) return fail("final", steps);
  std::printf("OK\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("arena")
    src = d / "arena_check.cpp"
    src.write_text(DRIVER)
    exe = d / "arena_check"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", str(ROOT / "paper_2512_00093_amd" / "csrc"),
                           str(src), "-o", str(exe)])
    return exe


@pytest.mark.parametrize("arena,steps,seed", [(1 << 16, 20000, 1), (1 << 30, 20000, 2), (4096, 5000, 3)])
def test_arena_matches_live_block_model(driver, arena, steps, seed):
    out = subprocess.run([str(driver), str(arena), str(steps), str(seed)], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
