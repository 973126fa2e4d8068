"""Host checks of bench.py (no GPU): the one-GPU contract, and the lookup of
HBM traffic in the committed rocprofv3 summaries (reported only while a
summary's source digest matches the current kernel sources)."""
import json
import pathlib
import subprocess
import sys

import pytest

import bench

ROOT = pathlib.Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                         timeout=300, cwd=ROOT)
    assert out.returncode != 0
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_source_digest_is_stable_and_covers_the_includes():
    a = bench.source_digest("generate.hip")
    assert a == bench.source_digest("generate.hip") and len(a) == 16
    assert a != bench.source_digest("lfg.hip")


def test_profiled_traffic_of_the_bulk_line():
    """The committed summary of the bulk line's launch was taken from the
    current sources: its traffic (fetch + write per dispatch) is at least the
    algorithmic bytes (4 GiB written, 392 MiB of states read) and within 5% of
    them; a kernel or grid that is not in the summary gives None."""
    digest = bench.source_digest("generate.hip")
    if digest not in (ROOT / "profiles" / "gen_bulk1m_hbm_traffic.md").read_text():
        pytest.skip("the bulk line's traffic summary predates the current generation sources")
    n = 1 << 20
    algo = 4 * n * 1024 + 392 * n
    t = bench.profiled_traffic("k_gen32_wide<1, true", n // 8 * 256, "generate.hip")
    assert t is not None and algo <= t <= 1.05 * algo
    assert bench.profiled_traffic("k_gen32_wide<1, true", n // 8 * 256 + 1, "generate.hip") is None
    assert bench.profiled_traffic("no_such_kernel", n // 8 * 256, "generate.hip") is None
