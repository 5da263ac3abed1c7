"""Host logic of bench.py (no GPU): the one-GPU contract and the pass schedule the roofline
figures are computed from (the library's rule: passes of k stages, a remainder of two or
more stages as one pass of that depth where the tile supports it, and no pass that both
reads and writes the caller's state)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("s", [2, 4, 6, 8, 16, 64, 98, 100, 400, 512, 514])
def test_pass_schedule_invariants(s, k):
    sched = bench.pass_schedule(s, k)
    assert sum(sched) == s
    assert all(p == 1 or p in (2, 3) for p in sched)
    assert all(p <= max(k, 1) for p in sched)
    if s > 1:
        assert sched[0] != s          # the first pass reads w, the last writes it
    if k == 1:
        assert sched == [1] * s
    if k == 3 and s >= 4:
        assert 1 not in sched         # no lone single-stage pass


def test_pass_schedule_examples():
    assert bench.pass_schedule(100, 3) == [3] * 32 + [2, 2]
    assert bench.pass_schedule(98, 3) == [3] * 32 + [2]
    assert bench.pass_schedule(100, 2) == [2] * 50
    assert bench.pass_schedule(2, 3) == [1, 1]
    assert bench.pass_schedule(3 + 1, 3) == [2, 2]
    assert bench.pass_schedule(64, 3) == [3] * 20 + [2, 2]
