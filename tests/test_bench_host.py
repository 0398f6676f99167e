"""Host logic of bench.py, on the CPU: the share of updates that reuse the
previous sweep's random words (which weights the roofline's issue slots
per update), and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_stash_fraction_by_hand():
    # 100 single-sweep a-rule passes, then 900 sweeps in passes of 8 from
    # sweep 100: the odd sweeps 101, 103, 105, 107 of each full pass (112
    # passes) and 901, 903 of the last pass of 4 (sweeps 996-999 -> 997, 999)
    assert bench.stash_fraction(100, 900, 8) == pytest.approx((112 * 4 + 2) / 1000)
    # passes of 1: nothing is reused
    assert bench.stash_fraction(100, 100, 1) == 0.0
    # an odd first sampling sweep: pass 5..12 reuses at 7, 9, 11 only
    assert bench.stash_fraction(5, 8, 8) == pytest.approx(3 / 13)
    # passes of 2 from an even sweep: every second sweep
    assert bench.stash_fraction(0, 10, 2) == pytest.approx(0.5)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
