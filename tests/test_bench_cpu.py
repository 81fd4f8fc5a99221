"""bench.py host logic (no GPU): the one-GPU guard and the workload sizing."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("name", ["batch", "beam_box", "plate_sweep"])
def test_workload_window_is_the_timed_steps(name):
    """The lock-in window is exactly the K timed steps after the warmup; the
    solves have room for the second (kernel-timing) pass after it."""
    import bench
    solves, desc = bench.workload(name, steps=100, warmup=10)
    assert desc.startswith(name)
    for s in solves:
        assert s.window_first == 10 and s.window_count == 100
        assert s.nsteps == 10 + 2 * 100
