"""bench.py's command-line contract on the CPU: more than one GPU is
refused with a message (the state and the sessions are not sharded), and
the helpers it reports with behave as documented."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout.strip() == ""


def test_percentile_helper():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.pct([], 50) is None
    assert bench.pct([3.0], 99) == 3.0
    assert bench.pct([1.0, 2.0, 3.0, 4.0], 50) == 2.5
    assert bench.pct(list(range(101)), 99) == 99.0
