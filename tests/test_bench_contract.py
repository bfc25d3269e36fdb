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


def test_counter_records_apply_only_to_the_kernel_they_were_taken_on(tmp_path):
    """The committed traffic and issue records are reported while the kernel
    source hash matches, and dropped (None) once it differs."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    from paper_2210_01076_amd import profiling
    h = profiling.kernel_source_hash()
    good, stale = tmp_path / "good.json", tmp_path / "stale.json"
    rec = {"kernel_source_hash": h, "hbm_bytes_per_launch": 123.0, "valu_issue_share": 0.5, "valu_bound_us": 20000.0}
    good.write_text(json.dumps(rec))
    stale.write_text(json.dumps(dict(rec, kernel_source_hash="0" * 16)))
    assert bench.load_traffic(str(good)) == 123.0 and bench.load_traffic(str(stale)) is None
    issue = bench.load_issue(str(good), 40.0)
    assert issue["valu_bound_ms"] == 20.0 and issue["frac_of_valu_bound"] == 0.5
    assert bench.load_issue(str(stale), 40.0) is None and bench.load_issue(str(tmp_path / "none.json"), 40.0) is None
