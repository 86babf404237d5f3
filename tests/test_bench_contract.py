"""bench.py's command-line contract on the CPU: a multi-GPU request exits
with a message (this path measures one GPU), before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_measured_traffic_needs_matching_sources():
    """roofline.traffic comes from the committed counter profile only while
    it was taken on the current library sources."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("no_such_kernel") is None
    assert bench.measured_traffic("k_down_off", "no_such_profile.json") is None
