"""bench.py's command-line contract that can be checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_measured_kernel_sources():
    """bench.py reports the measured HBM traffic only while the fill-kernel
    sources are the ones the counters were taken on, and null otherwise."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.traffic_bytes(0, 0)
    if bench.fill_sources_sha() == bench.TRAFFIC_SRC_SHA:
        assert t is not None and abs(t / (4 * 2**30) - 1) < 1e-3
    else:
        assert t is None
