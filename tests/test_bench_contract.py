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


def test_traffic_table_matches_the_kernel_sources():
    """The measured HBM traffic embedded in bench.py belongs to the current
    fill-kernel sources (otherwise bench.py reports traffic as null)."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.fill_sources_sha() == bench.TRAFFIC_SRC_SHA
    t = bench.traffic_bytes(0, 0)
    assert t is not None and abs(t / (4 * 2**30) - 1) < 1e-3
