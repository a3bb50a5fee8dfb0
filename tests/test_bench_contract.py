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


def test_binding_roof_is_the_longer_model_time():
    """A launch that takes exactly the HBM model time of its samples is at
    fraction 1 of the HBM roof; one that takes the VALU model time is at 1 of
    that roof, and the binding roof is always the one with the longer model
    time."""
    sys.path.insert(0, ROOT)
    import bench
    n = 1 << 30
    t_hbm_ms = 4.0 * n / (bench.HBM_PEAK_GBS * 1e9) * 1e3
    for g in range(5):
        for d in range(3):
            slots = (bench.SLOTS_GEN[g] + bench.SLOTS_DIST[d]) * n
            t_alu_ms = slots / (bench.VALU_PEAK_TSLOTS * 1e12) * 1e3
            r = bench.roofs(g, d, n, max(t_hbm_ms, t_alu_ms))
            assert abs(r["binding_frac"] - 1) < 1e-3
            assert r["binding"] == ("alu" if t_alu_ms > t_hbm_ms else "hbm")
            r2 = bench.roofs(g, d, n, 2 * max(t_hbm_ms, t_alu_ms))
            assert abs(r2["binding_frac"] - 0.5) < 1e-3
    # u32 Philox and Tyche need fewer slots per byte than HBM can absorb; every
    # normal fill needs more
    assert bench.roofs(0, 0, n, 1.0)["binding"] == "hbm"
    assert bench.roofs(4, 0, n, 1.0)["binding"] == "hbm"
    assert all(bench.roofs(g, 2, n, 1.0)["binding"] == "alu" for g in range(5))
