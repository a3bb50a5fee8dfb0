import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def O():
    """The oracle module (test infrastructure), built if absent."""
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def rocrand_xcheck(tmp_path_factory):
    """Path of a host-only program that evaluates rocRAND's block functions."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    out = str(tmp_path_factory.mktemp("xcheck") / "rocrand_xcheck")
    src = os.path.join(HERE, "xcheck", "rocrand_xcheck.cpp")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17", src, "-o", out],
                   check=True, capture_output=True)
    return out


def run_xcheck(exe, lines):
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True)
    return [list(map(int, l.split())) for l in res.stdout.strip().split("\n")]
