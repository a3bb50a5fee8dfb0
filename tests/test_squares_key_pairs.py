"""The Squares key K(seed) = SplitMix64(seed) | 1 maps two seeds to every
key (SplitMix64's output step is a bijection; the forced low bit merges the
seeds whose outputs differ only there).  A host program walks all 2^32 seeds
below 2^32, forms each seed's partner with the inverse of the SplitMix64
step, and finds exactly one pair of them that shares a key; the oracle's
Squares32 and Squares64 streams of that pair are equal, those of neighbouring
seeds are not."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIR = (369106595, 2888123536)


def test_one_pair_of_32_bit_seeds_shares_a_key(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "squares_key_pairs")
    subprocess.run([gxx, "-std=c++17", "-O2", "-pthread",
                    os.path.join(ROOT, "tests", "host", "squares_key_pairs.cc"),
                    os.path.join(ROOT, "oracle", "orng_oracle.cc"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.split()[:2] == ["pairs", "2"]  # one pair, counted from both sides


def test_the_pair_shares_its_streams(O):
    a, b = PAIR
    assert O.squares_key(a) == O.squares_key(b)
    for gen in (3, 8):  # Squares32, Squares64
        assert np.array_equal(O.fill(gen, 0, a, 7, 0, 4096), O.fill(gen, 0, b, 7, 0, 4096))
        assert not np.array_equal(O.fill(gen, 0, a, 7, 0, 4096), O.fill(gen, 0, a + 1, 7, 0, 4096))
        assert not np.array_equal(O.fill(gen, 0, b, 7, 0, 4096), O.fill(gen, 0, b - 1, 7, 0, 4096))
