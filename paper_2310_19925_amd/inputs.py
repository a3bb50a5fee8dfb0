"""Seeded synthetic workloads, shared by the tests, the benchmark and the oracle
checks.  This module holds no part of the generation method: it only draws the
seeds, counters, offsets, lengths and arrival times that the calls take.

Workload shapes follow the paper's experiments where it has them (section 5.1:
a Brownian walk over many independent particles; section 5.2: 16,000 parallel
streams of 3 draws) and otherwise the bulk, batched and served fill shapes
that the interface is built for.  No dataset is involved.
"""
from __future__ import annotations

import numpy as np

GEN_NAMES = ["philox4x32_10", "threefry4x32_20", "threefry2x64_20", "squares32", "tyche",
             "threefry4x32_13", "threefry2x64_13", "tyche_i", "squares64", "philox2x32_10"]
DIST_NAMES = ["u32", "f32_uniform", "f32_normal", "f64_uniform", "f64_normal"]
PERIOD = 1 << 32


def bulk_seed() -> int:
    """The 64-bit seed of the bulk fills: first raw draw of PCG64(231019925)."""
    return int(np.random.PCG64(231019925).random_raw())


# small multi-stream case: seed 42, 2^20 streams (ids 0..2^20-1) x 4 words
PLAIN_SEED, PLAIN_STREAMS, PLAIN_PER_STREAM = 42, 1 << 20, 4

# bulk fill: 2^30 samples per generator and distribution, one stream
BULK_N = 1 << 30

# walk: 2^24 particles in 3-D, 10^4 steps, dt = 1e-3, D = 1, from the origin
WALK = dict(n_particles=1 << 24, dim=3, n_steps=10_000, dt=1e-3, D=1.0, msd_every=1000)

# The paper's own 2-D Brownian dynamics run (section 5.1): one million
# particles, 10,000 steps, the generator of each particle keyed by its id and
# the loop iteration (which starts at 1).  Drag coefficient and time step are
# not given; gamma/mass = 1 and dt = 1e-3 here.  Particles start at rest at
# the origin.
BD2 = dict(n=1_000_000, pid0=0, step0=1, n_steps=10_000, dt=1e-3, gamma_over_m=1.0)


def batched_requests(n: int = 100_000, seed: int = 3, max_log2: float = 20.0):
    """Uneven Philox streams: lengths log-uniform in [1, 2^max_log2] words,
    random 64-bit seeds, random 32-bit counters, random word offsets with
    offset + length <= 2^32.  Returns a dict of numpy arrays plus packed
    output offsets (in samples) from a prefix sum of the lengths."""
    rng = np.random.default_rng(seed)
    top = 1 << int(max_log2)
    L = np.floor(2.0 ** (max_log2 * rng.random(n))).astype(np.int64)
    L = np.clip(L, 1, top)
    seeds = rng.integers(0, 2**63, size=n, dtype=np.int64).astype(np.uint64) * 2 + \
        rng.integers(0, 2, size=n, dtype=np.int64).astype(np.uint64)
    ctrs = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    offs = np.floor(rng.random(n) * (PERIOD - L + 1)).astype(np.uint64)
    out_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(L, out=out_off[1:])
    return dict(n=L.astype(np.uint64), seed=seeds, ctr=ctrs, offset=offs, out_off=out_off)


def serve_trace(n: int = 20_000, seed: int = 4, rate_per_s: float = 5000.0,
                log2_min: float = 10.0, log2_max: float = 26.0):
    """Poisson arrivals of mixed fill requests: exponential inter-arrival
    times (mean 1/rate), sizes log-uniform in [2^log2_min, 2^log2_max] words,
    generator uniform over the four families (Threefry split evenly between
    its 4x32 and 2x64 forms), distribution uniform over the three, random
    seed, counter and offset."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps) - gaps[0]
    size = np.floor(2.0 ** (log2_min + (log2_max - log2_min) * rng.random(n))).astype(np.uint64)
    fam = rng.integers(0, 4, size=n)
    tf_pick = rng.integers(0, 2, size=n)
    gen = np.select([fam == 0, fam == 1, fam == 2, fam == 3], [0, 1 + tf_pick, 3, 4])
    dist = rng.integers(0, 3, size=n)
    seeds = rng.integers(0, 2**63, size=n, dtype=np.int64).astype(np.uint64)
    ctrs = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    offs = np.floor(rng.random(n) * (PERIOD - size.astype(np.float64) + 1)).astype(np.uint64)
    return dict(t=t, n=size, gen=gen.astype(np.int32), dist=dist.astype(np.int32), seed=seeds,
                ctr=ctrs, offset=offs)
