#!/usr/bin/env python3
"""Benchmark of the counter-based generation hot path on one MI355X.

One step = one bulk fill of 2^30 samples for every generator (Philox4x32-10,
Threefry4x32-20, Threefry2x64-20, Squares32, Tyche) and every distribution
(u32, f32 uniform, f32 Box-Muller normal): 15 launches, 60 GiB written,
single stream (seed from PCG64(231019925), counter 0) counter-partitioned
across the grid.  `value` is whole-step throughput in GSamples/s with the
output resident in HBM.  Per-kernel durations come from HIP events recorded on
the launch stream around every launch of the timed steps.

Also reported (same JSON line): the fused Brownian walk (2^24 particles, 3-D,
10^4 steps) in steps/s; the paper's 2-D Brownian dynamics run (10^6
particles, 10^4 steps, float64) fused and with one launch per step; the
batched and served paths; and the CPU oracle on a bounded sample of the same
fill workload as the CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-walk] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
# VALU issue peak: 256 CUs x 64 lanes x 2.4 GHz full-rate 32-bit lane operations
# ("slots") per second.
VALU_PEAK_TSLOTS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic VALU slots per sample of each generator and distribution.  The
# operations the definitions require, written with the shortest gfx950 encoding
# of each (64-bit add, 32x32->64 product-add, three-input xor or add, funnel
# rotate: one instruction each); work on values uniform across a wave (keys,
# the stream counter) runs on the scalar unit and is not counted; an fp32
# operation counts half a slot (the published 157.3 TFLOP/s vector rate is two
# fp32 operations per lane and clock), a reciprocal or reciprocal square root
# one.  Every choice undercounts rather than overcounts.
#   Philox4x32-10: 10 rounds x (2 products + 2 xor3), round 1 half uniform: 38 / 4 words
#   Threefry4x32-20: 18 full rounds x 6 + rounds 1-2 (2 + 5) + counter add 1
#     + injections 4 x 2 (x0, x2 fold into the next round's add) + final 4: 128 / 4 words
#   Threefry2x64-20: 19 rounds x (add 1 + rotate 2 + xor 2) + round 1 (3) + counter add 1
#     + 5 injections x 2 adds: 109 / 4 words
#   Squares32: 4 rounds x (product-add, low product, shift-add) + 1 add (y -> z) per
#     word, one full y product (3) per 4 words
#   Tyche: one MIX (4 add, 4 xor, 4 rotate) per word + 20 MIX per 256 words (lane init)
#   f32 uniform: shift + convert + scale = 1 + 2 x 0.5
#   f32 normal, per pair: 16 integer ops, 37 fp32 ops, rcp + rsq = 36.5 slots
#   Threefry4x32-13: 11 full rounds x 6 + rounds 1-2 (7) + counter add 1 + 3
#     injections x 2 (no injection after round 13): 80 / 4 words
#   Threefry2x64-13: 12 rounds x 5 + round 1 (3) + counter add 1 + 3 x 2: 70 / 4 words
#   Philox2x32-10: 10 rounds x (1 product + 1 xor3) per two-word block: 10 / word
SLOTS_GEN = {0: 38 / 4, 1: 128 / 4, 2: 109 / 4, 3: 13 + 3 / 4, 4: 12 + 20 * 12 / 256,
             5: 80 / 4, 6: 70 / 4, 7: 12 + 20 * 12 / 256, 8: (5 * 3 + 2 + 1) / 2 + 3 / 4,
             9: 10.0}
SLOTS_DIST = {0: 0.0, 1: 2.0, 2: 36.5 / 2}
# Fused walk, per particle, step and coordinate: one Philox word, one
# Box-Muller sample (half a pair, 18.25) and the fmaf update (an fp32
# operation, 0.5).  The walk's Philox counter is (block, ctr0 + particle, 0,
# 0): the block index is the same for every lane of a wave (all particles are
# at the same step), so more of the first rounds is uniform than in a fill
# (whose block index varies by lane): round 1 leaves one vector xor, round 2 one
# product and one xor3, round 3 one product and two xor3, rounds 4-10 two of
# each: 34 slots per block, 8.5 per word.  27.25 slots; 81.75 per
# particle-step in 3-D.
WALK_SLOTS_PER_DIM = 34 / 4 + 36.5 / 2 + 0.5
# float64 uniform: two words per sample, then shift, two conversions, one
# exact fma and one scaling (float64 operations: one slot each at the
# published 78.6 TFLOP/s vector rate); 8 bytes written per sample
SLOTS_F64_CONVERT = 5
# float64 normal, per pair (two samples) counted from the definition, one slot
# per float64 operation (full rate: 78.6 TFLOP/s = one FMA per lane and clock):
# ln 35 (exponent split 5, division 11, series 11, assembly 8), square root 13,
# sin/cos 40 (integer quarter-turn split 10, series 22, rotation 8), products 2,
# word handling 6; 8 bytes written per sample
SLOTS_F64N_CONVERT = 96 / 2
# integer in [lo, hi): two words per sample, two 32x32->64 multiply-adds and
# the add of lo; 4 bytes written per sample
SLOTS_RANGE_CONVERT = 3
RANGE_LO, RANGE_HI = -10**9, 10**9 + 7


def roofs(gen, dist, n, ms):
    """HBM and VALU roofline fractions of one fill launch; the binding roof is
    the one whose model time is longer."""
    t = ms * 1e-3
    if dist == 3:  # float64 uniform
        slots, nbytes = (2 * SLOTS_GEN[gen] + SLOTS_F64_CONVERT) * n, 8.0 * n
    elif dist == 4:  # float64 normal
        slots, nbytes = (2 * SLOTS_GEN[gen] + SLOTS_F64N_CONVERT) * n, 8.0 * n
    elif dist == "range":  # int32 in [lo, hi)
        slots, nbytes = (2 * SLOTS_GEN[gen] + SLOTS_RANGE_CONVERT) * n, 4.0 * n
    else:
        slots, nbytes = (SLOTS_GEN[gen] + SLOTS_DIST[dist]) * n, 4.0 * n
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = slots / (VALU_PEAK_TSLOTS * 1e12)
    return {"valu_tslots_s": round(slots / t / 1e12, 2), "valu_frac": round(t_alu / t, 4),
            "binding": "alu" if t_alu > t_hbm else "hbm",
            "binding_frac": round(max(t_alu, t_hbm) / t, 4), "slots": slots}


# HBM traffic per launch of each bulk fill from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE, KiB per dispatch; see profiles/), with the
# calibration factors a 1 GiB device copy gives for each counter.  Valid only
# for the kernel sources and launch table they were measured on: bench.py
# reports null traffic when the hash of those sources differs.
TRAFFIC_SRC_SHA = "9a2c8864b6a9f0bb"
TRAFFIC_FACTORS = (1.9999227553638532, 1.0)  # FETCH, WRITE
TRAFFIC_KIB = {
    (0, 0): (80.4375, 4194304.0), (0, 1): (45.4375, 4195201.5), (0, 2): (63.4375, 4194307.75), (0, 3): (27.5, 4194304.0),
    (0, 4): (40.0, 4194320.75), (1, 0): (41.375, 4194319.875), (1, 1): (63.5625, 4194322.375), (1, 2): (65.375, 4194304.0),
    (1, 3): (56.0625, 4194325.9375), (1, 4): (73.0, 4194305.15625), (2, 0): (44.0, 4194308.5), (2, 1): (47.0, 4194363.875),
    (2, 2): (87.375, 4194304.0), (2, 3): (42.5, 4194322.875), (2, 4): (82.390625, 4194304.0), (3, 0): (37.5, 4194353.875),
    (3, 1): (31.0, 4195754.75), (3, 2): (72.5, 4194320.75), (3, 3): (36.0, 4198136.21875), (3, 4): (64.0, 4194321.65625),
    (4, 0): (33.125, 4194304.0), (4, 1): (27.1875, 4194304.0), (4, 2): (37.8125, 4194311.25), (4, 3): (33.765625, 4194304.0),
    (4, 4): (43.078125, 4194316.75), (5, 0): (43.5, 4195897.0), (5, 1): (45.5, 4195480.15625), (5, 2): (63.0, 4194332.5),
    (5, 3): (53.0, 4196126.71875), (5, 4): (70.0, 4194313.25), (6, 0): (52.0, 4194304.0), (6, 1): (53.5, 4197727.9375),
    (6, 2): (42.5, 4194329.65625), (6, 3): (37.0, 4197525.40625), (6, 4): (66.0, 4194310.6875), (7, 0): (31.421875, 4194304.0),
    (7, 1): (32.53125, 4194304.0), (7, 2): (36.53125, 4194354.1875), (7, 3): (31.65625, 4194304.0), (7, 4): (37.09375, 4194315.34375),
    (8, 0): (34.0, 4197164.53125), (8, 1): (35.578125, 4194304.0), (8, 2): (45.0, 4194361.6875), (8, 3): (35.5, 4197798.1875),
    (8, 4): (54.5, 4194315.8125), (9, 0): (51.0, 4194304.0), (9, 1): (19.0, 4194304.0), (9, 2): (26.0, 4194342.28125),
    (9, 3): (51.0, 4194304.0), (9, 4): (42.5, 4194315.40625),
}


def fill_sources_sha():
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2310_19925_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "orng_device.hpp")) +
                   glob.glob(os.path.join(csrc, "orng_host.hpp")) +
                   glob.glob(os.path.join(csrc, "orng_span.hpp")) +
                   glob.glob(os.path.join(csrc, "orng_fill.hip")) +
                   glob.glob(os.path.join(csrc, "orng_tune.cpp")))
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in files)).hexdigest()[:16]


def traffic_bytes(gen, dist):
    if fill_sources_sha() != TRAFFIC_SRC_SHA or (gen, dist) not in TRAFFIC_KIB:
        return None
    f, w = TRAFFIC_KIB[(gen, dist)]
    return round(f * 1024 * TRAFFIC_FACTORS[0] + w * 1024 * TRAFFIC_FACTORS[1])


def key32(gen, seed):
    """Philox2x32-10 (generator 9) keys with one 32-bit word: its fills take
    the low word of the seed the other generators use."""
    return seed & 0xFFFFFFFF if gen == 9 else seed


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_threads():
    """Every host core this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seed, target_s=30.0):
    """Oracle (test infrastructure, untuned) built for this host with -O3
    -march=native -ffp-contract=off, on every host core: the same 15 fills on
    a bounded sample of each, scaled to GSamples/s.  The sample is sized from
    a 2^20-sample trial run; the trial's fixed costs make the estimate about
    twice the real time, so target_s = 30 gives ~10-15 s."""
    import numpy as np
    from oracle import oracle as O
    L = O.lib_native()
    th = cpu_threads()
    per = 1 << 20
    buf_u = np.empty(per, np.uint32)
    t0 = time.perf_counter()
    for g in range(5):
        for d in range(3):
            assert L.oracle_fill(g, d, seed, 0, 0, per, buf_u.ctypes.data, th) == 0
    t_small = time.perf_counter() - t0
    # the native build computes the same words as the test-suite's build
    ref = O.fill(4, 2, seed, 0, 0, per)
    assert np.array_equal(buf_u, ref.view(np.uint32))
    scale = max(1, min(1024, int(target_s / max(t_small, 1e-3))))  # at most the whole 2^30
    per = per * scale
    buf_u = np.empty(per, np.uint32)
    t0 = time.perf_counter()
    for g in range(5):
        for d in range(3):
            assert L.oracle_fill(g, d, seed, 0, 0, per, buf_u.ctypes.data, th) == 0
    dt = time.perf_counter() - t0
    res = {"value": round(15 * per / dt / 1e9, 4), "unit": "GSamples/s", "cores": th,
           "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
           "build": "g++ " + " ".join(O.NATIVE_FLAGS) + " -ffp-contract=off",
           "sample": "first %d samples of each of the 15 fills (gen x dist), %.1f s wall"
                     % (per, dt)}
    # the plain multi-stream fill in full (2^20 streams x 4 words, u32 and f32 uniform)
    from paper_2310_19925_amd import inputs
    ns, ps = inputs.PLAIN_STREAMS, inputs.PLAIN_PER_STREAM
    buf_m = np.empty(ns * ps, np.uint32)
    t0 = time.perf_counter()
    for _ in range(5):
        for d in (0, 1):
            assert L.oracle_fill_multi(0, d, inputs.PLAIN_SEED, 0, ns, 0, ps,
                                       buf_m.ctypes.data, th) == 0
    t_m = (time.perf_counter() - t0) / 10
    res["plain_multi"] = {"ms": round(t_m * 1e3, 3),
                          "gsamples_s": round(ns * ps / t_m / 1e9, 4),
                          "sample": "whole fill, u32 and f32 uniform, 5 runs each"}
    # the walk on a subset of the particles (65,536 of 2^24), for as many of the 10^4
    # steps as fit about 4 s, reported per particle-step (extrapolated to the full walk)
    count, dim = 65536, 3
    sig = (np.float32(1e-3), np.float32(1.0))

    def walk(steps):
        pos = np.zeros((dim, count), np.float32)
        t = time.perf_counter()
        assert L.oracle_brownian(seed, 0, None, count, dim, 0, steps, sig[0], sig[1],
                                 pos.ctypes.data, None, 0, th) == 0
        return time.perf_counter() - t
    t_w = walk(50)
    steps = max(50, min(10000, int(50 * 4.0 / max(t_w, 1e-3))))
    t_w = walk(steps)
    ps_rate = count * steps / t_w
    res["walk"] = {"particle_steps_per_s": round(ps_rate, 1),
                   "full_walk_s_extrapolated": round(2**24 * 10000 / ps_rate, 1),
                   "sample": "%d particles x %d steps (3-D), %.1f s wall; extrapolated per "
                             "particle-step" % (count, steps, t_w)}
    return res


def _time_events(stream, fn, reps):
    import torch
    fn()  # warm-up
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    return ms[len(ms) // 2]


def bench_plain_multi(orng, inputs, stream, dev):
    """The configured plain multi-stream fill: one seed (42), 2^20 streams
    (counters 0..2^20-1) of 4 words each, u32 and float32 uniform (and the
    same streams as 4 integers each); one launch, so microseconds."""
    import torch
    ns, per = inputs.PLAIN_STREAMS, inputs.PLAIN_PER_STREAM
    n = ns * per
    out = torch.empty(n, dtype=torch.int32, device=dev)
    res = {"n_streams": ns, "per_stream": per}
    for d, name in ((0, "u32"), (1, "f32_uniform")):
        ms = _time_events(stream, lambda: orng.orng_fill_multi(0, d, inputs.PLAIN_SEED, 0, ns, 0,
                                                               per, out, stream), 21)
        res[name] = {"us": round(ms * 1e3, 2), "gsamples_s": round(n / (ms * 1e-3) / 1e9, 2)}
    # the same streams as integers in [lo, hi) (two words per sample)
    ms = _time_events(stream, lambda: orng.orng_fill_range(0, inputs.PLAIN_SEED, 0, ns, 0, per,
                                                           RANGE_LO, RANGE_HI, out, stream), 21)
    res["i32_range"] = {"us": round(ms * 1e3, 2), "gsamples_s": round(n / (ms * 1e-3) / 1e9, 2)}
    del out
    return res


def bench_batched(orng, inputs, stream, dev):
    """10^5 Philox u32 streams of log-uniform length in [1, 2^20] words, packed
    back to back: batched (the tuned schedule, with the persistent work-queue
    kernel and the allocation-free call timed beside it) vs one launch per
    stream vs one plain fill of the same number of words."""
    import torch
    b = inputs.batched_requests()
    total = int(b["out_off"][-1])
    buf = torch.empty(total, dtype=torch.int32, device=dev)
    reqs = orng.make_requests(0, 0, b["seed"], b["ctr"], b["offset"], b["n"],
                              buf.data_ptr() + 4 * b["out_off"][:-1])
    t_batched = _time_events(stream, lambda: orng.orng_fill_batched(reqs, stream), 5)
    # The persistent work-queue kernel on the same batch: a grid cap selects it
    # (4 workgroups per compute unit, the tuner's persistent shape); the tuned
    # default for Philox u32 is the static one-workgroup-per-tile schedule.
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    orng.orng_set_launch(max_wgs=4 * cus)
    try:
        t_queue = _time_events(stream, lambda: orng.orng_fill_batched(reqs, stream), 5)
    finally:
        orng.orng_reset_launch()
    # the allocation-free call (tables in the library's fixed device array;
    # its row upload is part of the timed span)
    t_noalloc = _time_events(stream, lambda: orng.orng_fill_batched_noalloc(reqs, stream), 5)
    t_each = _time_events(stream, lambda: orng.orng_fill_each(reqs, stream), 2)
    half = total // 2
    t_plain = _time_events(stream, lambda: orng.orng_fill_multi(0, 0, 42, 0, 2, 0, half, buf,
                                                                 stream), 5)
    # host time of one batched call (validation, tiling, staging, enqueue)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    orng.orng_fill_batched(reqs, stream)
    t_host = (time.perf_counter() - h0) * 1e3
    torch.cuda.synchronize()
    # back-to-back calls: host preparation of call k+1 overlaps call k on the device
    K = 8
    t_batched_pipe = _time_events(stream, lambda: [orng.orng_fill_batched(reqs, stream)
                                                   for _ in range(K)], 3) / K
    t_plain_pipe = _time_events(stream, lambda: [orng.orng_fill_multi(0, 0, 42, 0, 2, 0, half,
                                                                      buf, stream)
                                                 for _ in range(K)], 3) / K
    del buf
    torch.cuda.empty_cache()
    g = lambda ms, words: round(words / (ms * 1e-3) / 1e9, 2)
    return {"requests": int(b["n"].size), "words": total,
            "batched_ms": round(t_batched, 3), "batched_gsamples_s": g(t_batched, total),
            "schedule": "static (one workgroup per tile)",
            "queue_ms": round(t_queue, 3), "queue_gsamples_s": g(t_queue, total),
            "queue_vs_plain": round(t_plain / t_queue * total / (2 * half), 4),
            "noalloc_ms": round(t_noalloc, 3), "noalloc_gsamples_s": g(t_noalloc, total),
            "each_ms": round(t_each, 3), "each_gsamples_s": g(t_each, total),
            "plain_ms": round(t_plain, 3), "plain_gsamples_s": g(t_plain, 2 * half),
            "batched_vs_plain": round(t_plain / t_batched * total / (2 * half), 4),
            "batched_vs_each": round(t_each / t_batched, 2),
            "batched_host_ms": round(t_host, 3),
            "pipelined": {"batched_ms": round(t_batched_pipe, 3),
                          "plain_ms": round(t_plain_pipe, 3),
                          "batched_gsamples_s": g(t_batched_pipe, total),
                          "batched_vs_plain": round(t_plain_pipe / t_batched_pipe * total
                                                    / (2 * half), 4)}}


# the serving workload's HBM budget: 32 GB (10^9 bytes), in whole 256-byte granules
SERVE_ARENA_BYTES = 32_000_000_000 // 256 * 256


def _replay(orng, tr, idx, arena_bytes, open_loop):
    """Submit the requests of trace `tr` selected by `idx` to a fresh server
    (server-allocated outputs), at their arrival times (open loop) or all at
    once (saturated); a second thread waits for each ticket in order and
    releases it right after completion.  Returns the server statistics."""
    import threading
    srv = orng.orng_serve_create(arena_bytes)
    tickets = [None] * len(idx)
    ready = threading.Semaphore(0)

    def releaser():
        for k in range(len(idx)):
            ready.acquire()
            orng.orng_serve_wait(srv, tickets[k])
            orng.orng_serve_release(srv, tickets[k])

    if not open_loop:
        # every request arrives at t = 0: one submission of all of them, and the
        # client releases each result as soon as it is done
        reqs = orng.make_requests(tr["gen"][idx], tr["dist"][idx], tr["seed"][idx],
                                  tr["ctr"][idx], tr["offset"][idx], tr["n"][idx], 0)
        all_t = orng.orng_serve_submit_many(srv, reqs)
        for k in range(0, len(all_t), 64):
            orng.orng_serve_release_many(srv, all_t[k:k + 64])
        st = orng.orng_serve_stats(srv)
        orng.orng_serve_destroy(srv)
        return st
    th = threading.Thread(target=releaser)
    th.start()
    t0 = time.perf_counter()
    for k, i in enumerate(idx):
        dt = t0 + float(tr["t"][i]) - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets[k] = orng.orng_serve_submit(srv, int(tr["gen"][i]), int(tr["dist"][i]),
                                            int(tr["seed"][i]), int(tr["ctr"][i]),
                                            int(tr["offset"][i]), int(tr["n"][i]))
        ready.release()
    th.join()
    st = orng.orng_serve_stats(srv)
    orng.orng_serve_destroy(srv)
    return st


# VALU slots per particle-step of the paper's 2-D Brownian dynamics: one
# Philox block (round 1 on the zero counter words folds to one xor3; 9 rounds
# x (2 product-adds + 2 xor3): 37; the per-lane key schedule depends only on
# the particle and is formed once per launch, not per step) and 20 float64
# operations (two 53-bit conversions of 4 each; per component the centred
# kick (subtract, multiply), the decayed velocity (multiply, add) and the move
# (multiply, add)).  The published 78.6 TFLOP/s float64 vector rate is one
# operation per lane and clock, so each is one slot.
BD2_SLOTS = 37 + 20
BD2_BYTES_PER_STEP = 64  # one launch per step: load and store x, y, vx, vy


def bench_bd2(orng, inputs, stream, dev, per_step_too=True):
    """The paper's 2-D Brownian dynamics run (10^6 particles, 10^4 steps):
    all steps in one launch vs one launch per step (the paper's structure)."""
    import torch
    p = inputs.BD2
    n, T = p["n"], p["n_steps"]
    st = torch.zeros((4, n), dtype=torch.float64, device=dev)

    def run(spl):
        st.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        orng.orng_bd2(p["pid0"], n, p["step0"], T, p["dt"], p["gamma_over_m"], st[0], st[1],
                      st[2], st[3], spl, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    orng.orng_bd2(p["pid0"], n, p["step0"], 10, p["dt"], p["gamma_over_m"], st[0], st[1], st[2],
                  st[3], 1, stream)  # warm-up
    fused = min(run(0) for _ in range(2))
    per_step = run(1) if per_step_too else None
    ps = n * T
    slots = BD2_SLOTS * ps
    del st
    r = {"n_particles": n, "n_steps": T, "fused_ms": round(fused, 3),
         "fused_particle_steps_per_s": round(ps / (fused * 1e-3), 1),
         "fused_valu_tslots_s": round(slots / (fused * 1e-3) / 1e12, 2),
         "fused_valu_frac": round(slots / (fused * 1e-3) / 1e12 / VALU_PEAK_TSLOTS, 4)}
    if per_step is not None:
        r.update({"per_step_launch_ms": round(per_step, 3),
                  "fused_vs_per_step": round(per_step / fused, 3),
                  "per_step_gbs": round(BD2_BYTES_PER_STEP * ps / (per_step * 1e-3) / 1e9, 1)})
    return r


# VALU slots per 3-word micro-stream (one stream per particle and iteration):
# one counter block for Philox/Threefry (3 of its 4 words used); three
# Squares words plus the y product; Tyche seeds an instance (20 MIX) and runs
# 3 more for its 3 words (12 slots per MIX); the 13-round Threefry blocks;
# Tyche-i as Tyche;
# Squares64 two calls (5 rounds of 3 slots, the 64-bit adds and the XOR);
# Philox2x32 two two-word blocks.  The generators that run this shape with one
# key schedule per micro-stream (the flat schedule) also pay for it: Philox's
# 18 round-key additions, Threefry4x32's parity word, and Squares64's key
# (one SplitMix64 step, about 20 slots).
PART_SLOTS_3 = {0: 38 + 18, 1: 128 + 1, 2: 109, 3: 3 + 3 * 13, 4: 23 * 12, 5: 80 + 1, 6: 70,
                7: 23 * 12, 8: 3 + 2 * 18 + 20, 9: 40}


def bench_particles(orng, inputs, stream, dev):
    """Section 5.2's parallel-stream shape: 16,000 particles x 3 draws per
    iteration, ~4 GiB of concatenated micro-streams per generator."""
    import torch
    P, D = 16000, 3
    T = (1 << 30) // (P * D)
    out = torch.empty(T * P * D, dtype=torch.int32, device=dev)
    res = []
    for g in range(10):
        ms = _time_events(stream, lambda: orng.orng_particle_streams(g, 1, P, D, 1, T, out,
                                                                     stream), 3)
        words = T * P * D
        t_hbm = 4.0 * words / (HBM_PEAK_GBS * 1e9)
        t_alu = PART_SLOTS_3[g] * T * P / (VALU_PEAK_TSLOTS * 1e12)
        res.append({"gen": inputs.GEN_NAMES[g], "ms": round(ms, 4),
                    "write_gbs": round(4.0 * words / (ms * 1e-3) / 1e9, 1),
                    "binding": "alu" if t_alu > t_hbm else "hbm",
                    "binding_frac": round(max(t_alu, t_hbm) / (ms * 1e-3), 4)})
    del out
    torch.cuda.empty_cache()
    return {"particles": P, "draws": D, "iterations": T, "words": T * P * D, "gens": res}


def bench_serve(orng, inputs, stream, dev, bulk_rates=None):
    """Poisson arrivals (mean 5,000/s) of mixed fill requests, sizes
    log-uniform in [2^10, 2^26] words, four generator families x three
    distributions, 32 GB arena: open-loop replay (latency) and saturated
    replay of the same trace (throughput) vs one plain launch per request."""
    import numpy as np
    import torch
    tr = inputs.serve_trace()
    m = tr["n"].size
    idx = np.arange(m)
    words = int(tr["n"].sum())
    op = _replay(orng, tr, idx, SERVE_ARENA_BYTES, True)
    sat = _replay(orng, tr, idx, SERVE_ARENA_BYTES, False)
    # plain path on the same requests: one fill launch each, outputs in a ring
    cap = 8 << 30  # words
    buf = torch.empty(cap, dtype=torch.int32, device=dev)
    offs, pos = np.zeros(m, np.int64), 0
    for i in range(m):
        if pos + int(tr["n"][i]) > cap:
            pos = 0
        offs[i] = pos
        pos += (int(tr["n"][i]) + 63) // 64 * 64
    reqs = orng.make_requests(tr["gen"], tr["dist"], tr["seed"], tr["ctr"], tr["offset"],
                              tr["n"], buf.data_ptr() + 4 * offs)
    t_plain = _time_events(stream, lambda: orng.orng_fill_each(reqs, stream), 2)
    del buf
    torch.cuda.empty_cache()
    gs = lambda st: round(st["samples_done"] / st["first_submit_to_last_done_s"] / 1e9, 2)
    plain = words / (t_plain * 1e-3) / 1e9
    extra = {}
    if bulk_rates:
        # the same samples at the bulk-fill rate of each request's (gen, dist)
        t_bulk = sum(float(tr["n"][i]) / (bulk_rates[(int(tr["gen"][i]), int(tr["dist"][i]))] * 1e9)
                     for i in range(m))
        extra = {"bulk_rate_equiv_gsamples_s": round(words / t_bulk / 1e9, 2),
                 "saturated_vs_bulk_rate": round(gs(sat) / (words / t_bulk / 1e9), 4)}
    return {"requests": int(m), "samples": words, "offered_req_per_s": 5000,
            "arena_bytes": SERVE_ARENA_BYTES,
            "open_loop": {"p50_ms": round(op["latency_p50_ms"], 4),
                          "p99_ms": round(op["latency_p99_ms"], 4),
                          "mean_ms": round(op["latency_mean_ms"], 4),
                          "gsamples_s": gs(op), "steps": op["steps"],
                          "active_peak": op["active_peak"],
                          "arena_peak_gb": round(op["arena_peak_bytes"] / 1e9, 3)},
            "saturated": {"gsamples_s": gs(sat), "p50_ms": round(sat["latency_p50_ms"], 3),
                          "p99_ms": round(sat["latency_p99_ms"], 3), "steps": sat["steps"],
                          "active_peak": sat["active_peak"],
                          "arena_peak_gb": round(sat["arena_peak_bytes"] / 1e9, 3)},
            "plain_each_gsamples_s": round(plain, 2),
            "saturated_vs_plain": round(gs(sat) / plain, 4), **extra}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-walk", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-bd2", action="store_true")
    ap.add_argument("--no-particles", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--bd2-fused-only", action="store_true",
                    help="skip the one-launch-per-step Brownian dynamics run (counter runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (counter calibration)")
    ap.add_argument("--walk-steps", type=int, default=0, help="shorter walk (profiling runs)")
    ap.add_argument("--only", default="", help="gen:dist list to restrict the fills (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every stream is generated where it is used, "
              "with no communication between GPUs (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_19925_amd import inputs, orng
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    seed = inputs.bulk_seed()
    n = inputs.BULK_N
    combos = [(g, d) for g in range(5) for d in range(3)]
    if args.only:
        keep = {tuple(int(x) for x in s.split(":")) for s in args.only.split(",")}
        combos = [c for c in combos if c in keep]
    out = torch.empty(n, dtype=torch.int32, device=dev)

    def step(events=None):
        for k, (g, d) in enumerate(combos):
            if events is not None:
                events[k][0].record(stream)
            orng.orng_fill(g, d, seed, 0, 0, n, out, stream)
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in combos] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_kernel_ms = [sum(evs[s][k][0].elapsed_time(evs[s][k][1]) for s in range(args.steps))
                     / args.steps for k in range(len(combos))]
    total_samples = len(combos) * n * args.steps
    value = total_samples / wall / 1e9
    ms_per_step = wall / args.steps * 1e3

    # measured store-only ceiling: a plain store kernel (torch's fill) on the same buffer
    t_store = _time_events(stream, lambda: out.fill_(0), 5)
    ceiling_gbs = 4.0 * n / (t_store * 1e-3) / 1e9

    kernels = []
    for (g, d), ms in zip(combos, per_kernel_ms):
        gbs = 4.0 * n / (ms * 1e-3) / 1e9
        rf = roofs(g, d, n, ms)
        kernels.append({"gen": inputs.GEN_NAMES[g], "dist": inputs.DIST_NAMES[d],
                        "ms": round(ms, 4), "gsamples_s": round(n / (ms * 1e-3) / 1e9, 2),
                        "write_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "store_ceiling_frac": round(gbs / ceiling_gbs, 4),
                        "valu_tslots_s": rf["valu_tslots_s"], "valu_frac": rf["valu_frac"],
                        "binding": rf["binding"], "binding_frac": rf["binding_frac"]})
    # float64 uniform and normal fills (4 GiB each), measured beside the step:
    # not part of the configured workload, so not in `value`;
    # and the 13-round Threefry variants (4 GiB each)
    extra = []
    if not args.only:
        cases = [(g, 3) for g in range(10)] + [(g, 4) for g in range(10)] + \
            [(g, d) for g in (5, 6, 7, 8, 9) for d in range(3)]
        for g, d in cases:
            ns = n // 2 if d in (3, 4) else n
            sg = key32(g, seed)
            ms = _time_events(stream, lambda: orng.orng_fill(g, d, sg, 0, 0, ns, out, stream), 3)
            rf = roofs(g, d, ns, ms)
            gbs = 4.0 * n / (ms * 1e-3) / 1e9
            extra.append({"gen": inputs.GEN_NAMES[g], "dist": inputs.DIST_NAMES[d],
                          "ms": round(ms, 4), "gsamples_s": round(ns / (ms * 1e-3) / 1e9, 2),
                          "write_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                          "valu_frac": rf["valu_frac"], "binding": rf["binding"],
                          "binding_frac": rf["binding_frac"]})
        # integers in [lo, hi), 2^30 int32 samples each
        for g in range(10):
            sg = key32(g, seed)
            ms = _time_events(stream, lambda: orng.orng_fill_range(
                g, sg, 0, 1, 0, n, RANGE_LO, RANGE_HI, out, stream), 3)
            rf = roofs(g, "range", n, ms)
            gbs = 4.0 * n / (ms * 1e-3) / 1e9
            extra.append({"gen": inputs.GEN_NAMES[g], "dist": "i32_range",
                          "ms": round(ms, 4), "gsamples_s": round(n / (ms * 1e-3) / 1e9, 2),
                          "write_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                          "valu_frac": rf["valu_frac"], "binding": rf["binding"],
                          "binding_frac": rf["binding_frac"]})
    # the dominant (longest) kernel of the step, against its binding roof
    dom = max(range(len(combos)), key=lambda k: per_kernel_ms[k])
    dk = kernels[dom]
    drf = roofs(*combos[dom], n, per_kernel_ms[dom])
    common = {"traffic": traffic_bytes(*combos[dom]),
              "kernel": "%s/%s" % (dk["gen"], dk["dist"]), "algorithmic_bytes": 4 * n,
              "algorithmic_valu_slots": round(drf["slots"]),
              "hbm": {"achieved": dk["write_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": dk["hbm_frac"]}}
    if drf["binding"] == "alu":
        roofline = {"bound": "alu", "achieved": drf["valu_tslots_s"], "peak": VALU_PEAK_TSLOTS,
                    "unit": "Tslots/s", "frac": drf["valu_frac"], **common}
    else:
        roofline = {"bound": "hbm", "achieved": dk["write_gbs"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": dk["hbm_frac"], **common}
    total_ms = sum(per_kernel_ms)
    step_hbm_frac = (4.0 * n * len(combos) / (total_ms * 1e-3) / 1e9) / HBM_PEAK_GBS

    result = {
        "metric": "GSamples/s + % HBM write BW (fill), steps/s (walk); batched/served vs plain",
        "value": round(value, 3), "unit": "GSamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32,f32", "data": "synthetic",
        "config": {"workload": "bulk fill: 5 generators x {u32, f32 uniform, f32 normal}, "
                               "2^30 samples each, single stream (seed PCG64(231019925), ctr 0)",
                   "samples_per_fill": n, "fills_per_step": len(combos),
                   "parallelism": "single GPU"},
        "hbm_write_frac_step": round(step_hbm_frac, 4),
        "store_ceiling_gbs": round(ceiling_gbs, 1),
        "roofline": roofline,
        "kernels": kernels,
    }
    if extra:
        result["extra_kernels"] = extra
    del out
    torch.cuda.empty_cache()

    if not args.no_walk:
        w = dict(inputs.WALK)
        if args.walk_steps:
            w["n_steps"], w["msd_every"] = args.walk_steps, max(1, args.walk_steps // 10)
        pos = torch.zeros((w["dim"], w["n_particles"]), dtype=torch.float32, device=dev)
        msd = torch.zeros(w["n_steps"] // w["msd_every"], dtype=torch.float64, device=dev)
        orng.orng_brownian(seed, 0, w["n_particles"], w["dim"], 0, 100, w["dt"], w["D"], pos,
                           None, 0, stream)  # warm-up launch
        pos.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        orng.orng_brownian(seed, 0, w["n_particles"], w["dim"], 0, w["n_steps"], w["dt"], w["D"],
                           pos, msd, w["msd_every"], stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        m = (msd.cpu().numpy() / w["n_particles"]).tolist()
        ps = w["n_steps"] * w["n_particles"]
        wslots = WALK_SLOTS_PER_DIM * w["dim"] * ps
        result["walk"] = {"steps_per_s": round(w["n_steps"] / (ms * 1e-3), 1),
                          "valu_tslots_s": round(wslots / (ms * 1e-3) / 1e12, 2),
                          "valu_frac": round(wslots / (ms * 1e-3) / 1e12 / VALU_PEAK_TSLOTS, 4),
                          "particle_steps_per_s": round(w["n_steps"] * w["n_particles"]
                                                        / (ms * 1e-3), 1),
                          "ms": round(ms, 3), "n_particles": w["n_particles"], "dim": w["dim"],
                          "n_steps": w["n_steps"],
                          "msd_last": round(m[-1], 5),
                          "msd_expected_last": 2 * w["dim"] * w["D"] * w["n_steps"] * w["dt"]}
        del pos, msd

    if not args.no_bd2:
        result["bd2"] = bench_bd2(orng, inputs, stream, dev, not args.bd2_fused_only)

    if not args.no_plain:
        result["plain_multi"] = bench_plain_multi(orng, inputs, stream, dev)

    if not args.no_particles:
        result["particle_streams"] = bench_particles(orng, inputs, stream, dev)

    if not args.no_batched:
        result["batched"] = bench_batched(orng, inputs, stream, dev)

    if not args.no_serve:
        rates = {(g, d): k["gsamples_s"] for (g, d), k in zip(combos, kernels)}
        result["served"] = bench_serve(orng, inputs, stream, dev,
                                       rates if len(rates) == 15 else None)

    if not args.no_cpu:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(seed)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
