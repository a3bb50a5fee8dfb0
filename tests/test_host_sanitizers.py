"""Host code under the address and undefined-behaviour sanitizers (g++
-fsanitize=address,undefined, every report fatal):

- the oracle: a driver runs each of its bulk entry points (every generator and
  distribution, multi-stream fills, integer ranges, micro-streams, the walk,
  the 2-D Brownian dynamics, the normal transform) with several threads; its
  outputs must equal those of the ordinary oracle build byte for byte;
- the server's arena allocator (host-only header): 200,000 random
  allocations and releases checked against a granule-map model (first fit,
  bounds, no overlap, used and peak bytes, coalescing back to one range);
- the request-record checks of the batched and served paths (host-only
  header): 200,000 requests drawn on and around every boundary, each
  compared with the documented rules (return code, integer-range bounds,
  output alignment class);
- the serving loop's scheduling rules (host-only header): request tiling
  over random ranges and step planning over random request sets admitted
  over time, checked against their stated properties until every tile is
  scheduled once.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _gxx():
    g = shutil.which("g++")
    if not g:
        pytest.skip("g++ not available")
    return g


def _build(tmp, name, sources, extra=()):
    exe = str(tmp / name)
    subprocess.run([_gxx(), "-std=c++17", "-O1", "-g", "-pthread", *SAN, *extra, *sources, "-o",
                    exe], check=True, capture_output=True)
    return exe


def _run(cmd):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers_matches_the_plain_build(O, tmp_path):
    exe = _build(tmp_path, "oracle_check", [os.path.join(HERE, "oracle_check.cc"),
                                            os.path.join(ROOT, "oracle", "orng_oracle.cc")],
                 extra=["-ffp-contract=off", "-fno-fast-math"])
    out = tmp_path / "out"
    out.mkdir()
    assert _run([exe, str(out)]).strip().endswith("OK")

    def got(name, dtype):
        return np.fromfile(str(out / (name + ".bin")), dtype=dtype)

    for g in range(10):
        seed = 0x89ABCDEF if g == 9 else 0x0123456789ABCDEF
        for d in range(5):
            ref = O.fill(g, d, seed, 7, 16380, 5001)
            assert np.array_equal(got("fill_%d_%d" % (g, d), ref.dtype).view(np.uint8),
                                  ref.view(np.uint8)), ("fill", g, d)
            ref = O.fill_multi(g, d, seed, 0xFFFFFFF0, 3, 5, 77)
            assert np.array_equal(got("multi_%d_%d" % (g, d), ref.dtype).view(np.uint8),
                                  ref.view(np.uint8)), ("multi", g, d)
        assert np.array_equal(got("range_%d" % g, np.int32),
                              O.fill_range(g, seed, 3, 2, 1, 1001, -1000, 999))
        assert np.array_equal(got("particles_%d" % g, np.uint32),
                              O.particle_streams(g, 100, 300, 3, 9, 5))
    pos, _ = O.brownian(0xABCDEF, 11, n_particles=500, dim=3, n_steps=40, dt=1e-3, D=1.0)
    assert np.array_equal(got("walk", np.float32).view(np.uint32), pos.ravel().view(np.uint32))
    st = O.bd2(5, 700, step0=1, n_steps=30, dt=1e-3, c=1.0)
    assert np.array_equal(got("bd2", np.float64).view(np.uint64), st.ravel().view(np.uint64))
    i = np.arange(4096, dtype=np.uint64)
    x0 = (i * 2654435761 & 0xFFFFFFFF).astype(np.uint32)
    x1 = ((i * 40503 + 7) & 0xFFFFFFFF).astype(np.uint32)
    z0, z1 = O.normal_pair_n(x0, x1)
    assert np.array_equal(got("normal_pairs_z0", np.float32).view(np.uint32), z0.view(np.uint32))
    assert np.array_equal(got("normal_pairs_z1", np.float32).view(np.uint32), z1.view(np.uint32))


def test_arena_allocator_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "arena_check", [os.path.join(HERE, "arena_check.cc")])
    assert _run([exe, "200000"]).strip() == "OK 200000 steps"


def _request_model(gen, dist, flags, seed, offset, n, addr, lo, hi):
    """The request checks the fill calls document: (return code, lo bits,
    hi - lo mod 2^32, output alignment class in words)."""
    OK, EINVAL, ERANGE = 0, -1, -2
    lo = lo - (1 << 32) if lo >= 1 << 31 else lo
    hi = hi - (1 << 32) if hi >= 1 << 31 else hi
    rng = dist == 5
    bounds = ((lo & 0xFFFFFFFF, (hi - lo) & 0xFFFFFFFF) if rng else (0, 0))
    if gen > 9 or dist > 5 or flags != 0:
        return (EINVAL,) + bounds + (0,)
    if gen == 9 and seed >= 1 << 32:        # Philox2x32-10: one 32-bit key word
        return (EINVAL,) + bounds + (0,)
    if rng and lo >= hi:
        return (EINVAL,) + bounds + (0,)
    words = 2 if dist >= 3 else 1           # float64 and integer ranges read word pairs
    limit = (1 << 32) // words
    if offset > limit or n > limit - offset:
        return (ERANGE,) + bounds + (0,)
    if n == 0:
        return (OK,) + bounds + (0,)
    size = 8 if dist in (3, 4) else 4
    if addr == 0 or addr % size:
        return (EINVAL,) + bounds + (0,)
    first = offset if rng else offset * words
    return (OK,) + bounds + ((addr // 4 - first) % 4,)


def test_request_checks_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "request_check", [os.path.join(HERE, "request_check.cc")])
    n = 200000
    out = tmp_path / "rows.bin"
    assert _run([exe, str(n), str(out)]).strip() == "OK %d requests" % n
    rows = np.fromfile(str(out), dtype=np.uint64).reshape(n, 13)
    codes, aligned = {}, [0] * 4
    for row in rows.tolist():
        gen, dist, flags, seed, _ctr, offset, cnt, addr, lo, hi, rc, lob, packed = row
        rc = rc - (1 << 64) if rc >= 1 << 63 else rc
        got = (rc, lob, packed >> 32, packed & 0xFFFFFFFF)
        want = _request_model(gen, dist, flags, seed, offset, cnt, addr, lo, hi)
        assert got == want, (row, got, want)
        codes[rc] = codes.get(rc, 0) + 1
        if rc == 0 and cnt > 0:
            aligned[got[3]] += 1
    # the draw reaches every outcome often, and every alignment class
    assert min(codes.get(c, 0) for c in (0, -1, -2)) > 5000, codes
    assert min(aligned) > 1000, aligned


def test_serve_scheduling_rules_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "serve_plan_check", [os.path.join(HERE, "serve_plan_check.cc")])
    out = _run([exe, "300"]).strip()
    assert out.startswith("OK 300 rounds"), out
    assert int(out.split()[3]) > 10000, out  # many steps were planned
