"""Host-side logic of liborng that runs without a GPU: argument validation of
every entry point (errors are returned before any device work), the
launch-knob checks and the launch-table file loader."""
import ctypes as C
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_19925_amd", "liborng.so")
EINVAL, ERANGE, ENOMEM, ENOENT = -1, -2, -3, -7


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("liborng.so not built")
    lib = C.CDLL(LIB)
    u32, u64, i32, vp, f32 = C.c_uint32, C.c_uint64, C.c_int, C.c_void_p, C.c_float
    lib.orng_fill.argtypes = [i32, i32, u64, u32, u64, u64, vp, vp]
    lib.orng_fill_multi.argtypes = [i32, i32, u64, u32, u32, u64, u64, vp, vp]
    lib.orng_brownian.argtypes = [u64, u32, u32, u32, u64, u32, f32, f32, vp, vp, u32, vp]
    lib.orng_normal_pairs.argtypes = [vp, vp, u64, vp, vp, vp]
    lib.orng_bd2.argtypes = [u64, u32, u32, u32, C.c_double, C.c_double, vp, vp, vp, vp, u32, vp]
    lib.orng_particle_streams.argtypes = [i32, u64, u32, u32, u32, u32, vp, vp]
    lib.orng_fill_range.argtypes = [i32, u64, u32, u32, u64, u64, C.c_int32, C.c_int32, vp, vp]
    lib.orng_fill_batched.argtypes = [vp, C.c_size_t, vp]
    lib.orng_fill_each.argtypes = [vp, C.c_size_t, vp]
    lib.orng_tune_load.argtypes = [C.c_char_p]
    lib.orng_autotune.argtypes = [i32, i32, C.c_char_p]
    lib.orng_serve_create.argtypes = [vp, C.POINTER(vp)]
    return lib


FAKE = 0x10000  # a non-null, 16-byte aligned address that is never dereferenced


def test_fill_validation(L):
    assert L.orng_fill(-1, 0, 1, 1, 0, 4, FAKE, None) == EINVAL
    assert L.orng_fill(0, 5, 1, 1, 0, 4, FAKE, None) == EINVAL
    # float64 uniform: samples end at 2^31, 8-byte alignment
    assert L.orng_fill(0, 3, 1, 1, 2**31 - 3, 4, FAKE, None) == ERANGE
    assert L.orng_fill(0, 3, 1, 1, 2**31 + 1, 0, FAKE, None) == ERANGE
    assert L.orng_fill(0, 3, 1, 1, 0, 4, FAKE + 4, None) == EINVAL
    assert L.orng_fill(0, 3, 1, 1, 2**31, 0, None, None) == 0
    assert L.orng_fill(0, 0, 1, 1, 2**32 - 3, 4, FAKE, None) == ERANGE
    assert L.orng_fill(0, 0, 1, 1, 2**32 + 1, 0, FAKE, None) == ERANGE
    assert L.orng_fill(0, 0, 1, 1, 0, 4, FAKE + 2, None) == EINVAL
    assert L.orng_fill(0, 0, 1, 1, 0, 4, None, None) == EINVAL
    assert L.orng_fill(9, 0, 2**32, 1, 0, 4, FAKE, None) == EINVAL   # Philox2x32: 32-bit key
    assert L.orng_fill(0, 0, 1, 1, 2**32, 0, None, None) == 0


def test_fill_multi_validation(L):
    assert L.orng_fill_multi(0, 0, 1, 2**32 - 2, 3, 0, 4, FAKE, None) == ERANGE
    assert L.orng_fill_multi(0, 0, 1, 2**32 - 3, 3, 2**32 - 1, 2, FAKE, None) == ERANGE
    assert L.orng_fill_multi(0, 0, 1, 0, 0, 0, 4, None, None) == 0
    assert L.orng_fill_multi(0, 0, 1, 0, 5, 0, 0, None, None) == 0
    assert L.orng_fill_multi(10, 0, 1, 0, 5, 0, 4, FAKE, None) == EINVAL
    assert L.orng_fill_multi(9, 0, 2**32, 0, 5, 0, 4, FAKE, None) == EINVAL  # 32-bit key
    assert L.orng_fill_multi(0, 3, 1, 0, 2, 2**31 - 1, 2, FAKE, None) == ERANGE
    assert L.orng_fill_multi(0, 3, 1, 0, 2, 0, 2, FAKE + 4, None) == EINVAL


def test_brownian_validation(L):
    assert L.orng_brownian(1, 0, 4, 0, 0, 1, 1e-3, 1.0, FAKE, None, 0, None) == EINVAL
    assert L.orng_brownian(1, 0, 4, 4, 0, 1, 1e-3, 1.0, FAKE, None, 0, None) == EINVAL
    assert L.orng_brownian(1, 0, 4, 3, 0, 1, 1e-3, -1.0, FAKE, None, 0, None) == EINVAL
    assert L.orng_brownian(1, 0, 4, 3, 0, 1, float("nan"), 1.0, FAKE, None, 0, None) == EINVAL
    assert L.orng_brownian(1, 0, 4, 3, 2**32 // 3, 2, 1e-3, 1.0, FAKE, None, 0, None) == ERANGE
    assert L.orng_brownian(1, 2**32 - 2, 4, 3, 0, 2, 1e-3, 1.0, FAKE, None, 0, None) == ERANGE
    assert L.orng_brownian(1, 0, 4, 3, 0, 1, 1e-3, 1.0, None, None, 0, None) == EINVAL
    assert L.orng_brownian(1, 0, 4, 3, 0, 1, 1e-3, 1.0, FAKE, FAKE + 4, 1, None) == EINVAL
    assert L.orng_brownian(1, 0, 0, 3, 0, 1, 1e-3, 1.0, None, None, 0, None) == 0


def test_bd2_validation(L):
    F = (FAKE, FAKE + 64, FAKE + 128, FAKE + 192)
    assert L.orng_bd2(1, 4, 2**32 - 1, 2, 1e-3, 1.0, *F, 0, None) == ERANGE
    assert L.orng_bd2(2**64 - 2, 4, 1, 1, 1e-3, 1.0, *F, 0, None) == ERANGE
    assert L.orng_bd2(1, 4, 1, 1, -1e-3, 1.0, *F, 0, None) == EINVAL
    assert L.orng_bd2(1, 4, 1, 1, float("inf"), 1.0, *F, 0, None) == EINVAL
    assert L.orng_bd2(1, 4, 1, 1, 1e-3, float("nan"), *F, 0, None) == EINVAL
    assert L.orng_bd2(1, 4, 1, 1, 1e-3, 1.0, FAKE, None, FAKE, FAKE, 0, None) == EINVAL
    assert L.orng_bd2(1, 4, 1, 1, 1e-3, 1.0, FAKE, FAKE + 4, FAKE, FAKE, 0, None) == EINVAL
    # nothing to do: no pointer is looked at
    assert L.orng_bd2(1, 0, 1, 5, 1e-3, 1.0, None, None, None, None, 0, None) == 0
    assert L.orng_bd2(1, 4, 1, 0, 1e-3, 1.0, None, None, None, None, 0, None) == 0


def test_particle_streams_validation(L):
    assert L.orng_particle_streams(10, 0, 10, 3, 0, 1, FAKE, None) == EINVAL
    assert L.orng_particle_streams(9, 2**32 - 9, 10, 3, 0, 1, FAKE, None) == ERANGE
    assert L.orng_particle_streams(0, 0, 10, 0, 0, 1, FAKE, None) == EINVAL
    assert L.orng_particle_streams(0, 0, 10, 17, 0, 1, FAKE, None) == EINVAL
    assert L.orng_particle_streams(0, 0, 10, 3, 2**32 - 1, 2, FAKE, None) == ERANGE
    assert L.orng_particle_streams(0, 2**64 - 5, 10, 3, 0, 1, FAKE, None) == ERANGE
    assert L.orng_particle_streams(0, 0, 10, 3, 0, 1, None, None) == EINVAL
    assert L.orng_particle_streams(0, 0, 10, 3, 0, 1, FAKE + 2, None) == EINVAL
    assert L.orng_particle_streams(0, 0, 0, 3, 0, 1, None, None) == 0
    assert L.orng_particle_streams(0, 0, 10, 3, 0, 0, None, None) == 0


def test_normal_pairs_validation(L):
    assert L.orng_normal_pairs(FAKE, None, 4, FAKE, FAKE, None) == EINVAL
    assert L.orng_normal_pairs(FAKE, FAKE + 1, 4, FAKE, FAKE, None) == EINVAL
    assert L.orng_normal_pairs(None, None, 0, None, None, None) == 0


def _reqs(rows):
    """orng_req_t records (56 bytes, the header's field order) from rows
    (gen, dist, offset, n, out, flags[, lo, hi])."""
    dt = np.dtype([("seed", "<u8"), ("offset", "<u8"), ("n", "<u8"), ("out", "<u8"),
                   ("ctr", "<u4"), ("gen", "<u4"), ("dist", "<u4"), ("flags", "<u4"),
                   ("lo", "<i4"), ("hi", "<i4")])
    assert dt.itemsize == 56
    r = np.zeros(len(rows), dt)
    for i, row in enumerate(rows):
        gen, dist, off, n, out, flags = row[:6]
        lo, hi = row[6:] if len(row) > 6 else (0, 0)
        r[i] = (1, off, n, out, 2, gen, dist, flags, lo, hi)
    return r


@pytest.mark.parametrize("fn", ["orng_fill_batched", "orng_fill_each"])
def test_batched_validation_rejects_whole_batch(L, fn):
    f = getattr(L, fn)
    cases = [
        ([(0, 0, 0, 16, FAKE, 0), (10, 0, 0, 16, FAKE, 0)], EINVAL),    # bad generator
        ([(0, 6, 0, 16, FAKE, 0)], EINVAL),                              # bad distribution
        ([(0, 5, 0, 16, FAKE, 0, 7, 7)], EINVAL),                        # range, lo == hi
        ([(0, 5, 0, 16, FAKE, 0, 8, -8)], EINVAL),                       # range, lo > hi
        ([(0, 5, 2**31 - 8, 16, FAKE, 0, 0, 9)], ERANGE),                # range past 2^31
        ([(0, 5, 0, 16, FAKE + 2, 0, 0, 9)], EINVAL),                    # range, misaligned
        ([(9, 5, 0, 16, FAKE, 0, -2**31, 2**31 - 1), (9, 5, 0, 16, FAKE, 0, 0, 0)], EINVAL),
        ([(0, 0, 0, 16, FAKE, 1)], EINVAL),                              # reserved flags
        ([(0, 0, 2**32 - 8, 16, FAKE, 0)], ERANGE),                      # past the period
        ([(0, 0, 0, 16, 0, 0)], EINVAL),                                 # NULL output
        ([(0, 0, 0, 16, FAKE + 2, 0)], EINVAL),                          # misaligned output
        ([(0, 3, 2**31 - 8, 16, FAKE, 0)], ERANGE),                      # float64 past 2^31
        ([(0, 3, 0, 16, FAKE + 4, 0)], EINVAL),                          # float64, 4-byte aligned
    ]
    for rows, want in cases:
        r = _reqs(rows)
        assert f(r.ctypes.data, r.size, None) == want, rows
    empty = _reqs([(0, 0, 0, 0, 0, 0)])
    assert f(empty.ctypes.data, 1, None) == 0  # nothing to do
    assert f(None, 0, None) == 0
    assert f(None, 3, None) == EINVAL


@pytest.mark.parametrize("fn", ["orng_fill_batched", "orng_fill_each", "orng_fill_batched_noalloc"])
def test_batched_rejects_a_64_bit_philox2x32_seed(L, fn):
    f = getattr(L, fn)
    f.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p]
    r = _reqs([(0, 0, 0, 16, FAKE, 0), (9, 0, 0, 16, FAKE, 0)])
    r[1]["seed"] = 2**32
    assert f(r.ctypes.data, r.size, None) == EINVAL


@pytest.mark.parametrize("fn", ["orng_fill_batched", "orng_fill_each"])
def test_batched_validation_reports_the_first_bad_request(L, fn):
    """Large lists are validated in parallel ranges; the status returned is
    still that of the first bad request in list order."""
    f = getattr(L, fn)
    rows = [(0, 0, 0, 16, FAKE, 0)] * 20000
    for first, second, want in [((15000, 9), (19000, 2**32 - 8), EINVAL),
                                ((3000, 2**32 - 8), (17000, 9), ERANGE)]:
        r = _reqs(rows)
        for (i, what) in (first, second):
            if what == 9:
                r[i]["gen"] = 10
            else:
                r[i]["offset"] = what
        assert f(r.ctypes.data, r.size, None) == want


def test_launch_knob_validation(L):
    class cfg_t(C.Structure):
        _fields_ = [("wg_size", C.c_uint32), ("unroll", C.c_uint32), ("max_wgs", C.c_uint32),
                    ("nontemporal", C.c_uint32)]
    L.orng_set_launch.argtypes = [C.POINTER(cfg_t)]
    L.orng_get_launch.argtypes = [C.POINTER(cfg_t)]
    assert L.orng_set_launch(C.byref(cfg_t(100, 0, 0, 0))) == EINVAL
    assert L.orng_set_launch(C.byref(cfg_t(1024, 0, 0, 0))) == EINVAL
    assert L.orng_set_launch(C.byref(cfg_t(64, 65, 0, 0))) == EINVAL
    assert L.orng_set_launch(C.byref(cfg_t(64, 2, 0, 3))) == EINVAL
    assert L.orng_set_launch(C.byref(cfg_t(128, 2, 7, 1))) == 0
    got = cfg_t()
    assert L.orng_get_launch(C.byref(got)) == 0
    assert (got.wg_size, got.unroll, got.max_wgs, got.nontemporal) == (128, 2, 7, 1)
    assert L.orng_set_launch(None) == 0
    assert L.orng_get_launch(C.byref(got)) == 0 and got.wg_size == 0
    assert L.orng_get_launch(None) == EINVAL


def test_tune_table_loader(L, tmp_path):
    assert L.orng_tune_load(str(tmp_path / "missing.txt").encode()) == ENOENT
    bad = tmp_path / "bad.txt"
    bad.write_text("# header\n0 0 100 4 0 1 256 4 1 0\n10 0 256 4 0 1 256 4 1 0\nnot numbers\n")
    assert L.orng_tune_load(str(bad).encode()) == EINVAL  # no valid line
    good = tmp_path / "good.txt"
    good.write_text("# header\n0 0 256 2 0 2 256 4 1 0\n4 1 256 64 0 2 256 1 1 0\n")
    assert L.orng_tune_load(str(good).encode()) == 0
    assert L.orng_autotune(10, 0, None) == EINVAL
    assert L.orng_autotune(0, 6, None) == EINVAL  # 5 is the integer-range fill
    rng_line = tmp_path / "range.txt"
    rng_line.write_text("# header\n3 5 128 8 0 2 0 0 0 0\n")  # an integer-range row
    assert L.orng_tune_load(str(rng_line).encode()) == 0
    rng_line.write_text("# header\n3 5 100 8 0 2 0 0 0 0\n")  # not a workgroup size
    assert L.orng_tune_load(str(rng_line).encode()) == EINVAL


def test_serve_create_validation(L):
    class cfg_t(C.Structure):
        _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64),
                    ("max_slots", C.c_uint32), ("flags", C.c_uint32),
                    ("step_words", C.c_uint64)]
    h = C.c_void_p()
    assert L.orng_serve_create(None, C.byref(h)) == EINVAL
    assert L.orng_serve_create(C.cast(C.pointer(cfg_t(None, 0, 0, 0, 0)), C.c_void_p),
                               C.byref(h)) == EINVAL
    assert L.orng_serve_create(C.cast(C.pointer(cfg_t(None, 1 << 20, 0, 1, 0)), C.c_void_p),
                               C.byref(h)) == EINVAL
    assert L.orng_serve_create(C.cast(C.pointer(cfg_t(FAKE + 8, 1 << 20, 0, 0, 0)), C.c_void_p),
                               C.byref(h)) == EINVAL
    # a step of more than 2^34 words
    assert L.orng_serve_create(C.cast(C.pointer(cfg_t(None, 1 << 20, 0, 0, 2**34 + 1)),
                                      C.c_void_p), C.byref(h)) == EINVAL


def test_fill_range_validation(L):
    assert L.orng_fill_range(10, 0, 0, 1, 0, 4, 0, 10, FAKE, None) == EINVAL
    assert L.orng_fill_range(9, 2**32, 0, 1, 0, 4, 0, 10, FAKE, None) == EINVAL
    assert L.orng_fill_range(-1, 0, 0, 1, 0, 4, 0, 10, FAKE, None) == EINVAL
    assert L.orng_fill_range(0, 0, 0, 1, 0, 4, 10, 10, FAKE, None) == EINVAL
    assert L.orng_fill_range(0, 0, 0, 1, 0, 4, 11, 10, FAKE, None) == EINVAL
    assert L.orng_fill_range(0, 0, 0, 1, 2**31 - 3, 4, 0, 10, FAKE, None) == ERANGE
    assert L.orng_fill_range(0, 0, 0, 1, 2**31 + 1, 0, 0, 10, FAKE, None) == ERANGE
    assert L.orng_fill_range(0, 0, 2**32 - 2, 3, 0, 4, 0, 10, FAKE, None) == ERANGE
    assert L.orng_fill_range(0, 0, 0, 1, 0, 4, 0, 10, None, None) == EINVAL
    assert L.orng_fill_range(0, 0, 0, 1, 0, 4, 0, 10, FAKE + 2, None) == EINVAL
    # nothing to do: no pointer is looked at
    assert L.orng_fill_range(0, 0, 0, 0, 0, 4, 0, 10, None, None) == 0
    assert L.orng_fill_range(0, 0, 0, 1, 2**31, 0, 0, 10, None, None) == 0
