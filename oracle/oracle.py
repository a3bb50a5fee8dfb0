"""ctypes wrapper of the C++ oracle -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It loads ``liborng_oracle.so`` (built from
``orng_oracle.cc`` by :func:`build`) and returns numpy arrays.  It never
imports the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orng_oracle.cc")
LIB = os.path.join(HERE, "liborng_oracle.so")

(PHILOX, THREEFRY4X32, THREEFRY2X64, SQUARES, TYCHE, THREEFRY4X32_13, THREEFRY2X64_13, TYCHE_I,
 SQUARES64, PHILOX2X32) = range(10)
U32, F32_UNIFORM, F32_NORMAL, F64_UNIFORM, F64_NORMAL = range(5)
GENS = (PHILOX, THREEFRY4X32, THREEFRY2X64, SQUARES, TYCHE)
DISTS = (U32, F32_UNIFORM, F32_NORMAL)  # the float32/u32 set; F64_UNIFORM is separate

# contraction off: each float operation in the source is one IEEE operation
CXXFLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-pthread"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ into ``oracle/liborng_oracle.so``."""
    srcs = [SRC, os.path.join(os.path.dirname(SRC), "orng_oracle.h")]
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(f) for f in srcs):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["g++", *CXXFLAGS, SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _bind(L):
    """Declare the C signatures of the oracle library L."""
    if True:
        u32, u64, i32, vp, f32 = C.c_uint32, C.c_uint64, C.c_int, C.c_void_p, C.c_float
        P32, P64 = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        sig = {
            "oracle_philox4x32_10": (None, [P32, P32, P32]),
            "oracle_philox2x32_10": (None, [P32, u32, P32]),
            "oracle_threefry4x32_20": (None, [P32, P32, P32]),
            "oracle_threefry2x64_20": (None, [P64, P64, P64]),
            "oracle_threefry4x32_13": (None, [P32, P32, P32]),
            "oracle_threefry2x64_13": (None, [P64, P64, P64]),
            "oracle_squares32": (u32, [u64, u64]),
            "oracle_squares_key": (u64, [u64]),
            "oracle_tyche_mix": (None, [P32]),
            "oracle_tyche_init": (None, [u64, u32, u32, P32]),
            "oracle_tyche_next": (u32, [P32]),
            "oracle_tyche_mix_i": (None, [P32]),
            "oracle_tyche_i_init": (None, [u64, u32, u32, P32]),
            "oracle_tyche_i_next": (u32, [P32]),
            "oracle_squares64": (u64, [u64, u64]),
            "oracle_word": (u32, [i32, u64, u32, u64]),
            "oracle_sample": (None, [i32, i32, u64, u32, u64, vp]),
            "oracle_u01": (f32, [u32]),
            "oracle_ln_u1": (f32, [u32]),
            "oracle_sincos2pi": (None, [u32, C.POINTER(f32), C.POINTER(f32)]),
            "oracle_normal_pair": (None, [u32, u32, C.POINTER(f32)]),
            "oracle_u01_n": (None, [vp, u64, vp]),
            "oracle_ln_u1_n": (None, [vp, u64, vp]),
            "oracle_sincos2pi_n": (None, [vp, u64, vp, vp]),
            "oracle_normal_pair_n": (None, [vp, vp, u64, vp, vp]),
            "oracle_fill": (i32, [i32, i32, u64, u32, u64, u64, vp, i32]),
            "oracle_fill_multi": (i32, [i32, i32, u64, u32, u32, u64, u64, vp, i32]),
            "oracle_samples_at": (None, [i32, i32, u64, vp, vp, u64, vp, i32]),
            "oracle_walk_sigma": (f32, [f32, f32]),
            "oracle_brownian": (i32, [u64, u32, vp, u32, u32, u64, u32, f32, f32, vp, vp, u32,
                                      i32]),
            "oracle_u01_f64": (C.c_double, [u32, u32]),
            "oracle_particle_streams": (i32, [i32, u64, u32, u32, u32, u32, vp, i32]),
            "oracle_ln_u1_f64": (C.c_double, [u64]),
            "oracle_sincos_turn_f64": (None, [u64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
            "oracle_normal_pair_f64": (None, [u32, u32, u32, u32, C.POINTER(C.c_double)]),
            "oracle_ln_u1_f64_n": (None, [vp, u64, vp]),
            "oracle_sincos_turn_f64_n": (None, [vp, u64, vp, vp]),
            "oracle_range_i32": (C.c_int32, [u32, u32, C.c_int32, C.c_int32]),
            "oracle_fill_range": (i32, [i32, u64, u32, u32, u64, u64, C.c_int32, C.c_int32, vp,
                                        i32]),
            "oracle_bd2": (i32, [u64, vp, u32, u32, u32, C.c_double, C.c_double, vp, vp, vp, vp,
                                 i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
    return L


def lib():
    global _lib
    if _lib is None:
        build(force=False)  # rebuilds when the sources are newer than the library
        _lib = _bind(C.CDLL(LIB))
    return _lib


NATIVE_FLAGS = ["-O3", "-march=native"]
_native = None


def lib_native():
    """The same oracle source built for the host it runs on (-O3
    -march=native, contraction still off, no fast-math), into a temporary
    directory, for timing the oracle as a CPU baseline.  Every result is the
    same as lib()'s: each float expression stays one IEEE operation."""
    global _native
    if _native is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="orng_oracle_native_")
        path = os.path.join(d, "liborng_oracle_native.so")
        flags = [f for f in CXXFLAGS if not f.startswith("-O")] + NATIVE_FLAGS
        subprocess.run(["g++", *flags, SRC, "-o", path], check=True)
        _native = _bind(C.CDLL(path))
    return _native




def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def _arr32(vals):
    return (C.c_uint32 * len(vals))(*[int(v) & 0xFFFFFFFF for v in vals])


def philox4x32_10(ctr, key):
    out = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(_arr32(ctr), _arr32(key), out)
    return list(out)


def philox2x32_10(ctr, key):
    out = (C.c_uint32 * 2)()
    lib().oracle_philox2x32_10(_arr32(ctr), int(key) & 0xFFFFFFFF, out)
    return list(out)


def threefry4x32_20(ctr, key):
    out = (C.c_uint32 * 4)()
    lib().oracle_threefry4x32_20(_arr32(ctr), _arr32(key), out)
    return list(out)


def threefry2x64_20(ctr, key):
    out = (C.c_uint64 * 2)()
    c = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    lib().oracle_threefry2x64_20(c, k, out)
    return list(out)


def threefry2x64_13(ctr, key):
    out = (C.c_uint64 * 2)()
    c = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    lib().oracle_threefry2x64_13(c, k, out)
    return list(out)


def threefry4x32_13(ctr, key):
    out = (C.c_uint32 * 4)()
    lib().oracle_threefry4x32_13(_arr32(ctr), _arr32(key), out)
    return list(out)


def squares32(ctr, key):
    return lib().oracle_squares32(ctr, key)


def squares_key(seed):
    return lib().oracle_squares_key(seed)


def tyche_mix(state):
    st = _arr32(state)
    lib().oracle_tyche_mix(st)
    return list(st)


def tyche_init(seed, c_xor, d_xor):
    st = (C.c_uint32 * 4)()
    lib().oracle_tyche_init(seed, c_xor, d_xor, st)
    return list(st)


def tyche_stream(seed, c_xor, d_xor, count):
    st = (C.c_uint32 * 4)()
    lib().oracle_tyche_init(seed, c_xor, d_xor, st)
    return [lib().oracle_tyche_next(st) for _ in range(count)]


def word(gen, seed, ctr, p):
    return lib().oracle_word(gen, seed, ctr, p)


def u01(x):
    return lib().oracle_u01(x)


def ln_u1(k):
    return lib().oracle_ln_u1(k)


def sincos2pi(k):
    c, s = C.c_float(), C.c_float()
    lib().oracle_sincos2pi(k, C.byref(c), C.byref(s))
    return c.value, s.value


def normal_pair(x0, x1):
    out = (C.c_float * 2)()
    lib().oracle_normal_pair(x0, x1, out)
    return out[0], out[1]


def u01_n(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    out = np.empty(x.shape, np.float32)
    lib().oracle_u01_n(x.ctypes.data, x.size, out.ctypes.data)
    return out


def ln_u1_n(k):
    k = np.ascontiguousarray(k, dtype=np.uint32)
    out = np.empty(k.shape, np.float32)
    lib().oracle_ln_u1_n(k.ctypes.data, k.size, out.ctypes.data)
    return out


def sincos2pi_n(k):
    k = np.ascontiguousarray(k, dtype=np.uint32)
    c = np.empty(k.shape, np.float32)
    s = np.empty(k.shape, np.float32)
    lib().oracle_sincos2pi_n(k.ctypes.data, k.size, c.ctypes.data, s.ctypes.data)
    return c, s


def normal_pair_n(x0, x1):
    x0 = np.ascontiguousarray(x0, dtype=np.uint32)
    x1 = np.ascontiguousarray(x1, dtype=np.uint32)
    z0 = np.empty(x0.shape, np.float32)
    z1 = np.empty(x0.shape, np.float32)
    lib().oracle_normal_pair_n(x0.ctypes.data, x1.ctypes.data, x0.size, z0.ctypes.data,
                               z1.ctypes.data)
    return z0, z1


def _dtype(dist):
    return {U32: np.uint32, F64_UNIFORM: np.float64, F64_NORMAL: np.float64}.get(dist, np.float32)


def fill(gen, dist, seed, ctr, offset, n, nthreads=None):
    out = np.empty(n, dtype=_dtype(dist))
    rc = lib().oracle_fill(gen, dist, seed, ctr, offset, n, out.ctypes.data,
                           nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_fill rejected arguments (%d)" % rc)
    return out


def fill_multi(gen, dist, seed, ctr0, n_streams, offset, per_stream, nthreads=None):
    out = np.empty(n_streams * per_stream, dtype=_dtype(dist))
    rc = lib().oracle_fill_multi(gen, dist, seed, ctr0, n_streams, offset, per_stream,
                                 out.ctypes.data, nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_fill_multi rejected arguments (%d)" % rc)
    return out


def samples_at(gen, dist, seed, ctrs, pos, nthreads=None):
    ctrs = np.ascontiguousarray(ctrs, dtype=np.uint32)
    pos = np.ascontiguousarray(pos, dtype=np.uint64)
    assert ctrs.shape == pos.shape
    out = np.empty(pos.shape, dtype=_dtype(dist))
    lib().oracle_samples_at(gen, dist, seed, ctrs.ctypes.data, pos.ctypes.data, pos.size,
                            out.ctypes.data, nthreads or default_threads())
    return out


def walk_sigma(dt, D):
    return lib().oracle_walk_sigma(dt, D)


def brownian(seed, ctr0, n_particles=None, ids=None, dim=3, step0=0, n_steps=1, dt=1e-3, D=1.0,
             pos=None, msd_every=0, nthreads=None):
    """Returns (pos [dim][count] float32, msd float64 sums or None)."""
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        count = ids.size
    else:
        count = n_particles
    if pos is None:
        pos = np.zeros((dim, count), dtype=np.float32)
    else:
        pos = np.ascontiguousarray(pos, dtype=np.float32).copy()
    nsnap = n_steps // msd_every if msd_every else 0
    msd = np.zeros(nsnap, dtype=np.float64) if nsnap else None
    rc = lib().oracle_brownian(seed, ctr0, ids.ctypes.data if ids is not None else None, count,
                               dim, step0, n_steps, dt, D, pos.ctypes.data,
                               msd.ctypes.data if msd is not None else None, msd_every,
                               nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_brownian rejected arguments (%d)" % rc)
    return pos, msd


def u01_f64(w0, w1):
    return lib().oracle_u01_f64(int(w0) & 0xFFFFFFFF, int(w1) & 0xFFFFFFFF)


def bd2(pid0, n_particles=None, ids=None, step0=1, n_steps=1, dt=1e-3, c=1.0, state=None,
        nthreads=None):
    """The paper's 2-D Brownian dynamics example.  state: (x, y, vx, vy)
    float64 arrays of `count` entries (zeros when None).  Returns the updated
    copy as a (4, count) float64 array."""
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        count = ids.size
    else:
        count = n_particles
    st = np.zeros((4, count), np.float64) if state is None else \
        np.ascontiguousarray(np.asarray(state, np.float64).reshape(4, count)).copy()
    rc = lib().oracle_bd2(pid0, ids.ctypes.data if ids is not None else None, count, step0,
                          n_steps, dt, c, st[0].ctypes.data, st[1].ctypes.data,
                          st[2].ctypes.data, st[3].ctypes.data, nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_bd2 rejected arguments (%d)" % rc)
    return st


def particle_streams(gen, seed0, n_particles, draws, ctr0, n_iters, nthreads=None):
    """(n_iters * n_particles * draws) uint32 words of the concatenated
    per-particle micro-streams."""
    out = np.empty(n_iters * n_particles * draws, np.uint32)
    rc = lib().oracle_particle_streams(gen, seed0, n_particles, draws, ctr0, n_iters,
                                       out.ctypes.data, nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_particle_streams rejected arguments (%d)" % rc)
    return out


def range_i32(w0, w1, lo, hi):
    """Integer in [lo, hi) from the word pair (w0 at the even position)."""
    return lib().oracle_range_i32(int(w0) & 0xFFFFFFFF, int(w1) & 0xFFFFFFFF, lo, hi)


def fill_range(gen, seed, ctr0, n_streams, offset, per_stream, lo, hi, nthreads=None):
    """(n_streams * per_stream) int32: integer sample offset + j of stream
    (seed, ctr0 + i) at [i * per_stream + j]."""
    out = np.empty(n_streams * per_stream, np.int32)
    rc = lib().oracle_fill_range(gen, seed, ctr0, n_streams, offset, per_stream, lo, hi,
                                 out.ctypes.data, nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_fill_range rejected arguments (%d)" % rc)
    return out


def ln_u1_f64(K):
    return lib().oracle_ln_u1_f64(int(K))


def sincos_turn_f64(k):
    c, s = C.c_double(), C.c_double()
    lib().oracle_sincos_turn_f64(int(k), C.byref(c), C.byref(s))
    return c.value, s.value


def normal_pair_f64(w0, w1, w2, w3):
    out = (C.c_double * 2)()
    lib().oracle_normal_pair_f64(*(int(w) & 0xFFFFFFFF for w in (w0, w1, w2, w3)), out)
    return out[0], out[1]


def ln_u1_f64_n(K):
    K = np.ascontiguousarray(K, dtype=np.uint64)
    out = np.empty(K.shape, np.float64)
    lib().oracle_ln_u1_f64_n(K.ctypes.data, K.size, out.ctypes.data)
    return out


def sincos_turn_f64_n(k):
    k = np.ascontiguousarray(k, dtype=np.uint64)
    c = np.empty(k.shape, np.float64)
    s = np.empty(k.shape, np.float64)
    lib().oracle_sincos_turn_f64_n(k.ctypes.data, k.size, c.ctypes.data, s.ctypes.data)
    return c, s


def tyche_mix_i(state):
    st = _arr32(state)
    lib().oracle_tyche_mix_i(st)
    return list(st)


def tyche_i_init(seed, c_xor, d_xor):
    st = (C.c_uint32 * 4)()
    lib().oracle_tyche_i_init(seed, c_xor & 0xFFFFFFFF, d_xor & 0xFFFFFFFF, st)
    return list(st)


def tyche_i_stream(seed, c_xor, d_xor, count):
    st = (C.c_uint32 * 4)()
    lib().oracle_tyche_i_init(seed, c_xor & 0xFFFFFFFF, d_xor & 0xFFFFFFFF, st)
    return [lib().oracle_tyche_i_next(st) for _ in range(count)]


def squares64(ctr, key):
    return lib().oracle_squares64(ctr, key)
