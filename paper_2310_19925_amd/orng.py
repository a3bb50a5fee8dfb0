"""Thin ctypes binding of liborng.so (include/orng.h).

Argument marshalling only: every call goes straight to the C entry point of the
same name, which enqueues HIP kernels on the given (or current) stream.  The
library must have been built (``python -m paper_2310_19925_amd.build`` or
``__graft_entry__.build()``); importing this module fails loudly otherwise --
there is no CPU fallback.  PyTorch is used only for device buffers and
streams.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborng.so")

PHILOX4X32_10, THREEFRY4X32_20, THREEFRY2X64_20, SQUARES32, TYCHE = range(5)
THREEFRY4X32_13, THREEFRY2X64_13, TYCHE_I, SQUARES64, PHILOX2X32 = 5, 6, 7, 8, 9
U32, F32_UNIFORM, F32_NORMAL, F64_UNIFORM, F64_NORMAL = range(5)
I32_RANGE = 5  # request records only (batched, served): integers in [lo, hi)
OK, EINVAL, ERANGE, ENOMEM, EAGAIN, EBUSY, EHIP, ENOENT = 0, -1, -2, -3, -4, -5, -6, -7
TUNE_RANGE = 5  # orng_autotune(gen, TUNE_RANGE): the integer-range fill


class OrngError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.orng_strerror(status).decode()
        if status == EHIP:
            msg += " (hip error %d)" % _lib.orng_last_hip_error()
        super().__init__("%s: %s [%d]" % (where, msg, status))


class orng_launch_t(C.Structure):
    _fields_ = [("wg_size", C.c_uint32), ("unroll", C.c_uint32), ("max_wgs", C.c_uint32),
                ("nontemporal", C.c_uint32)]


class orng_serve_cfg_t(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("max_slots", C.c_uint32),
                ("flags", C.c_uint32), ("step_words", C.c_uint64)]


class orng_result_t(C.Structure):
    _fields_ = [("d_out", C.c_void_p), ("n", C.c_uint64), ("t_submit_ns", C.c_int64),
                ("t_admit_ns", C.c_int64), ("t_done_ns", C.c_int64), ("status", C.c_int32),
                ("pad", C.c_int32)]


class orng_serve_stats_t(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("released", C.c_uint64), ("failed", C.c_uint64), ("samples_done", C.c_uint64),
                ("steps", C.c_uint64), ("arena_peak_bytes", C.c_uint64),
                ("active_peak", C.c_uint32), ("queued", C.c_uint32),
                ("latency_p50_ms", C.c_double), ("latency_p99_ms", C.c_double),
                ("latency_mean_ms", C.c_double), ("first_submit_to_last_done_s", C.c_double)]


class orng_req_t(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("offset", C.c_uint64), ("n", C.c_uint64),
                ("out", C.c_void_p), ("ctr", C.c_uint32), ("gen", C.c_uint32),
                ("dist", C.c_uint32), ("flags", C.c_uint32), ("lo", C.c_int32),
                ("hi", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liborng.so is not built (%s); run paper_2310_19925_amd/build.py"
                          % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    i32, u32, u64, vp, f32 = C.c_int, C.c_uint32, C.c_uint64, C.c_void_p, C.c_float
    sig = {
        "orng_fill": [i32, i32, u64, u32, u64, u64, vp, vp],
        "orng_fill_multi": [i32, i32, u64, u32, u32, u64, u64, vp, vp],
        "orng_brownian": [u64, u32, u32, u32, u64, u32, f32, f32, vp, vp, u32, vp],
        "orng_fill_range": [i32, u64, u32, u32, u64, u64, C.c_int32, C.c_int32, vp, vp],
        "orng_bd2": [u64, u32, u32, u32, C.c_double, C.c_double, vp, vp, vp, vp, u32, vp],
        "orng_particle_streams": [i32, u64, u32, u32, u32, u32, vp, vp],
        "orng_normal_pairs": [vp, vp, u64, vp, vp, vp],
        "orng_fill_batched": [vp, C.c_size_t, vp],
        "orng_fill_batched_noalloc": [vp, C.c_size_t, vp],
        "orng_fill_each": [vp, C.c_size_t, vp],
        "orng_autotune": [i32, i32, C.c_char_p],
        "orng_tune_load": [C.c_char_p],
        "orng_serve_create": [C.POINTER(orng_serve_cfg_t), C.POINTER(C.c_void_p)],
        "orng_serve_submit": [vp, C.POINTER(orng_req_t), C.POINTER(C.c_uint64)],
        "orng_serve_try_submit": [vp, C.POINTER(orng_req_t), C.POINTER(C.c_uint64)],
        "orng_serve_submit_many": [vp, vp, C.c_size_t, vp],
        "orng_serve_release_many": [vp, vp, C.c_size_t, C.c_int64, C.POINTER(C.c_size_t)],
        "orng_serve_poll": [vp, u64, C.POINTER(orng_result_t)],
        "orng_serve_wait": [vp, u64, C.c_int64, C.POINTER(orng_result_t)],
        "orng_serve_release": [vp, u64],
        "orng_serve_stats": [vp, C.POINTER(orng_serve_stats_t)],
        "orng_serve_destroy": [vp],
        "orng_set_launch": [C.POINTER(orng_launch_t)],
        "orng_get_launch": [C.POINTER(orng_launch_t)],
        "orng_last_hip_error": [],
        "orng_version": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = i32
    L.orng_strerror.argtypes = [i32]
    L.orng_strerror.restype = C.c_char_p
    return L


_lib = _load()


def lib():
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status, where):
    if status != OK:
        raise OrngError(status, where)


def orng_fill(gen, dist, seed, ctr, offset, n, out, stream=None):
    _check(_lib.orng_fill(gen, dist, seed, ctr, offset, n, _ptr(out), _stream(stream)),
           "orng_fill")


def orng_fill_multi(gen, dist, seed, ctr0, n_streams, offset, per_stream, out, stream=None):
    _check(_lib.orng_fill_multi(gen, dist, seed, ctr0, n_streams, offset, per_stream, _ptr(out),
                                _stream(stream)), "orng_fill_multi")


def orng_fill_range(gen, seed, ctr0, n_streams, offset, per_stream, lo, hi, out, stream=None):
    _check(_lib.orng_fill_range(gen, seed, ctr0, n_streams, offset, per_stream, lo, hi,
                                _ptr(out), _stream(stream)), "orng_fill_range")


def orng_brownian(seed, ctr0, n_particles, dim, step0, n_steps, dt, D, pos, msd=None,
                  msd_every=0, stream=None):
    _check(_lib.orng_brownian(seed, ctr0, n_particles, dim, step0, n_steps, dt, D, _ptr(pos),
                              _ptr(msd), msd_every, _stream(stream)), "orng_brownian")


def orng_bd2(pid0, n, step0, n_steps, dt, gamma_over_m, x, y, vx, vy, steps_per_launch=0,
             stream=None):
    _check(_lib.orng_bd2(pid0, n, step0, n_steps, dt, gamma_over_m, _ptr(x), _ptr(y), _ptr(vx),
                         _ptr(vy), steps_per_launch, _stream(stream)), "orng_bd2")


def orng_particle_streams(gen, seed0, n_particles, draws, ctr0, n_iters, out, stream=None):
    _check(_lib.orng_particle_streams(gen, seed0, n_particles, draws, ctr0, n_iters, _ptr(out),
                                      _stream(stream)), "orng_particle_streams")


def orng_set_launch(wg_size=0, unroll=0, max_wgs=0, nontemporal=0):
    cfg = orng_launch_t(wg_size, unroll, max_wgs, nontemporal)
    _check(_lib.orng_set_launch(C.byref(cfg)), "orng_set_launch")


def orng_reset_launch():
    _check(_lib.orng_set_launch(None), "orng_set_launch")


def orng_get_launch():
    cfg = orng_launch_t()
    _check(_lib.orng_get_launch(C.byref(cfg)), "orng_get_launch")
    return dict(wg_size=cfg.wg_size, unroll=cfg.unroll, max_wgs=cfg.max_wgs,
                nontemporal=cfg.nontemporal)


def orng_normal_pairs(x0, x1, n, z0, z1, stream=None):
    _check(_lib.orng_normal_pairs(_ptr(x0), _ptr(x1), n, _ptr(z0), _ptr(z1), _stream(stream)),
           "orng_normal_pairs")


# orng_req_t as a numpy structured dtype (56 bytes, same field order)
REQ_BYTES = 56


def _req_dtype():
    import numpy as np
    return np.dtype([("seed", "<u8"), ("offset", "<u8"), ("n", "<u8"), ("out", "<u8"),
                     ("ctr", "<u4"), ("gen", "<u4"), ("dist", "<u4"), ("flags", "<u4"),
                     ("lo", "<i4"), ("hi", "<i4")], align=False)


def make_requests(gen, dist, seed, ctr, offset, n, out_ptr, lo=0, hi=0):
    """Build a contiguous orng_req_t array from per-request sequences (or
    scalars broadcast to the common length).  out_ptr: device addresses;
    lo, hi: bounds of I32_RANGE requests (ignored for the others)."""
    import numpy as np
    cols = [np.asarray(x) for x in (gen, dist, seed, ctr, offset, n, out_ptr, lo, hi)]
    m = max(c.size for c in cols)
    r = np.zeros(m, dtype=_req_dtype())
    r["gen"], r["dist"] = cols[0], cols[1]
    r["seed"], r["ctr"] = cols[2].astype(np.uint64), cols[3].astype(np.uint32)
    r["offset"], r["n"] = cols[4].astype(np.uint64), cols[5].astype(np.uint64)
    r["out"] = cols[6].astype(np.uint64)
    r["lo"], r["hi"] = cols[7].astype(np.int32), cols[8].astype(np.int32)
    return r


def orng_fill_batched(reqs, stream=None):
    """reqs: numpy array of dtype _req_dtype() (see make_requests)."""
    assert reqs.dtype.itemsize == REQ_BYTES and reqs.flags["C_CONTIGUOUS"]
    _check(_lib.orng_fill_batched(reqs.ctypes.data if reqs.size else None, reqs.size,
                                  _stream(stream)), "orng_fill_batched")


def orng_fill_batched_noalloc(reqs, stream=None):
    """As orng_fill_batched, with the batch tables in the library's fixed
    device array (no allocation; see include/orng.h for the limits)."""
    assert reqs.dtype.itemsize == REQ_BYTES and reqs.flags["C_CONTIGUOUS"]
    _check(_lib.orng_fill_batched_noalloc(reqs.ctypes.data if reqs.size else None, reqs.size,
                                          _stream(stream)), "orng_fill_batched_noalloc")


NOALLOC_MAX_REQUESTS, NOALLOC_MAX_TILES = 131072, 4194304


def orng_fill_each(reqs, stream=None):
    assert reqs.dtype.itemsize == REQ_BYTES and reqs.flags["C_CONTIGUOUS"]
    _check(_lib.orng_fill_each(reqs.ctypes.data if reqs.size else None, reqs.size,
                               _stream(stream)), "orng_fill_each")


def orng_autotune(gen, dist, cache_path=None):
    _check(_lib.orng_autotune(gen, dist, cache_path.encode() if cache_path else None),
           "orng_autotune")


def orng_tune_load(cache_path):
    _check(_lib.orng_tune_load(cache_path.encode()), "orng_tune_load")


def orng_serve_create(arena_bytes, arena=None, max_slots=0, step_words=0):
    cfg = orng_serve_cfg_t(_ptr(arena), arena_bytes, max_slots, 0, step_words)
    h = C.c_void_p()
    _check(_lib.orng_serve_create(C.byref(cfg), C.byref(h)), "orng_serve_create")
    return h.value


def orng_serve_submit(srv, gen, dist, seed, ctr, offset, n, out=None, lo=0, hi=0):
    r = orng_req_t(seed, offset, n, _ptr(out), ctr, gen, dist, 0, lo, hi)
    t = C.c_uint64()
    _check(_lib.orng_serve_submit(srv, C.byref(r), C.byref(t)), "orng_serve_submit")
    return t.value


def orng_serve_try_submit(srv, gen, dist, seed, ctr, offset, n, out=None, lo=0, hi=0):
    """Non-blocking submit: the ticket, or None when the server cannot admit
    the request at once (ORNG_EAGAIN; nothing was queued)."""
    r = orng_req_t(seed, offset, n, _ptr(out), ctr, gen, dist, 0, lo, hi)
    t = C.c_uint64()
    st = _lib.orng_serve_try_submit(srv, C.byref(r), C.byref(t))
    if st == EAGAIN:
        return None
    _check(st, "orng_serve_try_submit")
    return t.value


def orng_serve_submit_many(srv, reqs):
    """reqs: numpy array of orng_req_t records (make_requests; out = 0 asks for
    an arena output).  Returns a numpy array of tickets."""
    import numpy as np
    assert reqs.dtype.itemsize == REQ_BYTES and reqs.flags["C_CONTIGUOUS"]
    t = np.zeros(reqs.size, dtype=np.uint64)
    _check(_lib.orng_serve_submit_many(srv, reqs.ctypes.data if reqs.size else None, reqs.size,
                                       t.ctypes.data if reqs.size else None),
           "orng_serve_submit_many")
    return t


def orng_serve_release_many(srv, tickets, timeout_ns=-1):
    """Wait for and release tickets in order; returns how many were released."""
    import numpy as np
    t = np.ascontiguousarray(tickets, dtype=np.uint64)
    n = C.c_size_t()
    st = _lib.orng_serve_release_many(srv, t.ctypes.data if t.size else None, t.size, timeout_ns,
                                      C.byref(n))
    if st not in (OK, EBUSY):
        _check(st, "orng_serve_release_many")
    return n.value


def _result(res):
    return dict(d_out=res.d_out, n=res.n, t_submit_ns=res.t_submit_ns,
                t_admit_ns=res.t_admit_ns, t_done_ns=res.t_done_ns, status=res.status)


def orng_serve_poll(srv, ticket):
    """Returns the result dict when done, None while queued or running."""
    res = orng_result_t()
    st = _lib.orng_serve_poll(srv, ticket, C.byref(res))
    if st == EBUSY:
        return None
    _check(st, "orng_serve_poll")
    return _result(res)


def orng_serve_wait(srv, ticket, timeout_ns=-1):
    res = orng_result_t()
    st = _lib.orng_serve_wait(srv, ticket, timeout_ns, C.byref(res))
    if st == EBUSY:
        return None
    _check(st, "orng_serve_wait")
    return _result(res)


def orng_serve_release(srv, ticket):
    _check(_lib.orng_serve_release(srv, ticket), "orng_serve_release")


def orng_serve_stats(srv):
    st = orng_serve_stats_t()
    _check(_lib.orng_serve_stats(srv, C.byref(st)), "orng_serve_stats")
    return {k: getattr(st, k) for k, _ in orng_serve_stats_t._fields_}


def orng_serve_destroy(srv):
    _check(_lib.orng_serve_destroy(srv), "orng_serve_destroy")


# -------- convenience wrappers that allocate the output tensor ---------------
def _torch_dtype(dist):
    import torch
    return {U32: torch.int32, F64_UNIFORM: torch.float64, F64_NORMAL: torch.float64,
            I32_RANGE: torch.int32}.get(dist, torch.float32)


def fill(gen, dist, seed, ctr, offset, n, device="cuda", stream=None):
    """Returns a new device tensor (uint32 viewed as int32 for U32, float64 for
    F64_UNIFORM and F64_NORMAL, float32 otherwise)."""
    import torch
    dt = _torch_dtype(dist)
    out = torch.empty(n, dtype=dt, device=device)
    orng_fill(gen, dist, seed, ctr, offset, n, out, stream)
    return out


def fill_multi(gen, dist, seed, ctr0, n_streams, offset, per_stream, device="cuda", stream=None):
    import torch
    dt = _torch_dtype(dist)
    out = torch.empty(n_streams * per_stream, dtype=dt, device=device)
    orng_fill_multi(gen, dist, seed, ctr0, n_streams, offset, per_stream, out, stream)
    return out
