"""The C-ABI library loads on a machine without a GPU and exports every
function that include/*.h declares.  No compute calls are made here."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_19925_amd", "liborng.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(orng_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["orng_fill", "orng_fill_multi", "orng_brownian", "orng_strerror"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("liborng.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.orng_strerror.restype = ctypes.c_char_p
    assert lib.orng_strerror(0) == b"ok"
    assert lib.orng_strerror(-2).startswith(b"position")
    assert lib.orng_version() > 0
    # argument validation happens before any device work
    lib.orng_fill.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.orng_fill(10, 0, 1, 1, 0, 4, None, None) == -1
    assert lib.orng_fill(9, 0, 2**32, 1, 0, 4, None, None) == -1  # 32-bit key
    assert lib.orng_fill(0, 0, 1, 1, 2**32, 1, None, None) == -2
    assert lib.orng_fill(0, 0, 1, 1, 0, 0, None, None) == 0
    assert lib.orng_fill(0, 0, 1, 1, 0, 4, None, None) == -1


def test_header_is_plain_c_and_links(tmp_path):
    """include/orng.h compiles as C99 and a C program links against liborng.so
    and calls the host-only entry points."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    src = tmp_path / "t.c"
    src.write_text(
        '#include "orng.h"\n#include <stdio.h>\n'
        'int main(void) {\n'
        '  orng_req_t r = {0};\n'
        '  orng_launch_t l = {0};\n'
        '  orng_serve_stats_t st;\n'
        '  (void)r; (void)st;\n'
        '  if (orng_get_launch(&l) != ORNG_OK) return 1;\n'
        '  if (orng_fill(ORNG_SQUARES64 + 1, ORNG_U32, 1, 1, 0, 4, (void*)0, (void*)0) != ORNG_EINVAL) return 2;\n'
        '  printf("%s %d\\n", orng_strerror(ORNG_ERANGE), orng_version());\n'
        '  return sizeof(orng_req_t) == 56 ? 0 : 3;\n'
        '}\n')
    exe = tmp_path / "t"
    libdir = os.path.dirname(LIB)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), LIB, "-Wl,-rpath," + libdir, "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert r.stdout.startswith("position or counter out of range")


def test_noalloc_batched_limits_without_gpu():
    """orng_fill_batched_noalloc checks its requests and its fixed limits on
    the host, before any device call: too many requests or tiles give ENOMEM,
    a bad request its own error, an empty batch OK."""
    import numpy as np
    lib = ctypes.CDLL(LIB)
    fn = lib.orng_fill_batched_noalloc
    fn.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    fn.restype = ctypes.c_int
    dt = np.dtype([("seed", "<u8"), ("offset", "<u8"), ("n", "<u8"), ("out", "<u8"),
                   ("ctr", "<u4"), ("gen", "<u4"), ("dist", "<u4"), ("flags", "<u4"),
                   ("lo", "<i4"), ("hi", "<i4")])
    assert dt.itemsize == 56  # sizeof(orng_req_t)
    max_req, max_tiles = 131072, 4194304
    hdr = open(os.path.join(ROOT, "include", "orng.h")).read()
    assert "ORNG_NOALLOC_MAX_REQUESTS = %d" % max_req in hdr
    assert "ORNG_NOALLOC_MAX_TILES = %d" % max_tiles in hdr
    r = np.zeros(max_req + 1, dt)
    assert fn(r.ctypes.data, r.size, None) == -3          # ENOMEM: too many requests
    assert fn(r.ctypes.data, max_req, None) == 0          # all empty: nothing to do
    r = np.zeros(max_req, dt)
    r["n"], r["out"] = 1 << 20, 1 << 20                   # 64 tiles or more each
    assert fn(r.ctypes.data, r.size, None) == -3          # ENOMEM: too many tiles
    r[5]["gen"] = 10
    assert fn(r.ctypes.data, r.size, None) == -1          # the bad request comes first
    r = np.zeros(3, dt)
    r[1]["offset"], r[1]["n"], r[1]["out"] = 2**32 - 2, 4, 4096
    assert fn(r.ctypes.data, r.size, None) == -2          # ERANGE
