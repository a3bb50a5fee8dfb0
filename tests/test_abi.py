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
    assert lib.orng_fill(9, 0, 1, 1, 0, 4, None, None) == -1
    assert lib.orng_fill(0, 0, 1, 1, 2**32, 1, None, None) == -2
    assert lib.orng_fill(0, 0, 1, 1, 0, 0, None, None) == 0
    assert lib.orng_fill(0, 0, 1, 1, 0, 4, None, None) == -1
