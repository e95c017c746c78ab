"""The C ABI: the shared library loads on the CPU and exports every function that
include/srhd.h declares; host-side argument checks reject bad calls before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srhd.h")
LIB = os.path.join(ROOT, "paper_2012_11130_amd", "libsrhd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(srhd_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2012_11130_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_argument_errors_are_reported_without_a_gpu(lib):
    lib.srhd_prim2cons.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.srhd_last_error.restype = ctypes.c_char_p
    assert lib.srhd_prim2cons(7, 10, None, None, None) == -1
    assert b"dtype" in lib.srhd_last_error()
    assert lib.srhd_prim2cons(0, -1, None, None, None) == -1
    assert lib.srhd_prim2cons(0, 10, None, None, None) == -1
    assert b"NULL" in lib.srhd_last_error()
    assert lib.srhd_prim2cons(0, 0, None, None, None) == 0       # empty batch is a no-op
    # overlapping arrays are rejected before any launch (host addresses are never touched)
    buf = ctypes.create_string_buffer(800)
    a = ctypes.addressof(buf)
    assert lib.srhd_prim2cons(0, 10, a, a + 8, None) == -1
    assert b"overlap" in lib.srhd_last_error()
    assert lib.srhd_prim2cons(0, 1, a + 1, a + 400, None) == -1      # misaligned
    lib.srhd_abi_version.restype = ctypes.c_int
    assert lib.srhd_abi_version() == 1


def test_step_descriptor_checks(lib):
    from paper_2012_11130_amd import srhd as S  # noqa: F401  (struct definitions only)
    d = S.srhd_patches()
    d.n_patch = 4
    d.ghost = 1
    d.dtype = 0
    d.n_level = 1
    d.dh[0] = 0.1
    prm = S.srhd_step_params()
    prm.theta = 1.5
    prm.max_retry = 4
    rc = S._lib.srhd_fluid_step(ctypes.byref(d), None, None, ctypes.byref(prm), None, None)
    assert rc == -1 and b"ghost" in S._lib.srhd_last_error()
    d.ghost = 3
    prm.theta = 5.0
    rc = S._lib.srhd_fluid_step(ctypes.byref(d), None, None, ctypes.byref(prm), None, None)
    assert rc == -1 and b"theta" in S._lib.srhd_last_error()
    prm.theta = 1.5
    d.dtype = 1
    rc = S._lib.srhd_fluid_step(ctypes.byref(d), None, None, ctypes.byref(prm), None, None)
    assert rc == -3
