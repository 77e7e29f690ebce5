"""The C-ABI library loads on the CPU and exports every function include/zippir.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zippir.h")
LIB = os.path.join(ROOT, "paper_2603_09190_amd", "libzippir.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pir_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libzippir.so is not built (python -m paper_2603_09190_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pir_setup", "pir_hint", "pir_answer", "pir_compress", "pir_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header():
    from paper_2603_09190_amd import native
    assert set(declared_functions()) <= set(native.EXPORTED)


def test_strerror_without_gpu(lib):
    lib.pir_strerror.restype = ctypes.c_char_p
    assert lib.pir_strerror(0) == b"ok"
    assert lib.pir_strerror(-4) == b"hint missing or stale"


def test_setup_rejects_null_without_touching_the_gpu(lib):
    lib.pir_setup.restype = ctypes.c_int32
    lib.pir_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    st = lib.pir_setup(ctypes.byref(h), 0, None, None, 4, 4, None, 4, 0)
    assert st == -1 and h.value is None
    assert b"non-NULL" in lib.pir_last_error()


def test_engine_policy_capacity():
    from paper_2603_09190_amd import native
    assert native.engine_capacity(1000, 100, 32) == 10
    assert native.engine_capacity(10**12, 100, 32) == 32
    assert native.engine_capacity(99, 100, 32) == 0
    assert native.engine_capacity(0, 1, 8) == 0


def test_engine_policy_plan():
    from paper_2603_09190_amd import native
    assert native.engine_plan([64, 64, 64, 128, 64], 32) == 3   # stops at the first other limb count
    assert native.engine_plan([64, 64, 64], 2) == 2             # capacity bound
    assert native.engine_plan([128], 32) == 1
    assert native.engine_plan([], 32) == 0
    assert native.engine_plan([64, 64], 0) == 0


@pytest.mark.parametrize("rows,cols,n", [(4, (1 << 24) + 1, 4), ((1 << 30) + 1, 4, 4), (4, 4, (1 << 16) + 1)])
def test_setup_rejects_oversized_shapes_without_touching_the_gpu(lib, rows, cols, n):
    # Shapes beyond the documented limits (cols <= 2^24 keeps in-kernel offsets and grid
    # dimensions in range) fail with PIR_EINVAL before any device call; the pointers are
    # never read.
    lib.pir_setup.restype = ctypes.c_int32
    lib.pir_last_error.restype = ctypes.c_char_p
    dummy = ctypes.create_string_buffer(16)
    h = ctypes.c_void_p()
    st = lib.pir_setup(ctypes.byref(h), 0, None, dummy, ctypes.c_uint32(rows), ctypes.c_uint32(cols), dummy,
                       ctypes.c_uint32(n), 0)
    assert st == -1 and h.value is None
    assert b"shape too large" in lib.pir_last_error()


def test_engine_step_sizes_without_touching_the_gpu(lib):
    # An engine with an explicit budget is created without device calls; its step sizes are
    # accepted before any database is added, and 0 is rejected.
    lib.pir_engine_create.restype = ctypes.c_int32
    lib.pir_engine_set_steps.restype = ctypes.c_int32
    lib.pir_engine_set_steps.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
    lib.pir_engine_destroy.argtypes = [ctypes.c_void_p]
    lib.pir_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.pir_engine_create(ctypes.byref(h), 8, ctypes.c_uint64(1 << 30)) == 0 and h.value
    try:
        assert lib.pir_engine_set_steps(h, 1 << 20, 4096) == 0
        assert lib.pir_engine_set_steps(h, 0, 4096) == -1
        assert b"positive" in lib.pir_last_error()
        assert lib.pir_engine_set_steps(h, 1 << 20, 0) == -1
        assert lib.pir_engine_set_steps(None, 1 << 20, 4096) == -1
    finally:
        lib.pir_engine_destroy(h)
