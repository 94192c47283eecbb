"""The C-ABI library builds for gfx950, loads, and exports every declared entry point.

No compute calls here (no GPU needed).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qbsm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(qbsm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2011_11762_amd import qbsm
    if not os.path.exists(qbsm.LIB_PATH):
        from paper_2011_11762_amd import build
        build.build()
    return qbsm.LIB_PATH


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("qbsm_matrix_create", "qbsm_matrix_set_blocks", "qbsm_multiply_symbolic",
                 "qbsm_multiply_numeric", "qbsm_multiply_backward", "qbsm_batch_run_graph",
                 "qbsm_matrix_get_values", "qbsm_plan_get_products"):
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_abi(lib_path):
    from paper_2011_11762_amd import qbsm
    assert set(qbsm.ABI_SYMBOLS) == set(declared_functions())


def test_dynamic_symbol_table_is_c_linkage(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(qbsm_[a-z0-9_]+)\b", out))
    assert set(declared_functions()) <= exported


def test_status_strings_without_gpu(lib_path):
    lib = ctypes.CDLL(lib_path)
    lib.qbsm_status_string.restype = ctypes.c_char_p
    lib.qbsm_status_string.argtypes = [ctypes.c_int32]
    assert lib.qbsm_status_string(0) == b"ok"
    assert lib.qbsm_status_string(3) == b"invalid block pattern"
    assert lib.qbsm_version() == 10000


def test_create_validates_arguments_without_gpu(lib_path):
    lib = ctypes.CDLL(lib_path)
    h = ctypes.c_void_p()
    lib.qbsm_matrix_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p)]
    assert lib.qbsm_matrix_create(100, 100, 48, ctypes.byref(h)) == 6       # unsupported bs
    assert lib.qbsm_matrix_create(-1, 100, 64, ctypes.byref(h)) == 1        # negative size
    assert lib.qbsm_matrix_create(100, 100, 64, None) == 1                  # null out
    assert lib.qbsm_matrix_create(64 * 65537, 64, 64, ctypes.byref(h)) == 6  # grid too large
    assert lib.qbsm_matrix_create(100, 90, 64, ctypes.byref(h)) == 0
    lib.qbsm_matrix_destroy.argtypes = [ctypes.c_void_p]
    assert lib.qbsm_matrix_destroy(h) == 0
