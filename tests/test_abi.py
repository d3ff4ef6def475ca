"""The C ABI library loads and exports what include/qpir.h declares (CPU only).

No compute call is made here; only entry points that return before touching
the GPU (argument checks, status strings) are exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpir.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pir_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def qpir():
    import paper_2510_03631_amd as p
    return p


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("pir_db_open", "pir_answer", "pir_answer_batch", "pir_setup_hint",
                 "pir_update_rows", "pir_hint_update_rows", "pir_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol(qpir):
    lib = qpir.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(qpir.SIGNATURES)


def test_status_strings_and_version(qpir):
    lib = qpir.lib()
    for st in range(7):
        assert lib.pir_status_string(st)
    assert lib.pir_status_string(99) == b"unknown status"
    assert lib.pir_version() >> 16 == 1


def test_argument_checks_before_any_device_call(qpir):
    lib = qpir.lib()
    out = ctypes.c_void_p()
    assert lib.pir_db_open(None, 4, 4, 4, None, ctypes.byref(out)) == 1
    assert lib.pir_db_open(ctypes.c_void_p(16), 4, 4, 4, None, None) == 1
    assert lib.pir_db_open(ctypes.c_void_p(16), 0, 4, 4, None, ctypes.byref(out)) == 2
    assert lib.pir_db_open(ctypes.c_void_p(16), 4, 8, 4, None, ctypes.byref(out)) == 2
    assert lib.pir_db_open(ctypes.c_void_p(16), 1 << 31, 8, 8, None, ctypes.byref(out)) == 2
    assert lib.pir_answer(None, None, None, None, 0, None) == 1
    assert lib.pir_answer_batch(None, None, 4, None, None, 0, None) == 1
    assert lib.pir_setup_hint(None, None, 4, None, None, 0, None) == 1
    assert lib.pir_update_rows(None, None, 4, None, None) == 1
    assert lib.pir_hint_update_rows(None, None, 4, None, 4, None, None, 0, None) == 1
    assert lib.pir_workspace_bytes(None, 0) == 0
    assert lib.pir_db_close(None) == 0
