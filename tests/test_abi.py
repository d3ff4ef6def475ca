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
    assert lib.pir_answer_batch_qmajor(None, None, 4, None, None, 0, None) == 1
    assert lib.pir_client_query(None, 4, 4, None, None, None, 1, None, None) == 1
    assert lib.pir_client_decode(None, 4, 4, None, None, 1, None, None) == 1
    assert lib.pir_db_set_variant(None, 0, 0) == 1
    assert lib.pir_db_get_variant(None, 0) == 0
    assert lib.pir_server_create(None, None) == 1
    assert lib.pir_server_destroy(None) == 0
    assert lib.pir_server_submit(None, 0, None, None, 0, None) == 1
    assert lib.pir_server_now_ns() > 0
    assert lib.pir_chor_answer(None, 4, 4, 4, None, 1, None, None) == 1
    assert lib.pir_chor_answer(None, 4, 4, 4, None, 0, None, None) == 0


def test_gathered_variant_flag(qpir):
    # The flag that selects the row-gathered variant table has the value the
    # header defines, and the handle checks still come first.
    from paper_2510_03631_amd._lib import VARIANT_ROWS
    m = re.search(r"#define\s+PIR_VARIANT_ROWS\s+(0x[0-9a-fA-F]+)u", open(HEADER).read())
    assert m and int(m.group(1), 16) == VARIANT_ROWS
    lib = qpir.lib()
    assert lib.pir_db_set_variant(None, VARIANT_ROWS | 64, 1) == 1
    assert lib.pir_db_get_variant(None, VARIANT_ROWS | 64) == 0


def test_variant_tables(qpir):
    qp = qpir
    names0 = qp.variant_names(0)
    names64 = qp.variant_names(64)
    assert names0[0] == "auto" and names64[0] == "auto"
    assert len(set(names0)) == len(names0) and len(set(names64)) == len(names64)
    lib = qp.lib()
    assert lib.pir_variant_name(64, 999) == b"invalid"


def test_server_config_checks(qpir):
    qp = qpir
    from paper_2510_03631_amd._lib import ServerConfig
    lib = qp.lib()
    out = ctypes.c_void_p()
    bad = [ServerConfig(0, 1, 1 << 30, 0, 1), ServerConfig(3, 1, 1 << 30, 0, 1),
           ServerConfig(64, 0, 1 << 30, 0, 1), ServerConfig(64, 17, 1 << 30, 0, 1),
           ServerConfig(64, 2, 0, 0, 1), ServerConfig(2048, 2, 1 << 30, 0, 1)]
    for cfg in bad:
        assert lib.pir_server_create(ctypes.byref(cfg), ctypes.byref(out)) == 2
