"""The C-ABI library loads and exports every function include/insort.h
declares; the Python binding names the same functions.  No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "insort.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(isa_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["isa_ctx_create", "isa_ctx_destroy", "isa_group_by", "isa_group_by_segmented",
              "isa_batch_run", "isa_server_create", "isa_server_submit", "isa_server_poll",
              "isa_server_destroy", "isa_min_workspace_bytes", "isa_status_str"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2010_00152_amd as isa
    if not os.path.exists(isa.LIB_PATH):
        pytest.skip("libinsort.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(isa.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in isa.SIGNATURES, n


def test_host_only_calls():
    import paper_2010_00152_amd as isa
    if not os.path.exists(isa.LIB_PATH):
        pytest.skip("libinsort.so not built")
    L = isa.lib()
    assert L.isa_state_row_bytes(isa.ISA_ALL) == 48
    assert L.isa_state_row_bytes(0) == 8
    assert L.isa_state_row_bytes(isa.ISA_INT_AGGS) == 40
    assert L.isa_min_workspace_bytes(isa.ISA_ALL) > 0
    assert L.isa_status_str(isa.ISA_ETRUNC).decode().startswith("output capacity")
    # null arguments are rejected before any device work
    assert L.isa_group_by(None, None, 0, isa.isa_workspace(None, 0), isa.isa_spill(None, 0),
                          None, None, None) == isa.ISA_EINVAL
