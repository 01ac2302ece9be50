"""The C-ABI library loads and exports every entry point the header declares
(no compute call: this runs without a GPU)."""
import ctypes
import os

import pytest

import paper_2212_08836_amd as P


def test_header_declares_the_boundary_calls():
    names = P.header_symbols()
    for must in ("ecpic_create", "ecpic_add_species", "ecpic_push_deposit", "ecpic_field_iterate",
                 "ecpic_collide", "ecpic_step", "ecpic_destroy", "ecpic_sort", "ecpic_workspace_size",
                 "ecpic_bind_workspace", "ecpic_bind_fields", "ecpic_set_option"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libecpic.so not built")
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in P.header_symbols() if not hasattr(L, n)]
    assert missing == []


def test_status_strings_without_gpu():
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libecpic.so not built")
    L = P.lib()
    assert L.ecpic_status_string(0) == b"ok"
    assert L.ecpic_status_string(-4).startswith(b"Picard")
    assert L.ecpic_last_error(None) == b"null context"
