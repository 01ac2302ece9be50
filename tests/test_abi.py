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


@pytest.mark.parametrize("nr,nz", [(2049, 8), (8, 1025), (2048, 1024), (0, 8)])
def test_create_rejects_grids_beyond_the_limits(nr, nz):
    """ecpic_create rejects shapes beyond its kernels' limits (nr <= 2048,
    nz <= 1024, ceil(nr/4) ceil(nz/32) <= 8192) before it touches the
    device; the largest accepted shapes are solved in the GPU field-solve
    parity test."""
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libecpic.so not built")
    L = P.lib()
    g = P.GridDesc()
    g.nr, g.nz, g.R, g.L, g.xi_axis, g.dt, g.eps, g.mu = nr, nz, 0.1, 0.1, 2.0, 1e-11, 8.85e-12, 1.26e-6
    h = ctypes.c_void_p()
    assert L.ecpic_create(ctypes.byref(g), 0, None, ctypes.byref(h)) == -1
    assert not h.value
