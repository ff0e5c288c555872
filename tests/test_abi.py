"""The C-ABI library loads and exports every symbol the header declares;
host-side argument checks return RBF_E_INVALID_ARG without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2509_26222_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rbf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    decl = declared_symbols()
    assert len(decl) >= 19
    assert sorted(L.SIGNATURES) == decl


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = L.load()
    for code in range(8):
        assert lib.rbf_status_string(code)
    assert lib.rbf_status_string(0) == b"ok"


def test_null_arguments_are_rejected_on_host():
    lib = L.load()
    E = 1  # RBF_E_INVALID_ARG
    assert lib.rbf_ctx_create(None, 0, None) == E
    assert lib.rbf_ctx_destroy(None) == E
    assert lib.rbf_sync_status(None) == E
    assert lib.rbf_grid_destroy(None) == E
    assert lib.rbf_grid_info(None, None, None, None, None) == E
    assert lib.rbf_eval(None, None, None, None, None, 0, 2, None, 0.0, 0,
                        None, None, None, None) == E
    assert lib.rbf_eval_adjoint(None, None, None, None, None, 0, 2, None, 0,
                                None, None, None, None, None) == E
    assert lib.rbf_update(None, None, None, None, None, 0, None, None, 0, 0, 0,
                          None) == E
    assert lib.rbf_update_active(None, None, None, None, None, 0, None, None, 0, 0, 0,
                                 None, None, None) == E
    assert lib.rbf_select_centers(None, None, 0, None, 0.5, 0.5, 0, 0, None, 0,
                                  None) == E
    assert lib.rbf_select_centers_grow(None, None, 0, None, 0.5, 0.5, 0, 0, None, None, 0,
                                       None) == E
    assert lib.rbf_state_grow(None, None, None, None, 0, 0, 0) == E
    assert lib.rbf_last_error_index(None) == -1


def test_ctx_create_rejects_bad_device():
    lib = L.load()
    h = C.c_void_p()
    assert lib.rbf_ctx_create(C.byref(h), -1, None) == 1
    assert lib.rbf_ctx_create(C.byref(h), 1 << 20, None) == 1
