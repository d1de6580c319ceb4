"""The C-ABI library loads and exports every symbol include/fkconv.h declares
(no compute calls: this runs without a GPU), and the Python binding covers
exactly that surface."""
import ctypes
import os
import re

import pytest

from paper_1909_10547_amd import fkconv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fkconv.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fk_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["fk_load_table", "fk_conv_dis", "fk_conv_had", "fk_conv_backward", "fk_chi2",
                 "fk_submit", "fk_poll", "fk_create", "fk_destroy", "fk_load_covariance"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fkconv.library_path()):
        pytest.skip("library not built")
    lib = ctypes.CDLL(fkconv.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header():
    assert sorted(fkconv.SIGNATURES) == declared_functions()


def test_null_context_is_rejected_without_touching_the_device():
    if not os.path.exists(fkconv.library_path()):
        pytest.skip("library not built")
    L = fkconv.lib()
    h = ctypes.c_int64()
    assert L.fk_load_table(None, 1, 1, 1, 2, None, None, None, 0, ctypes.byref(h)) == fkconv.FK_E_ARG
    assert L.fk_conv_had(None, 1, None, None, 1, None, None) == fkconv.FK_E_ARG
    assert L.fk_submit(None, None, None) == fkconv.FK_E_ARG
    assert L.fk_create(None, 0, 0) == fkconv.FK_E_ARG
    assert b"NULL" in L.fk_last_error(None)
