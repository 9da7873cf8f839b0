"""The C-ABI library loads and exports every function include/gp.h declares.

Runs without a GPU: loading libgp.so resolves symbols only; no entry point is
called except the pure host function gp_lmax, checked against the §II-A bound.
"""
import ctypes
import os
import re

import pytest

import paper_1710_08231_amd as gp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gp.LIB_PATH):
        gp.build()
    return ctypes.CDLL(gp.LIB_PATH)


def test_header_declares_entry_points():
    names = _declared()
    for required in ("gp_lp_cluster", "gp_contract", "gp_lp_refine", "gp_partition"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(gp.EXPORTS) <= set(_declared())


def test_lmax_host_function(lib):
    lib.gp_lmax.restype = ctypes.c_int64
    lib.gp_lmax.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double]
    assert lib.gp_lmax(16384, 2, 0.03) == 8437
    assert lib.gp_lmax(1 << 22, 16, 0.03) == 270008
    assert lib.gp_lmax(10, 0, 0.03) == -1


def test_strerror_messages(lib):
    lib.gp_strerror.restype = ctypes.c_char_p
    assert b"argument" in lib.gp_strerror(-1)
    assert b"overflow" in lib.gp_strerror(-4)
