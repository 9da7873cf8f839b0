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


def _header_struct_fields(name):
    src = open(os.path.join(ROOT, "include", "gp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:  # "type a" or "type a, b, c" (array bounds allowed)
            for part in decl.split(","):
                fields.append(re.search(r"(\w+)\s*(\[\s*\d+\s*\])?$", part.strip()).group(1))
    return fields


@pytest.mark.parametrize("cls,name", [(gp.Graph, "gp_graph"), (gp.LPStats, "gp_lp_stats"),
                                      (gp.Params, "gp_params"), (gp.Result, "gp_result"),
                                      (gp.Tuning, "gp_tuning"), (gp.MLSStats, "gp_mls_stats")])
def test_binding_structs_match_header(cls, name):
    # the ctypes mirrors list the header's fields in the header's order
    assert [f for f, _ in cls._fields_] == _header_struct_fields(name)


def test_default_params_host_function(lib):
    p = gp.Params()
    lib.gp_default_params.argtypes = [ctypes.POINTER(gp.Params)]
    lib.gp_default_params(ctypes.byref(p))
    assert (p.rounds_coarsen, p.rounds_refine, p.coarsest_per_k, p.attempts) == (10, 25, 60, 4)
    assert (p.stall_num, p.stall_den, p.dir_alternate, p.seed) == (19, 20, 1, 0)
    assert (p.init_mode, p.mpnn_max_n, p.mpnn_seed, p.mpnn_params) == (0, 131072, 0, None)
    assert (p.active_set, p.init_fm) == (0, 0)
    assert (p.mls, p.mls_batch, p.mls_queue) == (0, 0, 64)


def test_workspace_bytes_host_function(lib):
    # gp_workspace_bytes is a host function: an upper bound of the scratch of one call
    lib.gp_workspace_bytes.restype = ctypes.c_size_t
    lib.gp_workspace_bytes.argtypes = [ctypes.c_int32] * 5
    cl = [lib.gp_workspace_bytes(gp.OP_LP_CLUSTER, n, 16 * n, 1, 1) for n in (1000, 10_000, 100_000)]
    assert 0 < cl[0] < cl[1] < cl[2]
    ref = lib.gp_workspace_bytes(gp.OP_LP_REFINE, 100_000, 1_600_000, 16, 1)
    assert 0 < ref < cl[2]  # k block weights instead of n label weights and hub tables
    # the active-set rounds keep more per vertex
    assert lib.gp_workspace_bytes(gp.OP_LP_REFINE, 100_000, 1_600_000, 16, 3) > ref
    assert lib.gp_workspace_bytes(gp.OP_CONTRACT, 100_000, 1_600_000, 1, 1) > 44 * 1_600_000
    assert lib.gp_workspace_bytes(gp.OP_CUT, 100_000, 1_600_000, 1, 1) >= 4 * 1_600_000
    # invalid arguments and the multilevel calls (their need depends on the hierarchy): 0
    assert lib.gp_workspace_bytes(99, 10, 10, 1, 1) == 0
    assert lib.gp_workspace_bytes(gp.OP_LP_REFINE, 10, 10, 0, 1) == 0
    assert lib.gp_workspace_bytes(gp.OP_LP_CLUSTER, -1, 10, 1, 1) == 0


def test_null_workspace_with_bytes_is_rejected_before_device_work(lib):
    # the argument check comes first, so no GPU is touched
    g = gp.Graph(0, 0, None, None, None, None)
    lib.gp_lp_cluster.argtypes = [ctypes.POINTER(gp.Graph), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]
    assert lib.gp_lp_cluster(ctypes.byref(g), 1, 1, 1, None, None, None, 64, None) == -1
