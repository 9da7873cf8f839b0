"""Plain CPU oracle — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and shares
no code with it. ``oracle.c`` is the plain definition of every
result of the partitioner's hot path (see its header for the paper sections it
follows); this module is argument marshalling for it plus the checks the tests
use to pin it (brute-force optimal cuts and the matrix form of contraction are
written out in the pin tests, ``tests/test_oracle_pins.py``).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xadj", I32P), ("adjncy", I32P), ("adjwgt", I32P),
                ("vwgt", I32P)]


class _LPStats(ctypes.Structure):
    _fields_ = [("rounds_run", ctypes.c_int32), ("moves", ctypes.c_int64),
                ("edge_visits", ctypes.c_int64)]


class _Params(ctypes.Structure):
    _fields_ = [("rounds_coarsen", ctypes.c_int32), ("rounds_refine", ctypes.c_int32),
                ("coarsest_per_k", ctypes.c_int32), ("attempts", ctypes.c_int32),
                ("stall_num", ctypes.c_int32), ("stall_den", ctypes.c_int32),
                ("dir_alternate", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("init_mode", ctypes.c_int32), ("mpnn_max_n", ctypes.c_int32),
                ("mpnn_seed", ctypes.c_uint64), ("mpnn_params", ctypes.POINTER(ctypes.c_float)),
                ("lp_async", ctypes.c_int32), ("active_set", ctypes.c_int32), ("mls", ctypes.c_int32),
                ("init_fm", ctypes.c_int32), ("mls_batch", ctypes.c_int32), ("mls_queue", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("max_block_w", ctypes.c_int64),
                ("lmax", ctypes.c_int64), ("ucl", ctypes.c_int64),
                ("balanced", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("edge_visits_cluster", ctypes.c_int64), ("edge_visits_refine", ctypes.c_int64),
                ("coarsest_n", ctypes.c_int32), ("n_isolated", ctypes.c_int32),
                ("learned_tried", ctypes.c_int32), ("learned_kept", ctypes.c_int32),
                ("plain_cut_coarsest", ctypes.c_int64), ("learned_cut_coarsest", ctypes.c_int64)]


def build_lib():
    """Compile oracle.c and mpnn.c with gcc (always rebuilds). Building the checker is not
    using it. -ffp-contract=off keeps every binary32 product and sum that mpnn.c does not
    write as fmaf rounded on its own."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-std=gnu11", "-fopenmp",
                           "-ffp-contract=off", "-o", tmp, os.path.join(_HERE, "oracle.c"),
                           os.path.join(_HERE, "mpnn.c"), os.path.join(_HERE, "mls.c"), "-lm"])
    os.replace(tmp, _LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_lib()
    lib = ctypes.CDLL(_LIB_PATH)
    G = ctypes.POINTER(_Graph)
    lib.orc_set_threads.argtypes = [ctypes.c_int32]
    lib.orc_lmax.restype = ctypes.c_int64
    lib.orc_lmax.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double]
    lib.orc_lp_round.restype = ctypes.c_int64
    lib.orc_lp_round.argtypes = [G, I32P, I64P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int32, I32P]
    lib.orc_lp_cluster.argtypes = [G, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, I32P,
                                   ctypes.POINTER(_LPStats)]
    lib.orc_lp_refine.argtypes = [G, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int32, I32P, ctypes.POINTER(_LPStats)]
    lib.orc_contract.argtypes = [G, I32P, I32P, I32P, I32P, I32P, I32P, I32P, I32P]
    lib.orc_project.argtypes = [ctypes.c_int32, I32P, I32P, I32P]
    lib.orc_cut.restype = ctypes.c_int64
    lib.orc_cut.argtypes = [G, I32P]
    lib.orc_block_weights.argtypes = [G, I32P, ctypes.c_int32, I64P]
    lib.orc_mix4.restype = ctypes.c_uint64
    lib.orc_mix4.argtypes = [ctypes.c_uint64] * 4
    lib.orc_recursive_bisection.argtypes = [G, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_int32, I32P]
    lib.orc_rebalance.argtypes = [G, ctypes.c_int32, ctypes.c_int64, I32P]
    lib.orc_initial_partition.argtypes = [G, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          I32P]
    lib.orc_fill_isolated.argtypes = [G, ctypes.c_int32, I32P, I64P]
    lib.orc_partition.argtypes = [G, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_Params),
                                  I32P, ctypes.POINTER(_Result)]
    lib.orc_lp_cluster_async.argtypes = [G, ctypes.c_int64, ctypes.c_int32, I32P, ctypes.POINTER(_LPStats)]
    lib.orc_colour_classes.restype = ctypes.c_int32
    lib.orc_colour_classes.argtypes = [G, I32P]
    lib.orc_lp_cluster_colour.argtypes = [G, ctypes.c_int64, ctypes.c_int32, I32P, ctypes.POINTER(_LPStats)]
    lib.orc_lp_refine_colour.argtypes = [G, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, I32P,
                                         ctypes.POINTER(_LPStats)]
    lib.orc_lp_refine_async.argtypes = [G, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, I32P,
                                        ctypes.POINTER(_LPStats)]
    lib.orc_coarsest.argtypes = [G, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_Params),
                                 I32P, I32P, I32P, I32P, I32P, I32P, I32P]
    F32P = ctypes.POINTER(ctypes.c_float)
    lib.orc_mpnn_param_count.restype = ctypes.c_int32
    lib.orc_mpnn_param_count.argtypes = [ctypes.c_int32]
    lib.orc_bf16.restype = ctypes.c_float
    lib.orc_bf16.argtypes = [ctypes.c_float]
    lib.orc_mpnn_features.argtypes = [G, ctypes.c_uint64, F32P]
    lib.orc_mpnn_infer.argtypes = [G, ctypes.c_int32, F32P, ctypes.c_uint64, F32P, I32P]
    lib.orc_mpnn_decode.argtypes = [G, ctypes.c_int32, F32P, ctypes.c_int64, I32P]
    _lib = lib
    return lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p32(a):
    return None if a is None else a.ctypes.data_as(I32P)


class _G:
    """Holds contiguous int32 copies alive while the C struct points into them."""

    def __init__(self, g):
        self.xadj = _i32(g["xadj"])
        self.adjncy = _i32(g["adjncy"])
        self.adjwgt = None if g.get("adjwgt") is None else _i32(g["adjwgt"])
        self.vwgt = None if g.get("vwgt") is None else _i32(g["vwgt"])
        self.n = len(self.xadj) - 1
        self.s = _Graph(self.n, _p32(self.xadj), _p32(self.adjncy), _p32(self.adjwgt),
                        _p32(self.vwgt))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def set_threads(t):
    """Threads of the proposal loop of full LP rounds (1 = the plain sequential loop).
    Results do not depend on it."""
    _load().orc_set_threads(int(t))


def lmax(total, k, eps):
    return int(_load().orc_lmax(total, k, eps))


def total_vwgt(g):
    return int(g["vwgt"].astype(np.int64).sum()) if g.get("vwgt") is not None else len(g["xadj"]) - 1


def lp_round(g, C, W, U, r, dir_alternate=1):
    """One LP round in place on copies; returns (C', W', moves, prop)."""
    G = _G(g)
    C = _i32(C).copy()
    W = np.ascontiguousarray(W, dtype=np.int64).copy()
    prop = np.zeros(G.n, dtype=np.int32)
    m = _load().orc_lp_round(G.ref, _p32(C), W.ctypes.data_as(I64P), len(W), U, r,
                             dir_alternate, _p32(prop))
    return C, W, int(m), prop


LP_DIR_ALTERNATE, LP_ACTIVE_SET = 1, 2


def _flags(dir_alternate, active):
    return (LP_DIR_ALTERNATE if dir_alternate else 0) | (LP_ACTIVE_SET if active else 0)


def lp_cluster(g, U, rounds=10, dir_alternate=1, active=False):
    G = _G(g)
    out = np.zeros(G.n, dtype=np.int32)
    st = _LPStats()
    _load().orc_lp_cluster(G.ref, U, rounds, _flags(dir_alternate, active), _p32(out), ctypes.byref(st))
    return out, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits}


def lp_refine(g, part, k, lmax_, rounds=25, dir_alternate=1, active=False):
    G = _G(g)
    P = _i32(part).copy()
    st = _LPStats()
    _load().orc_lp_refine(G.ref, k, lmax_, rounds, _flags(dir_alternate, active), _p32(P), ctypes.byref(st))
    return P, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits}


class _MLSStats(ctypes.Structure):
    _fields_ = [("gain", ctypes.c_int64), ("searches", ctypes.c_int64), ("moves", ctypes.c_int64),
                ("local_iters", ctypes.c_int64)]


def mls(g, part, k, lmax_, seed=0, global_iters=3, alpha=0.1, max_idle=50, batch=0, max_queue=0):
    """§III-C multi-try local search from a partition (oracle-only); returns (part', stats).
    batch > 0: searches in batches that start from the same state, their kept moves
    applied in seed order with recomputed gains (§IV-C); batch = 1 equals batch = 0.
    max_queue > 0 bounds the vertices one search may queue."""
    G = _G(g)
    P = _i32(part).copy()
    st = _MLSStats()
    lib = _load()
    lib.orc_mls_batched.restype = ctypes.c_int64
    lib.orc_mls_batched.argtypes = [ctypes.POINTER(_Graph), ctypes.c_int32, ctypes.c_int64, I32P, ctypes.c_uint64,
                                    ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.POINTER(_MLSStats)]
    lib.orc_mls_batched(G.ref, k, lmax_, _p32(P), seed, global_iters, alpha, max_idle, batch, max_queue,
                        ctypes.byref(st))
    return P, {f: getattr(st, f) for f, _ in _MLSStats._fields_}


def mls_gain(g, part, k, lmax_, v):
    """(gain, target) of moving v to its best feasible adjacent block (target -1: none)."""
    G = _G(g)
    P = _i32(part)
    B = np.zeros(k, np.int64)
    vw = g.get("vwgt")
    np.add.at(B, P, vw.astype(np.int64) if vw is not None else 1)
    t = ctypes.c_int32(-1)
    lib = _load()
    lib.orc_mls_gain.restype = ctypes.c_int64
    lib.orc_mls_gain.argtypes = [ctypes.POINTER(_Graph), I32P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                 ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    gn = lib.orc_mls_gain(G.ref, _p32(P), B.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k, lmax_, v,
                          ctypes.byref(t))
    return int(gn), int(t.value)


def lp_cluster_async(g, U, rounds=10):
    """The paper's sequential LP clustering (oracle-only comparison mode)."""
    G = _G(g)
    out = np.zeros(G.n, dtype=np.int32)
    st = _LPStats()
    _load().orc_lp_cluster_async(G.ref, U, rounds, _p32(out), ctypes.byref(st))
    return out, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits}


def lp_refine_async(g, part, k, lmax_, rounds=25):
    G = _G(g)
    P = _i32(part).copy()
    st = _LPStats()
    _load().orc_lp_refine_async(G.ref, k, lmax_, rounds, _p32(P), ctypes.byref(st))
    return P, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits}


def colour_classes(g):
    """(number of colours, colour[n]) of the colour-class LP's first-fit colouring."""
    G = _G(g)
    col = np.zeros(max(G.n, 1), np.int32)
    ncol = int(_load().orc_colour_classes(G.ref, _p32(col)))
    return ncol, col[:G.n].copy()


def lp_cluster_colour(g, U, rounds=10):
    """Colour-class LP clustering (oracle-only comparison mode)."""
    G = _G(g)
    out = np.zeros(max(G.n, 1), dtype=np.int32)
    st = _LPStats()
    _load().orc_lp_cluster_colour(G.ref, U, rounds, _p32(out), ctypes.byref(st))
    return out[:G.n].copy(), {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits}


def lp_refine_colour(g, part, k, lmax_, rounds=25):
    G = _G(g)
    P = _i32(part).copy()
    st = _LPStats()
    _load().orc_lp_refine_colour(G.ref, k, lmax_, rounds, _p32(P), ctypes.byref(st))
    return P, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits}


def contract(g, labels):
    G = _G(g)
    n, nnz = G.n, len(G.adjncy)
    xc = np.zeros(n + 1, np.int32)
    ac = np.zeros(max(nnz, 1), np.int32)
    wc = np.zeros(max(nnz, 1), np.int32)
    vc = np.zeros(max(n, 1), np.int32)
    f2c = np.zeros(max(n, 1), np.int32)
    nc, nnzc = ctypes.c_int32(), ctypes.c_int32()
    lab = _i32(labels)
    _load().orc_contract(G.ref, _p32(lab), _p32(xc), _p32(ac), _p32(wc), _p32(vc), _p32(f2c),
                         ctypes.byref(nc), ctypes.byref(nnzc))
    nc, nnzc = nc.value, nnzc.value
    cg = {"xadj": xc[:nc + 1].copy(), "adjncy": ac[:nnzc].copy(), "adjwgt": wc[:nnzc].copy(),
          "vwgt": vc[:nc].copy()}
    return cg, f2c[:n].copy()


def project(f2c, part_coarse):
    f2c = _i32(f2c)
    pc = _i32(part_coarse)
    out = np.zeros(len(f2c), np.int32)
    _load().orc_project(len(f2c), _p32(f2c), _p32(pc), _p32(out))
    return out


def cut(g, part):
    G = _G(g)
    P = _i32(part)
    return int(_load().orc_cut(G.ref, _p32(P)))


def block_weights(g, part, k):
    G = _G(g)
    P = _i32(part)
    B = np.zeros(k, np.int64)
    _load().orc_block_weights(G.ref, _p32(P), k, B.ctypes.data_as(I64P))
    return B


def mix4(seed, a, base, ks):
    return int(_load().orc_mix4(seed, a, base, ks))


def recursive_bisection(g, k, seed=0, attempt=0, lmax_=0, fm=0):
    """BFS-grow recursive bisection; fm > 0: at most fm 2-way FM passes after every
    bisection, a side that will hold j blocks weighing at most j * lmax_."""
    G = _G(g)
    P = np.zeros(G.n, np.int32)
    _load().orc_recursive_bisection(G.ref, k, seed, attempt, lmax_, fm, _p32(P))
    return P


def rebalance(g, k, lmax_, part):
    G = _G(g)
    P = _i32(part).copy()
    bal = _load().orc_rebalance(G.ref, k, lmax_, _p32(P))
    return P, bool(bal)


def initial_partition(g, k, lmax_, seed=0, attempts=4, rounds_refine=25, dir_alternate=1, fm=0):
    G = _G(g)
    P = np.zeros(G.n, np.int32)
    a = _load().orc_initial_partition(G.ref, k, lmax_, seed, attempts, rounds_refine,
                                      dir_alternate, fm, _p32(P))
    return P, int(a)


def fill_isolated(g, k, part, B):
    G = _G(g)
    P = _i32(part).copy()
    Bc = np.ascontiguousarray(B, dtype=np.int64).copy()
    _load().orc_fill_isolated(G.ref, k, _p32(P), Bc.ctypes.data_as(I64P))
    return P, Bc


DEFAULT_PARAMS = dict(rounds_coarsen=10, rounds_refine=25, coarsest_per_k=60, attempts=4,
                      stall_num=19, stall_den=20, dir_alternate=1, seed=0, init_mode=0,
                      mpnn_max_n=131072, mpnn_seed=0, mpnn_params=None, lp_async=0, active_set=0, mls=0,
                      init_fm=0, mls_batch=0, mls_queue=0)


def _params(params):
    """(_Params, keep-alive) from keyword overrides; mpnn_params is a float array or None."""
    prm = dict(DEFAULT_PARAMS)
    prm.update(params)
    w = prm.pop("mpnn_params")
    keep = None
    if w is not None:
        keep = np.ascontiguousarray(w, dtype=np.float32)
        prm["mpnn_params"] = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    return _Params(**prm), keep


def mpnn_param_count(k):
    return int(_load().orc_mpnn_param_count(k))


def bf16(x):
    """Round binary32 values to bfloat16 (nearest, ties to even); returns float32 array."""
    x = np.asarray(x, dtype=np.float32)
    lib = _load()
    return np.array([lib.orc_bf16(float(v)) for v in x.ravel()], dtype=np.float32).reshape(x.shape)


def mpnn_features(g, seed=0):
    G = _G(g)
    X = np.zeros((G.n, 18), np.float32)
    _load().orc_mpnn_features(G.ref, seed, X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return X


def mpnn_infer(g, k, params, seed=0):
    """Binary32 inference: (logits [n, k], argmax blocks [n])."""
    G = _G(g)
    w = np.ascontiguousarray(params, dtype=np.float32)
    assert w.size == mpnn_param_count(k)
    F32P = ctypes.POINTER(ctypes.c_float)
    Z = np.zeros((G.n, k), np.float32)
    P = np.zeros(G.n, np.int32)
    _load().orc_mpnn_infer(G.ref, k, w.ctypes.data_as(F32P), seed, Z.ctypes.data_as(F32P), _p32(P))
    return Z, P


def mpnn_decode(g, k, Z, lmax_):
    """Capacity-respecting decoding of logits Z [n, k] under block bound lmax_."""
    G = _G(g)
    z = np.ascontiguousarray(Z, dtype=np.float32)
    P = np.zeros(G.n, np.int32)
    _load().orc_mpnn_decode(G.ref, k, z.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), lmax_, _p32(P))
    return P


def coarsest(g, k, eps=0.03, **params):
    """Coarsest graph (CSR dict with weights) and its initial partition."""
    G = _G(g)
    p, keep = _params(params)
    n, nnz = G.n, len(G.adjncy)
    xc = np.zeros(n + 1, np.int32)
    ac = np.zeros(max(nnz, 1), np.int32)
    wc = np.zeros(max(nnz, 1), np.int32)
    vc = np.zeros(max(n, 1), np.int32)
    pc = np.zeros(max(n, 1), np.int32)
    nc, nnzc = ctypes.c_int32(), ctypes.c_int32()
    _load().orc_coarsest(G.ref, k, eps, ctypes.byref(p), _p32(xc), _p32(ac), _p32(wc), _p32(vc),
                         _p32(pc), ctypes.byref(nc), ctypes.byref(nnzc))
    nc, nnzc = nc.value, nnzc.value
    cg = {"xadj": xc[:nc + 1].copy(), "adjncy": ac[:nnzc].copy(), "adjwgt": wc[:nnzc].copy(),
          "vwgt": vc[:nc].copy()}
    return cg, pc[:nc].copy()


def partition(g, k, eps=0.03, **params):
    G = _G(g)
    p, keep = _params(params)
    P = np.zeros(G.n, np.int32)
    r = _Result()
    code = _load().orc_partition(G.ref, k, eps, ctypes.byref(p), _p32(P), ctypes.byref(r))
    res = {f: getattr(r, f) for f, _ in _Result._fields_}
    res["code"] = code
    return P, res
