"""MI355X (gfx950) size-constrained label-propagation graph partitioner.

Python binding of ``libgp.so`` (C ABI in ``include/gp.h``). This module only
marshals arguments: graphs are dicts of int32 torch tensors on the GPU
(``xadj``, ``adjncy``, optional ``adjwgt`` / ``vwgt``), outputs are torch
tensors the binding allocates, and the current torch stream is passed to the
library. Every step of the method runs in the library's HIP kernels; there is
no CPU fallback: if ``libgp.so`` is missing or no GPU is present the calls
raise.

Method: Akhremtsev, Sanders, Schulz, "High-Quality Shared-Memory Graph
Partitioning" (arXiv 1710.08231): size-constrained label propagation for
clustering (§III-A, §IV-A) and refinement (§III-C), contraction (§III-A,
§IV-A), projection (§III-C), inside the multilevel scheme of §III.
"""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libgp.so")
SOURCES = ["lp.hip", "contract.hip", "initpart.hip", "partition.hip", "batch.hip", "mpnn.hip", "mls.hip"]
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

GP_OK, GP_WARN_IMBALANCED = 0, 1

_lib = None


class GPError(RuntimeError):
    pass


def build():
    """Compile libgp.so for gfx950 with hipcc (always rebuilds)."""
    src = [os.path.join(_HERE, "csrc", f) for f in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I" + os.path.join(_ROOT, "include"), "-o", tmp, *src]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("xadj", ctypes.c_void_p),
                ("adjncy", ctypes.c_void_p), ("adjwgt", ctypes.c_void_p), ("vwgt", ctypes.c_void_p)]


class LPStats(ctypes.Structure):
    _fields_ = [("rounds_run", ctypes.c_int32), ("moves", ctypes.c_int64),
                ("edge_visits", ctypes.c_int64), ("ms", ctypes.c_float), ("workspace_bytes", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("rounds_coarsen", ctypes.c_int32), ("rounds_refine", ctypes.c_int32),
                ("coarsest_per_k", ctypes.c_int32), ("attempts", ctypes.c_int32),
                ("stall_num", ctypes.c_int32), ("stall_den", ctypes.c_int32),
                ("dir_alternate", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("init_mode", ctypes.c_int32), ("mpnn_max_n", ctypes.c_int32),
                ("mpnn_seed", ctypes.c_uint64), ("mpnn_params", ctypes.c_void_p), ("active_set", ctypes.c_int32),
                ("init_fm", ctypes.c_int32), ("mls", ctypes.c_int32), ("mls_batch", ctypes.c_int32),
                ("mls_queue", ctypes.c_int32)]


class MLSStats(ctypes.Structure):
    _fields_ = [("gain", ctypes.c_int64), ("searches", ctypes.c_int64), ("moves", ctypes.c_int64),
                ("local_iters", ctypes.c_int64), ("ms", ctypes.c_float), ("workspace_bytes", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("tier_max", ctypes.c_int32 * 4), ("dense_split", ctypes.c_int32), ("dense_chunk", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("cut", ctypes.c_int64), ("max_block_w", ctypes.c_int64), ("lmax", ctypes.c_int64),
                ("ucl", ctypes.c_int64), ("balanced", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("coarsest_n", ctypes.c_int32), ("n_isolated", ctypes.c_int32),
                ("edge_visits_cluster", ctypes.c_int64), ("edge_visits_refine", ctypes.c_int64),
                ("ms_coarsen", ctypes.c_float), ("ms_init", ctypes.c_float),
                ("ms_refine", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("learned_tried", ctypes.c_int32), ("learned_kept", ctypes.c_int32),
                ("plain_cut_coarsest", ctypes.c_int64), ("learned_cut_coarsest", ctypes.c_int64),
                ("mls_gain", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64)]


EXPORTS = ["gp_default_params", "gp_lmax", "gp_lp_cluster", "gp_lp_refine", "gp_contract",
           "gp_project", "gp_cut_and_blocks", "gp_partition", "gp_partition_batch", "gp_strerror", "gp_last_error", "gp_release_cache", "gp_get_tuning", "gp_set_tuning",
           "gp_profile_enable", "gp_profile_select", "gp_profile_reserve", "gp_profile_count", "gp_profile_get", "gp_coarsest", "gp_coarsest_batch",
           "gp_mpnn_param_count", "gp_mpnn_features", "gp_mpnn_forward", "gp_mpnn_decode", "gp_mpnn_backward", "gp_mpnn_adam_step",
           "gp_workspace_bytes", "gp_lp_refine_static", "gp_mls_refine"]


def load():
    """Load libgp.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GPError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    G = ctypes.POINTER(Graph)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.gp_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.gp_workspace_bytes.restype = ctypes.c_size_t
    lib.gp_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
    lib.gp_lmax.restype = i64
    lib.gp_lmax.argtypes = [i64, i32, ctypes.c_double]
    lib.gp_lp_cluster.argtypes = [G, i64, i32, i32, vp, ctypes.POINTER(LPStats), vp, ctypes.c_size_t, vp]
    lib.gp_lp_refine.argtypes = [G, i32, i64, i32, i32, vp, ctypes.POINTER(LPStats), vp, ctypes.c_size_t, vp]
    lib.gp_lp_refine_static.argtypes = [G, i32, i64, i32, i32, vp, ctypes.POINTER(LPStats), vp]
    lib.gp_mls_refine.argtypes = [G, i32, i64, vp, ctypes.c_uint64, i32, i32, i32, ctypes.POINTER(MLSStats), vp,
                                  ctypes.c_size_t, vp]
    lib.gp_contract.argtypes = [G, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, ctypes.c_size_t, vp]
    lib.gp_project.argtypes = [i32, vp, vp, vp, vp]
    lib.gp_cut_and_blocks.argtypes = [G, i32, vp, ctypes.POINTER(i64), vp, vp, ctypes.c_size_t, vp]
    lib.gp_partition.argtypes = [G, i32, ctypes.c_double, ctypes.POINTER(Params), vp,
                                 ctypes.POINTER(Result), vp, ctypes.c_size_t, vp]
    lib.gp_partition_batch.argtypes = [G, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.c_double,
                                       ctypes.POINTER(Params), vp, ctypes.POINTER(Result), vp, ctypes.c_size_t, vp]
    lib.gp_coarsest.argtypes = [G, i32, ctypes.c_double, ctypes.POINTER(Params), vp, vp, vp, vp, vp,
                                ctypes.POINTER(i32), ctypes.POINTER(i32), vp, ctypes.c_size_t, vp]
    lib.gp_coarsest_batch.argtypes = [G, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.c_double,
                                      ctypes.POINTER(Params), vp, vp, vp, vp, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(i32), vp, ctypes.c_size_t, vp]
    lib.gp_mpnn_param_count.restype = i32
    lib.gp_mpnn_param_count.argtypes = [i32]
    lib.gp_mpnn_features.argtypes = [G, ctypes.c_uint64, vp, vp, ctypes.c_size_t, vp]
    lib.gp_mpnn_forward.argtypes = [G, i32, vp, ctypes.c_uint64, vp, vp, vp, ctypes.c_size_t, vp]
    lib.gp_mpnn_decode.argtypes = [G, i32, vp, i64, vp, vp, ctypes.c_size_t, vp]
    lib.gp_mpnn_backward.argtypes = [G, i32, vp, ctypes.c_uint64, vp, ctypes.c_float, vp,
                                     ctypes.POINTER(ctypes.c_double), vp, ctypes.c_size_t, vp]
    lib.gp_mpnn_adam_step.argtypes = [vp, vp, vp, vp, i32, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, vp]
    lib.gp_release_cache.argtypes = []
    lib.gp_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.gp_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.gp_strerror.restype = ctypes.c_char_p
    lib.gp_strerror.argtypes = [ctypes.c_int]
    lib.gp_last_error.restype = ctypes.c_char_p
    lib.gp_last_error.argtypes = []
    lib.gp_profile_enable.argtypes = [ctypes.c_int]
    lib.gp_profile_select.argtypes = [ctypes.c_char_p]
    lib.gp_profile_reserve.argtypes = [ctypes.c_int]
    lib.gp_profile_count.restype = ctypes.c_int
    lib.gp_profile_get.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(i64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        lib = load()
        raise GPError(f"{lib.gp_strerror(rc).decode()} ({rc}): {lib.gp_last_error().decode()}")
    return rc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise GPError("no GPU: the partitioner runs only on the MI355X")
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ws(ws):
    """(pointer, bytes) of a caller workspace (a contiguous CUDA tensor), or (NULL, 0): the library cache."""
    if ws is None:
        return None, 0
    if not ws.is_cuda or not ws.is_contiguous():
        raise GPError("ws must be a contiguous CUDA tensor")
    return ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _gstruct(g):
    torch = _torch()
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        t = g.get(key)
        if t is not None and (t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous()):
            raise GPError(f"graph['{key}'] must be a contiguous int32 CUDA tensor")
    n = g["xadj"].numel() - 1
    nnz = g["adjncy"].numel()
    return Graph(n, nnz, _ptr(g["xadj"]), _ptr(g["adjncy"]), _ptr(g.get("adjwgt")), _ptr(g.get("vwgt")))


def to_device(g, device="cuda"):
    """numpy CSR dict -> dict of int32 CUDA tensors (inputs resident in HBM)."""
    torch = _torch()
    out = {}
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        if g.get(key) is not None:
            out[key] = torch.from_numpy(g[key]).to(device=device, dtype=torch.int32).contiguous()
    return out


OP_LP_CLUSTER, OP_LP_REFINE, OP_CONTRACT, OP_CUT = 1, 2, 3, 4


def workspace_bytes(op, n, nnz, k=1, flags=1):
    """Workspace size that always suffices for one call of kind `op` (gp_workspace_bytes)."""
    lib = load()
    b = int(lib.gp_workspace_bytes(op, n, nnz, k, flags))
    if b == 0:
        raise GPError(lib.gp_last_error().decode())
    return b


def lmax(total_vwgt, k, eps):
    return int(load().gp_lmax(total_vwgt, k, eps))


def default_params():
    p = Params()
    load().gp_default_params(ctypes.byref(p))
    return p


LP_DIR_ALTERNATE, LP_ACTIVE_SET = 1, 2


def _lp_flags(dir_alternate, active):
    return (LP_DIR_ALTERNATE if dir_alternate else 0) | (LP_ACTIVE_SET if active else 0)


def lp_cluster(g, U, rounds=10, dir_alternate=1, active=False, ws=None):
    torch = _torch()
    gs = _gstruct(g)
    labels = torch.empty(gs.n, dtype=torch.int32, device=g["xadj"].device)
    st = LPStats()
    _check(load().gp_lp_cluster(ctypes.byref(gs), U, rounds, _lp_flags(dir_alternate, active), _ptr(labels),
                                ctypes.byref(st), *_ws(ws), _stream()))
    return labels, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits, "ms": st.ms,
                    "workspace_bytes": st.workspace_bytes}


def lp_refine(g, part, k, lmax_, rounds=25, dir_alternate=1, active=False, ws=None):
    torch = _torch()
    gs = _gstruct(g)
    P = part.to(dtype=torch.int32).clone().contiguous()
    st = LPStats()
    _check(load().gp_lp_refine(ctypes.byref(gs), k, lmax_, rounds, _lp_flags(dir_alternate, active), _ptr(P),
                               ctypes.byref(st), *_ws(ws), _stream()))
    return P, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits, "ms": st.ms,
               "workspace_bytes": st.workspace_bytes}


def lp_refine_static(g, part, k, lmax_, rounds=25, dir_alternate=1, active=False):
    """gp_lp_refine on the library's static scratch (gp_lp_refine_static): no allocation."""
    torch = _torch()
    gs = _gstruct(g)
    P = part.to(dtype=torch.int32).clone().contiguous()
    st = LPStats()
    _check(load().gp_lp_refine_static(ctypes.byref(gs), k, lmax_, rounds, _lp_flags(dir_alternate, active), _ptr(P),
                                      ctypes.byref(st), _stream()))
    return P, {"rounds_run": st.rounds_run, "moves": st.moves, "edge_visits": st.edge_visits, "ms": st.ms,
               "workspace_bytes": st.workspace_bytes}


def mls_refine(g, part, k, lmax_, seed=0, global_iters=3, batch=1, queue=64, ws=None):
    """Multi-try k-way local search from a partition (gp_mls_refine); returns (part', stats)."""
    torch = _torch()
    gs = _gstruct(g)
    P = part.to(dtype=torch.int32).clone().contiguous()
    st = MLSStats()
    _check(load().gp_mls_refine(ctypes.byref(gs), k, lmax_, _ptr(P), seed, global_iters, batch, queue,
                                ctypes.byref(st), *_ws(ws), _stream()))
    return P, {f: getattr(st, f) for f, _ in MLSStats._fields_}


def contract(g, labels, ws=None):
    torch = _torch()
    gs = _gstruct(g)
    dev = g["xadj"].device
    xc = torch.empty(gs.n + 1, dtype=torch.int32, device=dev)
    ac = torch.empty(max(gs.nnz, 1), dtype=torch.int32, device=dev)
    wc = torch.empty(max(gs.nnz, 1), dtype=torch.int32, device=dev)
    vc = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    f2c = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    nc, nnzc = ctypes.c_int32(), ctypes.c_int32()
    lab = labels.to(dtype=torch.int32).contiguous()
    _check(load().gp_contract(ctypes.byref(gs), _ptr(lab), _ptr(xc), _ptr(ac), _ptr(wc), _ptr(vc), _ptr(f2c),
                              ctypes.byref(nc), ctypes.byref(nnzc), *_ws(ws), _stream()))
    nc, nnzc = nc.value, nnzc.value
    cg = {"xadj": xc[:nc + 1], "adjncy": ac[:nnzc], "adjwgt": wc[:nnzc], "vwgt": vc[:nc]}
    return cg, f2c[:gs.n]


def project(f2c, part_coarse):
    torch = _torch()
    out = torch.empty_like(f2c)
    _check(load().gp_project(f2c.numel(), _ptr(f2c), _ptr(part_coarse.contiguous()), _ptr(out), _stream()))
    return out


def cut_and_blocks(g, part, k, ws=None):
    torch = _torch()
    gs = _gstruct(g)
    B = torch.empty(k, dtype=torch.int64, device=g["xadj"].device)
    cut = ctypes.c_int64()
    _check(load().gp_cut_and_blocks(ctypes.byref(gs), k, _ptr(part.contiguous()), ctypes.byref(cut), _ptr(B),
                                    *_ws(ws), _stream()))
    return cut.value, B


def _params(params):
    """gp_params from keyword overrides; mpnn_params is a float32 CUDA tensor (kept alive by the caller)."""
    torch = _torch()
    p = default_params()
    for key, val in params.items():
        if key == "mpnn_params":
            if val is not None and (val.dtype != torch.float32 or not val.is_cuda or not val.is_contiguous()):
                raise GPError("mpnn_params must be a contiguous float32 CUDA tensor")
            val = None if val is None else val.data_ptr()
        setattr(p, key, val)
    return p


def partition(g, k, eps=0.03, ws=None, **params):
    torch = _torch()
    gs = _gstruct(g)
    p = _params(params)
    part = torch.empty(max(gs.n, 1), dtype=torch.int32, device=g["xadj"].device)
    r = Result()
    code = _check(load().gp_partition(ctypes.byref(gs), k, eps, ctypes.byref(p), _ptr(part), ctypes.byref(r),
                                      *_ws(ws), _stream()))
    res = {f: getattr(r, f) for f, _ in Result._fields_}
    res["code"] = code
    return part[:gs.n], res


def union_graph(graphs):
    """Disjoint union of numpy CSR graphs -> (numpy CSR dict, vtx_off list). Input plumbing only."""
    import numpy as np
    xs, adj, aw, vw, off, eoff = [np.zeros(1, np.int32)], [], [], [], [0], 0
    any_w = any(g.get("adjwgt") is not None for g in graphs)
    any_v = any(g.get("vwgt") is not None for g in graphs)
    for g in graphs:
        n = len(g["xadj"]) - 1
        xs.append((g["xadj"][1:] + eoff).astype(np.int32))
        adj.append((g["adjncy"] + off[-1]).astype(np.int32))
        if any_w:
            aw.append(g["adjwgt"] if g.get("adjwgt") is not None else np.ones(len(g["adjncy"]), np.int32))
        if any_v:
            vw.append(g["vwgt"] if g.get("vwgt") is not None else np.ones(n, np.int32))
        off.append(off[-1] + n)
        eoff += len(g["adjncy"])
    u = {"xadj": np.concatenate(xs).astype(np.int32),
         "adjncy": np.concatenate(adj).astype(np.int32) if adj else np.zeros(0, np.int32)}
    if any_w:
        u["adjwgt"] = np.concatenate(aw).astype(np.int32)
    if any_v:
        u["vwgt"] = np.concatenate(vw).astype(np.int32)
    return u, off


def partition_batch(g, vtx_off, ks, eps=0.03, ws=None, **params):
    """Partition the graphs of a disjoint-union graph together (see gp_partition_batch)."""
    torch = _torch()
    gs = _gstruct(g)
    G = len(ks)
    p = _params(params)
    part = torch.empty(max(gs.n, 1), dtype=torch.int32, device=g["xadj"].device)
    off = (ctypes.c_int32 * (G + 1))(*vtx_off)
    kk = (ctypes.c_int32 * G)(*ks)
    res = (Result * G)()
    code = _check(load().gp_partition_batch(ctypes.byref(gs), G, off, kk, eps, ctypes.byref(p), _ptr(part), res,
                                            *_ws(ws), _stream()))
    out = []
    for r in res:
        d = {f: getattr(r, f) for f, _ in Result._fields_}
        out.append(d)
    return part[:gs.n], out, code


def coarsest(g, k, eps=0.03, ws=None, **params):
    """Coarsest graph of the hierarchy (CSR dict of device tensors) and its initial partition."""
    torch = _torch()
    gs = _gstruct(g)
    p = _params(params)
    dev = g["xadj"].device
    xc = torch.empty(gs.n + 1, dtype=torch.int32, device=dev)
    ac = torch.empty(max(gs.nnz, 1), dtype=torch.int32, device=dev)
    wc = torch.empty(max(gs.nnz, 1), dtype=torch.int32, device=dev)
    vc = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    pc = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    nc, nnzc = ctypes.c_int32(), ctypes.c_int32()
    _check(load().gp_coarsest(ctypes.byref(gs), k, eps, ctypes.byref(p), _ptr(xc), _ptr(ac), _ptr(wc), _ptr(vc),
                              _ptr(pc), ctypes.byref(nc), ctypes.byref(nnzc), *_ws(ws), _stream()))
    nc, nnzc = nc.value, nnzc.value
    return {"xadj": xc[:nc + 1], "adjncy": ac[:nnzc], "adjwgt": wc[:nnzc], "vwgt": vc[:nc]}, pc[:nc]


def coarsest_batch(g, vtx_off, ks, eps=0.03, ws=None, **params):
    """Coarsest graphs of the graphs of a disjoint-union graph, side by side.
    Returns (CSR dict of device tensors, coarse vertex offsets [G+1], graph-local partition)."""
    torch = _torch()
    gs = _gstruct(g)
    G = len(ks)
    p = _params(params)
    dev = g["xadj"].device
    xc = torch.empty(gs.n + 1, dtype=torch.int32, device=dev)
    ac = torch.empty(max(gs.nnz, 1), dtype=torch.int32, device=dev)
    wc = torch.empty(max(gs.nnz, 1), dtype=torch.int32, device=dev)
    vc = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    pc = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    off = (ctypes.c_int32 * (G + 1))(*vtx_off)
    kk = (ctypes.c_int32 * G)(*ks)
    offc = (ctypes.c_int32 * (G + 1))()
    nnzc = ctypes.c_int32()
    _check(load().gp_coarsest_batch(ctypes.byref(gs), G, off, kk, eps, ctypes.byref(p), _ptr(xc), _ptr(ac), _ptr(wc),
                                    _ptr(vc), _ptr(pc), offc, ctypes.byref(nnzc), *_ws(ws), _stream()))
    nc, nnzc = offc[G], nnzc.value
    cg = {"xadj": xc[:nc + 1], "adjncy": ac[:nnzc], "adjwgt": wc[:nnzc], "vwgt": vc[:nc]}
    return cg, list(offc), pc[:nc]


def mpnn_param_count(k):
    n = int(load().gp_mpnn_param_count(k))
    if n < 0:
        raise GPError("the network's head supports 1 <= k <= 64")
    return n


def _fparams(params, k):
    torch = _torch()
    if params.dtype != torch.float32 or not params.is_cuda or not params.is_contiguous():
        raise GPError("params must be a contiguous float32 CUDA tensor")
    if params.numel() != mpnn_param_count(k):
        raise GPError(f"params must hold {mpnn_param_count(k)} floats for k={k}")
    return _ptr(params)


def mpnn_features(g, seed=0, ws=None):
    torch = _torch()
    gs = _gstruct(g)
    X = torch.empty((max(gs.n, 1), 18), dtype=torch.float32, device=g["xadj"].device)
    _check(load().gp_mpnn_features(ctypes.byref(gs), seed, _ptr(X), *_ws(ws), _stream()))
    return X[:gs.n]


def mpnn_forward(g, k, params, seed=0, ws=None):
    """(logits [n, k], argmax blocks [n]) of the network with bfloat16-rounded weights."""
    torch = _torch()
    gs = _gstruct(g)
    dev = g["xadj"].device
    Z = torch.empty((max(gs.n, 1), k), dtype=torch.float32, device=dev)
    P = torch.empty(max(gs.n, 1), dtype=torch.int32, device=dev)
    _check(load().gp_mpnn_forward(ctypes.byref(gs), k, _fparams(params, k), seed, _ptr(Z), _ptr(P), *_ws(ws), _stream()))
    return Z[:gs.n], P[:gs.n]


def mpnn_decode(g, k, Z, lmax_, ws=None):
    """Blocks [n] from logits Z [n, k] (float32 CUDA) under the block bound lmax_."""
    torch = _torch()
    gs = _gstruct(g)
    z = Z.to(dtype=torch.float32).contiguous()
    if z.numel() != gs.n * k:
        raise GPError("Z must hold n * k logits")
    P = torch.empty(max(gs.n, 1), dtype=torch.int32, device=g["xadj"].device)
    _check(load().gp_mpnn_decode(ctypes.byref(gs), k, _ptr(z), lmax_, _ptr(P), *_ws(ws), _stream()))
    return P[:gs.n]


def mpnn_backward(g, k, params, target, seed=0, lam=1.0, grad=None, ws=None):
    """(gradient [P] float32, (edge loss, balance loss)) for a target partition."""
    torch = _torch()
    gs = _gstruct(g)
    if grad is None:
        grad = torch.empty(mpnn_param_count(k), dtype=torch.float32, device=params.device)
    t = target.to(dtype=torch.int32).contiguous()
    loss = (ctypes.c_double * 2)()
    _check(load().gp_mpnn_backward(ctypes.byref(gs), k, _fparams(params, k), seed, _ptr(t), lam, _ptr(grad), loss,
                                   *_ws(ws), _stream()))
    return grad, (loss[0], loss[1])


def mpnn_adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of params in place (m, v: moment tensors of the same size)."""
    for t in (params, m, v, grad):
        if t.numel() != params.numel() or not t.is_contiguous():
            raise GPError("params, m, v and grad must be contiguous and of one size")
    _check(load().gp_mpnn_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), step, lr, beta1,
                                    beta2, eps, _stream()))


def get_tuning():
    """Current LP execution thresholds as a dict."""
    t = Tuning()
    load().gp_get_tuning(ctypes.byref(t))
    return {"tier_max": list(t.tier_max), "dense_split": t.dense_split, "dense_chunk": t.dense_chunk}


def set_tuning(tuning=None):
    """Set the LP execution thresholds (dict as from get_tuning; None restores the defaults)."""
    lib = load()
    if tuning is None:
        _check(lib.gp_set_tuning(None))
        return
    t = Tuning((ctypes.c_int32 * 4)(*tuning["tier_max"]), tuning["dense_split"], tuning["dense_chunk"])
    _check(lib.gp_set_tuning(ctypes.byref(t)))


def release_cache():
    """Free the device memory the library keeps for reuse between calls."""
    _check(load().gp_release_cache())


PROFILE_KERNELS, PROFILE_BY_LEVEL, PROFILE_EAGER, PROFILE_CALLS = 1, 2, 4, 8


def profile_enable(mode=PROFILE_KERNELS):
    """Start (clearing) or stop (mode 0 / False) the library's HIP-event timing; mode is a
    combination of the PROFILE_* bits (True = PROFILE_KERNELS)."""
    load().gp_profile_enable(int(mode))


def profile_select(name=None):
    """Record only launches of kernel `name` (None: all)."""
    load().gp_profile_select(None if name is None else name.encode())


def profile_reserve(launches):
    """Pre-create the events of `launches` recorded launches (none are created while timing)."""
    _check(load().gp_profile_reserve(int(launches)))


def profile_entries():
    """[{name, launches, ms, bytes}] accumulated since profile_enable(True)."""
    lib = load()
    out = []
    buf = ctypes.create_string_buffer(256)
    for i in range(lib.gp_profile_count()):
        n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib.gp_profile_get(i, buf, 256, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)))
        out.append({"name": buf.value.decode(), "launches": n.value, "ms": ms.value, "bytes": b.value})
    return out
