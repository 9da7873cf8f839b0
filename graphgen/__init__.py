"""Seeded synthetic input graphs shared by the oracle and the GPU library.

The C implementation (``gen.c``) is compiled into ``libgraphgen.so`` by
``build_lib()``. Nothing here computes any step of the partitioner: this module
only produces symmetric int32 CSR inputs of the shapes of the paper's graph
families (random geometric graphs, see the paper's instance section) and of
the synthetic workloads (R-MAT, 3-D grids, batches of uneven graphs).

A graph is a dict of numpy arrays: ``xadj`` (int32, n+1), ``adjncy`` (int32,
nnz), optional ``adjwgt`` (int32, nnz) and ``vwgt`` (int32, n); absent weights
mean unit weights.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build_lib():
    """Compile gen.c with gcc/OpenMP into libgraphgen.so (always rebuilds)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, os.path.join(_HERE, "gen.c"), "-lm"])
    os.replace(tmp, _LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_lib()
    lib = ctypes.CDLL(_LIB_PATH)
    P32 = ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))
    lib.gg_rand.restype = ctypes.c_uint64
    lib.gg_rand.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_free.argtypes = [ctypes.c_void_p]
    lib.gg_rgg2d.restype = ctypes.c_int64
    lib.gg_rgg2d.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, P32, P32]
    lib.gg_rmat.restype = ctypes.c_int64
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, P32, P32]
    lib.gg_rmat_m.restype = ctypes.c_int64
    lib.gg_rmat_m.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_uint64, P32, P32]
    lib.gg_grid3d.restype = ctypes.c_int64
    lib.gg_grid3d.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                              ctypes.c_int32, P32, P32, P32]
    _lib = lib
    return lib


def _take(ptr, count):
    """Copy a malloc'ed int32 buffer into numpy and release it."""
    lib = _load()
    if count > 0:
        arr = np.ctypeslib.as_array(ptr, shape=(count,)).copy()
    else:
        arr = np.zeros(0, dtype=np.int32)
    lib.gg_free(ctypes.cast(ptr, ctypes.c_void_p))
    return arr


def rand_u64(seed, i):
    """i-th output of the counter-based splitmix64 stream `seed`."""
    return int(_load().gg_rand(seed, i))


def rgg_radius(n):
    """The paper's random geometric graph radius 0.55*sqrt(ln n / n)."""
    return 0.55 * math.sqrt(math.log(n) / n)


def rgg2d(n, seed, radius=None):
    lib = _load()
    r = rgg_radius(n) if radius is None else float(radius)
    px, pa = ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)()
    nnz = lib.gg_rgg2d(n, seed, r, ctypes.byref(px), ctypes.byref(pa))
    if nnz < 0:
        raise RuntimeError("gg_rgg2d failed")
    return {"xadj": _take(px, n + 1), "adjncy": _take(pa, nnz)}


def rmat(scale, seed, edge_factor=16, a=0.57, b=0.19, c=0.19):
    lib = _load()
    px, pa = ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)()
    nnz = lib.gg_rmat(scale, edge_factor, a, b, c, seed, ctypes.byref(px), ctypes.byref(pa))
    if nnz < 0:
        raise RuntimeError("gg_rmat failed")
    return {"xadj": _take(px, (1 << scale) + 1), "adjncy": _take(pa, nnz)}


def rmat_m(scale, m, seed, a=0.57, b=0.19, c=0.19):
    """R-MAT with exactly m edge draws (before symmetrisation and deduplication)."""
    lib = _load()
    px, pa = ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)()
    nnz = lib.gg_rmat_m(scale, m, a, b, c, seed, ctypes.byref(px), ctypes.byref(pa))
    if nnz < 0:
        raise RuntimeError("gg_rmat_m failed")
    return {"xadj": _take(px, (1 << scale) + 1), "adjncy": _take(pa, nnz)}


def _u01(seed, i):
    return (rand_u64(seed, i) >> 11) * (1.0 / 9007199254740992.0)


def batch(master_seed=4, count=512, log2_min=10, log2_max=18):
    """Batch of `count` uneven graphs: the first half 2-D random geometric, the
    second half R-MAT (.57,.19,.19,.05). Graph i draws u1,u2,u3 from the master
    stream (counters 3i..3i+2): n = floor(2^(lo+(hi-lo)u1)) (R-MAT: 2^round(..)),
    average degree d = 8 + 8 u2 (rgg radius sqrt(d/(pi n)); R-MAT draws d n / 2
    edges), k = (2, 8, 32)[floor(3 u3)]; graph seed = R(master, 3 count + i).
    Returns (list of CSR dicts, list of k)."""
    graphs, ks = [], []
    span = log2_max - log2_min
    for i in range(count):
        u1, u2, u3 = (_u01(master_seed, 3 * i + j) for j in range(3))
        d = 8.0 + 8.0 * u2
        k = (2, 8, 32)[min(2, int(3 * u3))]
        gseed = rand_u64(master_seed, 3 * count + i)
        if i < count // 2:
            n = int(math.floor(2.0 ** (log2_min + span * u1)))
            g = rgg2d(n, gseed, radius=math.sqrt(d / (math.pi * n)))
        else:
            scale = int(round(log2_min + span * u1))
            g = rmat_m(scale, int(round(d * (1 << scale) / 2)), gseed)
        graphs.append(g)
        ks.append(k)
    return graphs, ks


def grid3d(X, Y, Z, seed=3, wmax=10):
    lib = _load()
    px, pa, pw = (ctypes.POINTER(ctypes.c_int32)() for _ in range(3))
    nnz = lib.gg_grid3d(X, Y, Z, seed, wmax, ctypes.byref(px), ctypes.byref(pa), ctypes.byref(pw))
    if nnz < 0:
        raise RuntimeError("gg_grid3d failed")
    g = {"xadj": _take(px, X * Y * Z + 1), "adjncy": _take(pa, nnz)}
    if wmax > 0:
        g["adjwgt"] = _take(pw, nnz)
    else:
        lib.gg_free(ctypes.cast(pw, ctypes.c_void_p))
    return g


def random_small(n, p, seed, wmax=1, vmax=1):
    """Small Erdos-Renyi-style graph for property tests (numpy only).

    Edge {i,j} present iff U(seed, i*n+j) < p for i<j; weights drawn from the
    same stream family. Returns a CSR dict with explicit weights if w/vmax > 1.
    """
    rows = [[] for _ in range(n)]
    wts = [[] for _ in range(n)]
    for i in range(n):
        for j in range(i + 1, n):
            x = rand_u64(seed, i * n + j)
            if (x >> 11) * (1.0 / 9007199254740992.0) < p:
                w = 1 + (rand_u64(seed ^ 0x5151, i * n + j) % wmax) if wmax > 1 else 1
                rows[i].append(j); wts[i].append(w)
                rows[j].append(i); wts[j].append(w)
    xadj = np.zeros(n + 1, dtype=np.int32)
    adj, aw = [], []
    for v in range(n):
        order = np.argsort(rows[v], kind="stable")
        adj.extend(int(rows[v][o]) for o in order)
        aw.extend(int(wts[v][o]) for o in order)
        xadj[v + 1] = xadj[v] + len(rows[v])
    g = {"xadj": xadj, "adjncy": np.asarray(adj, dtype=np.int32)}
    if wmax > 1:
        g["adjwgt"] = np.asarray(aw, dtype=np.int32)
    if vmax > 1:
        g["vwgt"] = np.asarray([1 + rand_u64(seed ^ 0xA5A5, v) % vmax for v in range(n)],
                               dtype=np.int32)
    return g


def from_edges(n, edges, weights=None, vwgt=None):
    """CSR from an undirected edge list (for hand-made test graphs)."""
    rows = [dict() for _ in range(n)]
    for idx, (u, v) in enumerate(edges):
        if u == v:
            raise ValueError("self-loop")
        w = 1 if weights is None else int(weights[idx])
        rows[u][v] = w
        rows[v][u] = w
    xadj = np.zeros(n + 1, dtype=np.int32)
    adj, aw = [], []
    for v in range(n):
        for u in sorted(rows[v]):
            adj.append(u)
            aw.append(rows[v][u])
        xadj[v + 1] = xadj[v] + len(rows[v])
    g = {"xadj": xadj, "adjncy": np.asarray(adj, dtype=np.int32)}
    if weights is not None:
        g["adjwgt"] = np.asarray(aw, dtype=np.int32)
    if vwgt is not None:
        g["vwgt"] = np.asarray(vwgt, dtype=np.int32)
    return g
