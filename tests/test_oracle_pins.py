"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here calls the GPU library. Every check uses a route other than the
oracle's own loops: hand-derived worked vectors (tests/golden), closed forms
(L_max, the matrix form of contraction A' = offdiag(S^T A S), c' = S^T c),
invariants the method guarantees (size constraint, weight conservation,
direction alternation, strict gain, prefix admission), brute force on tiny
graphs, and the published splitmix64 output sequence.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "lp_worked_vectors.json")) as f:
        return json.load(f)


def _adj(g):
    n = len(g["xadj"]) - 1
    w = g.get("adjwgt")
    data = np.ones(len(g["adjncy"]), np.int64) if w is None else w.astype(np.int64)
    return sp.csr_matrix((data, g["adjncy"], g["xadj"]), shape=(n, n))


def _vw(g):
    n = len(g["xadj"]) - 1
    return np.ones(n, np.int64) if g.get("vwgt") is None else g["vwgt"].astype(np.int64)


# ---------------------------------------------------------------- worked vectors

@pytest.mark.parametrize("case", _golden()["cases"], ids=lambda c: c["name"])
def test_worked_lp_vectors(case):
    g = graphgen.from_edges(case["n"], case["edges"], vwgt=case.get("vwgt"))
    if case["mode"] == "cluster":
        lab, st = oracle.lp_cluster(g, case["U"], case["rounds"])
    else:
        lab, st = oracle.lp_refine(g, case["part_in"], case["k"], case["lmax"], case["rounds"])
    assert lab.tolist() == case["labels"]
    assert st["rounds_run"] == case["rounds_run"]
    assert st["moves"] == case["moves"]
    assert st["edge_visits"] == case["rounds_run"] * len(g["adjncy"])


@pytest.mark.parametrize("case", _golden()["contractions"], ids=lambda c: c["name"])
def test_worked_contractions(case):
    g = graphgen.from_edges(case["n"], case["edges"])
    cg, f2c = oracle.contract(g, case["labels"])
    assert f2c.tolist() == case["f2c"]
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert cg[key].tolist() == case[key], key


# ---------------------------------------------------------------- closed forms

def test_lmax_values():
    # (1+eps)*ceil(W/k) for the workloads: rgg n=2^14 k=2; R-MAT/grid n=2^24, 2^22 with k=64, 16
    assert oracle.lmax(16384, 2, 0.03) == 8437
    assert oracle.lmax(1 << 24, 64, 0.03) == 270008
    assert oracle.lmax(1 << 22, 16, 0.03) == 270008
    assert oracle.lmax(1 << 24, 16, 0.03) == 1080033
    assert oracle.lmax(1024, 32, 0.03) == 32
    assert oracle.lmax(7, 7, 0.0) == 1
    assert oracle.lmax(8, 3, 0.5) == 4  # ceil(8/3)=3, 1.5*3=4.5 -> 4


def test_lmax_matches_exact_rational_for_three_percent():
    # floor(1.03 * q) in binary64 equals the exact floor(103 q / 100) on this range
    qs = np.arange(1, 2_000_001, 997, dtype=np.int64)
    for q in qs.tolist():
        assert oracle.lmax(q, 1, 0.03) == (103 * q) // 100


def test_splitmix64_published_sequence():
    # First outputs of splitmix64 started at state 0 (Steele, Lea & Flood 2014 / Vigna's reference code)
    expected = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [graphgen.rand_u64(0, i) for i in range(3)] == expected
    # the oracle's start-vertex hash is the chained finaliser: mix4 starts with output 0 of state 0
    assert oracle.mix4(0, 0, 0, 0) != oracle.mix4(0, 0, 0, 1)


# ---------------------------------------------------------------- LP round: independent vectorised form

def _round_vectorised(g, C, W, U, r):
    """Same round via sparse products, masked argmax and a sort + cumsum admission."""
    A = _adj(g)
    n = A.shape[0]
    nl = len(W)
    c = _vw(g)
    H = sp.csr_matrix((np.ones(n, np.int64), (np.arange(n), C)), shape=(n, nl))
    conn = (A @ H).toarray()
    own = conn[np.arange(n), C]
    labels = np.arange(nl)[None, :]
    mask = (conn > 0) & (labels != C[:, None])
    mask &= (labels < C[:, None]) if r % 2 == 0 else (labels > C[:, None])
    mask &= (W[None, :] + c[:, None]) <= U
    masked = np.where(mask, conn, -1)
    best = masked.argmax(axis=1)  # first maximum = smallest label
    bconn = masked[np.arange(n), best]
    prop = np.where((bconn > 0) & (bconn > own), best, -1)
    movers = np.nonzero(prop >= 0)[0]
    order = np.lexsort((movers, prop[movers]))
    mv = movers[order]
    tgt = prop[mv]
    cs = np.cumsum(c[mv])
    starts = np.r_[0, np.nonzero(np.diff(tgt))[0] + 1] if len(mv) else np.zeros(0, int)
    seg_base = np.zeros(len(mv), np.int64)
    for s, e in zip(starts, list(starts[1:]) + [len(mv)]):
        seg_base[s:e] = cs[s - 1] if s > 0 else 0
    ok = W[tgt] + (cs - seg_base) <= U
    C2, W2 = C.copy(), W.copy()
    for v, t in zip(mv[ok], tgt[ok]):
        W2[t] += c[v]
        W2[C2[v]] -= c[v]
        C2[v] = t
    return C2, W2, int(ok.sum()), prop


def _random_graphs():
    out = []
    for seed in range(12):
        n = 8 + (seed * 7) % 40
        p = [0.08, 0.2, 0.5][seed % 3]
        out.append((seed, graphgen.random_small(n, p, seed, wmax=1 + seed % 4, vmax=1 + seed % 3)))
    return out


@pytest.mark.parametrize("seed,g", _random_graphs(), ids=lambda x: str(x) if isinstance(x, int) else "")
def test_lp_rounds_match_vectorised_form_and_invariants(seed, g):
    n = len(g["xadj"]) - 1
    c = _vw(g)
    A = _adj(g)
    U = int(c.max()) + seed % 5 + 1
    C = np.arange(n, dtype=np.int32)
    W = c.copy()
    for r in range(10):
        C1, W1, m1, p1 = oracle.lp_round(g, C, W, U, r)
        C2, W2, m2, p2 = _round_vectorised(g, C.astype(np.int64), W.astype(np.int64), U, r)
        assert p1.tolist() == p2.tolist()
        assert C1.tolist() == C2.tolist() and W1.tolist() == W2.tolist() and m1 == m2
        # invariants
        assert (W1 <= U).all()
        assert W1.sum() == c.sum()
        assert np.array_equal(np.bincount(C1, weights=c, minlength=n).astype(np.int64), W1)
        moved = np.nonzero(C1 != C)[0]
        for v in moved:
            nb = g["adjncy"][g["xadj"][v]:g["xadj"][v + 1]]
            assert C1[v] in set(C[nb].tolist())  # a move goes to a label held by a neighbour
            assert (C1[v] < C[v]) if r % 2 == 0 else (C1[v] > C[v])
            row = A.getrow(v)
            conn_new = sum(int(w) for u, w in zip(row.indices, row.data) if C[u] == C1[v])
            conn_old = sum(int(w) for u, w in zip(row.indices, row.data) if C[u] == C[v])
            assert conn_new > conn_old
        if (p1 >= 0).any():
            assert m1 >= 1  # the first proposer to any target always fits
        C, W = C1, W1


def test_lp_cluster_stops_after_two_idle_rounds():
    g = graphgen.rgg2d(400, 11)
    lab, st = oracle.lp_cluster(g, 30, rounds=50)
    assert st["rounds_run"] < 50
    # continuing from the fixed point moves nothing in either direction
    c = _vw(g)
    W = np.bincount(lab, weights=c, minlength=len(lab)).astype(np.int64)
    for r in (0, 1):
        _, _, m, _ = oracle.lp_round(g, lab, W, 30, r)
        assert m == 0


# ---------------------------------------------------------------- contraction: matrix closed form

@pytest.mark.parametrize("seed", range(8))
def test_contract_equals_offdiag_StAS(seed):
    g = graphgen.random_small(30 + seed * 5, 0.15, 100 + seed, wmax=5, vmax=4)
    n = len(g["xadj"]) - 1
    U = 6 + seed
    lab, _ = oracle.lp_cluster(g, U, 10)
    cg, f2c = oracle.contract(g, lab)
    nc = len(cg["xadj"]) - 1
    used = np.unique(lab)
    assert nc == len(used)
    assert f2c.tolist() == np.searchsorted(used, lab).tolist()  # rank among used labels
    S = sp.csr_matrix((np.ones(n, np.int64), (np.arange(n), f2c)), shape=(n, nc))
    A = _adj(g)
    Ac = (S.T @ A @ S).tolil()
    Ac.setdiag(0)
    Ac = sp.csr_matrix(Ac)
    Ac.eliminate_zeros()
    Ac.sort_indices()
    assert cg["xadj"].tolist() == Ac.indptr.tolist()
    assert cg["adjncy"].tolist() == Ac.indices.tolist()
    assert cg["adjwgt"].tolist() == Ac.data.tolist()
    assert cg["vwgt"].tolist() == (S.T @ _vw(g)).tolist()
    # conservation: sum w' = sum w - intra-cluster weight (both directions)
    intra = sum(int(w) for v in range(n) for u, w in zip(A.getrow(v).indices, A.getrow(v).data)
                if f2c[u] == f2c[v])
    assert int(cg["adjwgt"].sum()) == int(A.sum()) - intra


@pytest.mark.parametrize("seed", range(6))
def test_projection_preserves_cut_and_balance(seed):
    # §III-A: a partition of the coarse graph corresponds to one of the fine graph with equal cut and balance
    g = graphgen.random_small(60, 0.1, 200 + seed, wmax=4, vmax=3)
    lab, _ = oracle.lp_cluster(g, 8, 10)
    cg, f2c = oracle.contract(g, lab)
    nc = len(cg["xadj"]) - 1
    k = 3
    pc = np.array([graphgen.rand_u64(seed, i) % k for i in range(nc)], np.int32)
    pf = oracle.project(f2c, pc)
    assert oracle.cut(g, pf) == oracle.cut(cg, pc)
    assert oracle.block_weights(g, pf, k).tolist() == oracle.block_weights(cg, pc, k).tolist()


def test_cut_closed_form():
    g = graphgen.random_small(40, 0.2, 7, wmax=6)
    A = _adj(g)
    part = np.array([graphgen.rand_u64(3, i) % 4 for i in range(40)], np.int32)
    diff = part[:, None] != part[None, :]
    assert oracle.cut(g, part) == int((A.toarray() * diff).sum()) // 2


# ---------------------------------------------------------------- initial partition pieces

@pytest.mark.parametrize("n,k", [(17, 2), (64, 4), (100, 3), (37, 5), (1000, 16), (5, 8)])
def test_bisection_block_weights_unit(n, k):
    # unit weights: the grown side weighs exactly ceil(c(S)*ceil(k_S/2)/k_S)
    g = graphgen.rgg2d(n, 5) if n > 8 else graphgen.from_edges(n, [(i, i + 1) for i in range(n - 1)])

    def expect(size, ks):
        if ks == 1:
            return [size]
        kl = (ks + 1) // 2
        left = min(size, -(-size * kl // ks))
        return expect(left, kl) + expect(size - left, ks - kl)

    P = oracle.recursive_bisection(g, k, seed=1, attempt=0)
    assert np.bincount(P, minlength=k).tolist() == expect(n, k)


def test_bisection_left_side_is_connected():
    g = graphgen.grid3d(20, 20, 5, wmax=0)
    A = _adj(g)
    ncomp, _ = sp.csgraph.connected_components(A, directed=False)
    assert ncomp == 1
    for a in range(4):
        P = oracle.recursive_bisection(g, 2, seed=9, attempt=a)
        sub = A[P == 0][:, P == 0]
        assert sp.csgraph.connected_components(sub, directed=False)[0] == 1


def test_rebalance_worked_example():
    # path 0-1-2-3, P=[0,0,0,1], L_max=2: gains to block 1 are -1 (v0), -2 (v1), 0 (v2) -> move v2
    g = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    P, bal = oracle.rebalance(g, 2, 2, [0, 0, 0, 1])
    assert P.tolist() == [0, 0, 1, 1] and bal


def test_rebalance_ties_and_recomputed_gains():
    # edges 0-1, 2-3 inside block 0; P = [0,0,0,0,1,2], k = 3, L_max = 2 (B = [4,1,1]).
    # step 1: every vertex of block 0 has gain -1 to blocks 1 and 2 -> lowest vertex,
    #         lowest block: v0 -> 1 (B = [3,2,1]).
    # step 2: v1 now has gain 0 to block 2 (its neighbour left block 0; block 1 is full),
    #         v2, v3 have -1 -> v1 -> 2 (B = [2,2,2]).
    g = graphgen.from_edges(6, [(0, 1), (2, 3)])
    P, bal = oracle.rebalance(g, 3, 2, [0, 0, 0, 0, 1, 2])
    assert P.tolist() == [1, 2, 0, 0, 1, 2] and bal


def test_rebalance_room_is_at_most_lmax():
    # vwgt [2,1,1,1], edges 0-3 (w 1) and 1-2 (w 5), P = [0,0,0,1], L_max = 3 (B = [4,1]):
    # v0 -> 1 has gain 1 and fills block 1 exactly (1 + 2 = 3 <= 3); v1, v2 would lose 5
    g = graphgen.from_edges(4, [(0, 3), (1, 2)], weights=[1, 5], vwgt=[2, 1, 1, 1])
    P, bal = oracle.rebalance(g, 2, 3, [0, 0, 0, 1])
    assert P.tolist() == [1, 0, 0, 1] and bal


def test_fill_isolated_worked_example():
    # 0-1-2 placed (B = [2,1,0]); isolated 3 (weight 2), 4, 5 in ascending order into the
    # lightest block, ties to the lowest: 3 -> 2 (B = [2,1,2]), 4 -> 1 (B = [2,2,2]),
    # 5 -> 0 (B = [3,2,2]). Descending order or ties to the highest block differ.
    g = graphgen.from_edges(6, [(0, 1), (1, 2)], vwgt=[1, 1, 1, 2, 1, 1])
    part = np.array([0, 0, 1, -1, -1, -1], np.int32)
    P, B = oracle.fill_isolated(g, 3, part, np.array([2, 1, 0], np.int64))
    assert P.tolist() == [0, 0, 1, 2, 1, 0]
    assert B.tolist() == [3, 2, 2]


def test_rebalance_flags_infeasible():
    g = graphgen.from_edges(3, [(0, 1), (1, 2)], vwgt=[5, 1, 1])
    P, bal = oracle.rebalance(g, 2, 4, [0, 1, 1])
    assert not bal


def test_fill_isolated_bound_unit_weights():
    # lightest block holds at most ceil(W/k)-1 before each insertion -> max B <= max(B_before, ceil(W/k))
    n, k = 50, 7
    g = graphgen.from_edges(n, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)])
    part = np.full(n, -1, np.int32)
    part[:6] = [0, 0, 0, 0, 1, 1]
    B = np.zeros(k, np.int64)
    B[0], B[1] = 4, 2
    P, B2 = oracle.fill_isolated(g, k, part, B)
    assert (P >= 0).all() and B2.sum() == n
    assert B2.max() <= max(4, -(-n // k))
    assert np.bincount(P, minlength=k).tolist() == B2.tolist()


# ---------------------------------------------------------------- full partition vs brute force

def _brute_force_cut(g, k, lmax):
    n = len(g["xadj"]) - 1
    c = _vw(g)
    A = _adj(g).toarray()
    best = None
    for bits in itertools.product(range(k), repeat=n - 1):
        part = np.array((0,) + bits)
        if np.bincount(part, weights=c, minlength=k).max() > lmax:
            continue
        cut = int((A * (part[:, None] != part[None, :])).sum()) // 2
        best = cut if best is None else min(best, cut)
    return best


@pytest.mark.parametrize("seed", range(6))
def test_partition_balanced_and_not_below_optimum(seed):
    n = 10 + seed
    g = graphgen.random_small(n, 0.3, 300 + seed, wmax=3)
    P, res = oracle.partition(g, 2, 0.03, seed=seed)
    lm = oracle.lmax(n, 2, 0.03)
    opt = _brute_force_cut(g, 2, lm)
    assert res["balanced"] == 1 and res["code"] == 0
    assert res["cut"] == oracle.cut(g, P) >= opt
    assert np.bincount(P, minlength=2).max() <= lm


def test_partition_two_cliques_finds_zero_cut():
    edges = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    edges += [(i + 5, j + 5) for i, j in edges]
    g = graphgen.from_edges(10, edges)
    for seed in range(4):
        P, res = oracle.partition(g, 2, 0.03, seed=seed)
        assert res["cut"] == 0 and res["balanced"] == 1


def test_partition_rgg_small_config():
    g = graphgen.rgg2d(16384, 1)
    P, res = oracle.partition(g, 2, 0.03)
    assert res["lmax"] == 8437 and res["ucl"] == 245
    assert res["balanced"] == 1
    assert res["coarsest_n"] <= 120
    assert res["cut"] == oracle.cut(g, P)
    B = np.bincount(P, minlength=2)
    assert B.max() == res["max_block_w"] <= res["lmax"]


def test_partition_isolated_vertices_and_empty():
    g = graphgen.from_edges(6, [(0, 1)])
    P, res = oracle.partition(g, 3, 0.03)
    assert (P >= 0).all() and res["n_isolated"] == 4 and res["balanced"] == 1
    g0 = graphgen.from_edges(4, [])
    P, res = oracle.partition(g0, 2, 0.03)
    assert np.bincount(P, minlength=2).tolist() == [2, 2] and res["cut"] == 0


# ---------------------------------------------------------------- generators

def test_rgg_edge_count_matches_analytic_expectation():
    # E[m] = C(n,2) (pi r^2 - 8 r^3/3 + r^4/2) for the unit square; Table I: rgg24 ~132.6M, rgg26 ~574.6M
    def em(n):
        r = graphgen.rgg_radius(n)
        return n * (n - 1) / 2 * (math.pi * r * r - 8 * r ** 3 / 3 + r ** 4 / 2)
    assert abs(em(1 << 24) / 1e6 - 132.6) < 0.1
    assert abs(em(1 << 26) / 1e6 - 574.6) < 0.1
    g = graphgen.rgg2d(16384, 1)
    m = len(g["adjncy"]) // 2
    assert abs(m - em(16384)) < 6 * math.sqrt(em(16384))


def test_grid_and_rmat_structure():
    g = graphgen.grid3d(7, 5, 4, seed=3, wmax=10)
    assert len(g["adjncy"]) == 2 * (6 * 5 * 4 + 7 * 4 * 4 + 7 * 5 * 3)
    assert 3 * 255 * 256 * 256 == 50_135_040  # 256^3 grid edge count
    A = _adj(g)
    assert (A != A.T).nnz == 0 and A.diagonal().sum() == 0
    assert g["adjwgt"].min() >= 1 and g["adjwgt"].max() <= 10
    r = graphgen.rmat(12, 77)
    A = _adj(r)
    assert (A != A.T).nnz == 0 and A.diagonal().sum() == 0 and A.max() == 1
    for v in range(0, 4096, 97):
        row = r["adjncy"][r["xadj"][v]:r["xadj"][v + 1]]
        assert (np.diff(row) > 0).all()
