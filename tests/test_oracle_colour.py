"""Pins of the oracle's colour-class LP (an oracle-only comparison mode, lp_async = 2).

The mode visits the vertices of one colour class at a time (§III-A's rule for
each vertex, §IV-A's ascending-id admission per target), with the classes of a
first-fit colouring in decreasing hash priority. Pinned here:
  * the colouring: proper (no edge inside a class) and first fit (a vertex of
    colour c has neighbours of every colour below c); K_m takes m colours, a
    star two; and it equals the colouring of the parallel rule (Jones and
    Plassmann) run step by step with splitmix64 priorities written from the
    published definition, which is what a GPU colouring would compute;
  * the sweep, traced by hand on paths whose colouring the oracle reports:
    a class proposes from the labels its earlier classes left, so a label
    travels two hops in one round, and the admission inside a class refuses
    the later proposer when the bound is reached;
  * invariants: clusters stay within U; in refinement no two movers of a class
    are adjacent, so every round lowers the cut by at least its number of moves.
"""
import numpy as np
import pytest

import graphgen
import oracle
from hand_graphs import path, star


def _check_colouring(g):
    ncol, col = oracle.colour_classes(g)
    xadj, adj = g["xadj"], g["adjncy"]
    n = len(xadj) - 1
    assert n == 0 or ncol == col.max() + 1
    for v in range(n):
        nb = col[adj[xadj[v]:xadj[v + 1]]]
        assert col[v] not in nb, v
        assert set(range(col[v])) <= set(nb.tolist()), v
    return ncol, col


@pytest.mark.parametrize("g", [graphgen.rgg2d(3000, 2), graphgen.rmat(11, 4), graphgen.grid3d(9, 8, 7, wmax=0),
                               path(9), graphgen.random_small(200, 0.05, 3)], ids=["rgg", "rmat", "grid", "path",
                                                                                   "random"])
def test_colouring_is_proper_and_first_fit(g):
    _check_colouring(g)


def test_colouring_special_graphs():
    m = 7
    kg = graphgen.from_edges(m, [(i, j) for i in range(m) for j in range(i + 1, m)])
    ncol, col = _check_colouring(kg)
    assert ncol == m and sorted(col.tolist()) == list(range(m))
    assert _check_colouring(star(9))[0] == 2
    assert oracle.colour_classes(graphgen.from_edges(5, []))[0] == 1


def test_sweep_traced_on_a_path():
    g = path(5)
    # the oracle's colouring of this path alternates, classes {0, 2, 4} then {1, 3}
    assert oracle.colour_classes(g)[1].tolist() == [0, 1, 0, 1, 0]
    # U = 3, round 0, class {0, 2, 4}: 0 -> label 1; 2 ties labels 1 and 3 -> 1; 4 -> 3.
    #   Admitted (1: 1 + 1 + 1 <= 3; 3: 1 + 1 <= 3) -> [1, 1, 1, 3, 3]. Class {1, 3}: 1 is
    #   settled; 3 would join label 1 (weight 3 + 1 > 3): stays. Two idle rounds follow.
    lab, st = oracle.lp_cluster_colour(g, 3, 10)
    assert lab.tolist() == [1, 1, 1, 3, 3] and (st["rounds_run"], st["moves"]) == (3, 3)
    # U = 2: the admission to label 1 takes 0 (1 + 1 <= 2) and refuses 2 (1 + 2 > 2)
    lab, st = oracle.lp_cluster_colour(g, 2, 10)
    assert lab.tolist() == [1, 1, 2, 3, 3] and st["moves"] == 2
    # the synchronous rounds with direction alternation need more than one round to do
    # the same: after round 0 no label has travelled two hops
    sync, _ = oracle.lp_cluster(g, 3, 1, 1)
    assert sync.tolist() != [1, 1, 1, 3, 3]


def test_sweep_traced_on_three_vertices():
    g = path(3)
    assert oracle.colour_classes(g)[1].tolist() == [0, 1, 0]
    # class {0, 2} proposes label 1 twice; U = 2 admits only 0, U = 3 both
    assert oracle.lp_cluster_colour(g, 2, 1)[0].tolist() == [1, 1, 2]
    assert oracle.lp_cluster_colour(g, 3, 1)[0].tolist() == [1, 1, 1]


@pytest.mark.parametrize("g,U", [(graphgen.rgg2d(5000, 3), 7), (graphgen.rmat(12, 5), 40),
                                 (graphgen.grid3d(12, 10, 9, seed=1, wmax=8), 5)])
def test_clusters_stay_within_the_bound(g, U):
    lab, st = oracle.lp_cluster_colour(g, U, 10)
    c = g["vwgt"] if g.get("vwgt") is not None else np.ones(len(g["xadj"]) - 1, np.int64)
    assert np.bincount(lab, weights=c).max() <= U
    assert st["moves"] > 0 and st["edge_visits"] == st["rounds_run"] * len(g["adjncy"])


@pytest.mark.parametrize("g,k", [(graphgen.rgg2d(4000, 6), 8), (graphgen.grid3d(12, 12, 8, seed=2, wmax=9), 16),
                                 (graphgen.rmat(12, 7), 4)])
def test_refinement_rounds_lower_the_cut_by_their_moves(g, k):
    n = len(g["xadj"]) - 1
    P = np.array([graphgen.rand_u64(k + 1, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(n, k, 0.03)
    for _ in range(6):
        before = oracle.cut(g, P)
        P2, st = oracle.lp_refine_colour(g, P, k, lm, 1)
        assert before - oracle.cut(g, P2) >= st["moves"]
        assert oracle.block_weights(g, P2, k).max() <= max(lm, oracle.block_weights(g, P, k).max())
        P = P2


@pytest.mark.parametrize("g,k", [(graphgen.rgg2d(16384, 1), 2), (graphgen.grid3d(20, 20, 20, seed=3, wmax=10), 16),
                                 (graphgen.rmat(13, 2), 8)])
def test_multilevel_scheme_in_colour_mode(g, k):
    p1, r1 = oracle.partition(g, k, 0.03, lp_async=2)
    p2, r2 = oracle.partition(g, k, 0.03, lp_async=2)
    assert np.array_equal(p1, p2) and r1["balanced"]
    assert r1["cut"] == oracle.cut(g, p1)
    assert r1["levels"] >= 1 and r1["edge_visits_cluster"] > 0


@pytest.mark.parametrize("g,k", [(graphgen.grid3d(24, 24, 24, seed=3, wmax=10), 16), (graphgen.rmat(13, 6), 8)])
def test_clustering_only_mode_composes_the_other_two(g, k):
    # lp_async = 3: colour classes in clustering, synchronous rounds in refinement. Its
    # hierarchy is that of lp_async = 2 (same clustering), its refinement that of lp_async = 0
    p2, r2 = oracle.partition(g, k, 0.03, lp_async=2)
    p3, r3 = oracle.partition(g, k, 0.03, lp_async=3)
    for key in ("levels", "coarsest_n", "edge_visits_cluster"):
        assert r3[key] == r2[key], key
    c2, i2 = oracle.coarsest(g, k, 0.03, lp_async=2)
    c3, i3 = oracle.coarsest(g, k, 0.03, lp_async=3)
    assert all(np.array_equal(c2[f], c3[f]) for f in c2) and np.array_equal(i2, i3)
    assert r3["balanced"] and r3["cut"] == oracle.cut(g, p3)


def test_clustering_only_mode_without_coarsening_is_the_synchronous_scheme():
    # 2,000 vertices <= 60 k for k = 64: no clustering runs, so lp_async = 3 is lp_async = 0
    # exactly (the refinement rounds are the synchronous ones in both)
    g = graphgen.rgg2d(2000, 5)
    p0, r0 = oracle.partition(g, 64, 0.03)
    p3, r3 = oracle.partition(g, 64, 0.03, lp_async=3)
    assert r0["levels"] == 1 and np.array_equal(p0, p3)
    assert (r0["cut"], r0["edge_visits_refine"]) == (r3["cut"], r3["edge_visits_refine"])


def test_thread_count_changes_nothing():
    g = graphgen.grid3d(40, 40, 30, seed=3, wmax=10)
    try:
        oracle.set_threads(1)
        p1, r1 = oracle.partition(g, 16, 0.03, lp_async=2)
        oracle.set_threads(4)
        p4, r4 = oracle.partition(g, 16, 0.03, lp_async=2)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(p1, p4) and r1 == r4


def _splitmix64(x):
    # the finaliser of state x + gamma (Steele, Lea & Flood 2014), on uint64 arrays
    m = np.uint64(0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & m
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & m
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & m
        return z ^ (z >> np.uint64(31))


def _parallel_rule_colouring(g):
    # steps of the parallel rule: a vertex whose neighbours of higher priority are all
    # coloured takes the smallest colour absent among them; all such vertices at once
    n = len(g["xadj"]) - 1
    p = _splitmix64(np.arange(n, dtype=np.uint64))
    col = np.full(n, -1)
    while (col < 0).any():
        ready = []
        for v in np.flatnonzero(col < 0):
            nb = g["adjncy"][g["xadj"][v]:g["xadj"][v + 1]]
            hi = nb[(p[nb] > p[v]) | ((p[nb] == p[v]) & (nb > v))]
            if (col[hi] >= 0).all():
                ready.append((v, set(col[hi].tolist())))
        assert ready
        for v, used in ready:
            c = 0
            while c in used:
                c += 1
            col[v] = c
    return col


def test_colouring_is_that_of_the_parallel_rule():
    # the published first output of splitmix64 from state 0 guards the numpy finaliser
    assert int(_splitmix64(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF
    for g in (graphgen.rgg2d(1500, 7), graphgen.rmat(9, 3), graphgen.grid3d(7, 6, 5, wmax=0), path(12),
              graphgen.random_small(120, 0.08, 5)):
        assert np.array_equal(oracle.colour_classes(g)[1], _parallel_rule_colouring(g))
