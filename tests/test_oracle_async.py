"""Pins of the oracle-only sequential LP (§III-A as the paper states it), used
to measure what the round-synchronous reading costs in quality."""
import numpy as np
import pytest

import graphgen
import oracle


def test_async_worked_path():
    # path 0-1-2-3, unit weights, U = 2; queue by degree: [0, 3, 1, 2].
    # iteration 1: 0 joins 1 (W[1] = 2), 3 joins 2 (W[2] = 2); 1 and 2 cannot
    # join the other full cluster and stay. Iteration 2 (queue [1, 2]): no move.
    g = graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    lab, st = oracle.lp_cluster_async(g, 2, 10)
    assert lab.tolist() == [1, 1, 2, 2]
    assert st == {"rounds_run": 2, "moves": 2, "edge_visits": 1 + 1 + 2 + 2 + 2 + 2}


def test_async_worked_star_and_tie():
    # star 0-{1,2}, U = 3: both leaves join 0 in queue order [1, 2, 0]
    g = graphgen.from_edges(3, [(0, 1), (0, 2)])
    lab, st = oracle.lp_cluster_async(g, 3, 10)
    assert lab.tolist() == [0, 0, 0] and st["moves"] == 2 and st["rounds_run"] == 2
    # path 0-1-2, U = 2: 0 joins 1; 2 cannot (full); 1 ties between its own
    # cluster and cluster 2 and keeps its own
    g = graphgen.from_edges(3, [(0, 1), (1, 2)])
    lab, st = oracle.lp_cluster_async(g, 2, 10)
    assert lab.tolist() == [1, 1, 2] and st["moves"] == 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_async_invariants(seed):
    g = graphgen.random_small(120, 0.06, seed, wmax=7, vmax=4)
    n = len(g["xadj"]) - 1
    U = 9
    lab, st = oracle.lp_cluster_async(g, U, 10)
    W = np.bincount(lab, weights=g["vwgt"], minlength=n)
    assert W.max() <= U  # singletons start at c(v) <= 4 <= U and a move needs room
    assert W.sum() == g["vwgt"].sum()
    # one more iteration over every vertex finds no move: a fixed point unless
    # the iteration budget ran out first
    if st["rounds_run"] < 10:
        lab2, st2 = oracle.lp_cluster_async(g, U, 10)
        assert np.array_equal(lab, lab2)
    # refinement keeps every block within the bound it started within, and
    # each sequential move lowers the cut by its strict gain
    k = 4
    part = (np.arange(n) % k).astype(np.int32)
    lm = int(np.bincount(part, weights=g["vwgt"], minlength=k).max()) + 2
    p2, st = oracle.lp_refine_async(g, part, k, lm, 25)
    assert np.bincount(p2, weights=g["vwgt"], minlength=k).max() <= lm
    assert oracle.cut(g, p2) < oracle.cut(g, part) or st["moves"] == 0


@pytest.mark.parametrize("case", ["rgg", "grid", "rmat"])
def test_async_partition_is_valid(case):
    if case == "rgg":
        g, k = graphgen.rgg2d(4000, 5), 4
    elif case == "grid":
        g, k = graphgen.grid3d(20, 20, 20, seed=3, wmax=10), 16
    else:
        g, k = graphgen.rmat(13, 5), 8
    p0, r0 = oracle.partition(g, k)
    p1, r1 = oracle.partition(g, k, lp_async=1)
    assert r1["balanced"] == 1 and r0["balanced"] == 1
    assert oracle.cut(g, p1) == r1["cut"]
