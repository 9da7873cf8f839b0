"""Pins of the oracle-only multi-try k-way local search (§III-C): searches
started at single boundary vertices, moves by largest gain under L_max, the
best prefix of each search kept, local iterations around moved vertices and
three global iterations. It measures what the GPU path's LP-only refinement
leaves on the table."""
import numpy as np
import pytest

import graphgen
import oracle


def _bridge():
    # a = 0 and b = 1 (block 0) are tied by an edge of weight 5; a has unit
    # edges to 2, 3, 4 and b to 5, 6, 7, all in block 1, where each of them
    # has a weight-3 edge to the centre 8. 9-10 (weight 10) stay in block 0.
    edges = [(0, 1), (0, 2), (0, 3), (0, 4), (1, 5), (1, 6), (1, 7)] + [(i, 8) for i in range(2, 8)] + [(9, 10)]
    w = [5, 1, 1, 1, 1, 1, 1] + [3] * 6 + [10]
    g = graphgen.from_edges(11, edges, weights=w)
    part = np.array([0, 0, 1, 1, 1, 1, 1, 1, 1, 0, 0], np.int32)
    return g, part


def test_mls_worked_negative_first_move():
    g, part = _bridge()
    assert oracle.cut(g, part) == 6
    # every single move loses: a and b have gain 3 - 5 = -2, the block-1
    # leaves 1 - 3 = -2, so label propagation keeps the partition
    P, st = oracle.lp_refine(g, part, 2, 100, 25)
    assert P.tolist() == part.tolist() and st["moves"] == 0
    assert oracle.mls_gain(g, part, 2, 100, 0) == (-2, 1)
    assert oracle.mls_gain(g, part, 2, 100, 8) == (0, -1)  # no adjacent other block
    # a search moves a first (gain -2, lowest id among the -2 ties); b's gain
    # becomes 3 + 5 = +8 and b follows: the prefix of both moves gains 6
    P, st = oracle.mls(g, part, 2, 100)
    assert P.tolist() == [1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0]
    assert oracle.cut(g, P) == 0 and st["gain"] == 6 and st["moves"] == 2


def test_mls_respects_lmax():
    # with L_max = 8 block 1 (weight 7) takes one more vertex only: a moves
    # (gain -2) but b cannot follow, so the search keeps nothing
    g, part = _bridge()
    P, st = oracle.mls(g, part, 2, 8)
    assert P.tolist() == part.tolist() and st["gain"] == 0 and st["moves"] == 0


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_mls_invariants(seed):
    g = graphgen.random_small(200, 0.05, seed, wmax=6, vmax=3)
    n = len(g["xadj"]) - 1
    k = 4
    W = int(g["vwgt"].sum())
    lm = oracle.lmax(W, k, 0.03)
    part, _ = oracle.partition(g, k)
    c0 = oracle.cut(g, part)
    P, st = oracle.mls(g, part, k, lm, seed=seed)
    B = np.bincount(P, weights=g["vwgt"], minlength=k)
    assert B.max() <= lm  # the start partition is balanced and no move breaks L_max
    assert oracle.cut(g, P) == c0 - st["gain"] and st["gain"] >= 0
    # deterministic, and a second run from the result gains no more than it finds
    P2, st2 = oracle.mls(g, part, k, lm, seed=seed)
    assert np.array_equal(P, P2)
    P3, st3 = oracle.mls(g, P, k, lm, seed=seed)
    assert oracle.cut(g, P3) == oracle.cut(g, P) - st3["gain"]


def test_mls_gain_matches_definition():
    # gain(v) = max over adjacent blocks b != block(v) with B[b] + c(v) <= L_max
    # of conn(v, b) - conn(v, block(v)); ties -> lowest b; spot checks
    g = graphgen.random_small(60, 0.1, 7, wmax=5, vmax=2)
    n = len(g["xadj"]) - 1
    k = 3
    part = (np.arange(n) % k).astype(np.int32)
    B = np.bincount(part, weights=g["vwgt"], minlength=k)
    lm = int(B.max()) + 1
    for v in range(n):
        conn = np.zeros(k, np.int64)
        for e in range(g["xadj"][v], g["xadj"][v + 1]):
            conn[part[g["adjncy"][e]]] += g["adjwgt"][e]
        cands = [b for b in range(k) if b != part[v] and conn[b] > 0 and B[b] + g["vwgt"][v] <= lm]
        gn, t = oracle.mls_gain(g, part, k, lm, v)
        if not cands:
            assert t == -1
        else:
            best = max(cands, key=lambda b: (conn[b], -b))
            assert (gn, t) == (int(conn[best] - conn[part[v]]), best)


def test_partition_with_mls_is_balanced_and_better():
    # MLS after every level's LP refinement: balanced, and a lower cut here
    for g, k in ((graphgen.rgg2d(4000, 5), 8), (graphgen.rmat(11, 4), 8)):
        p0, r0 = oracle.partition(g, k)
        p1, r1 = oracle.partition(g, k, mls=3)
        assert r1["balanced"] == 1 and oracle.cut(g, p1) == r1["cut"]
        assert r1["cut"] < r0["cut"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batched_mls_of_one_is_sequential(seed):
    # searches in batches of one see every earlier move and mark, and the
    # recomputed gains of a kept prefix equal the search's own: the result
    # is the sequential one, statistics included
    g = graphgen.random_small(300, 0.04, seed, wmax=6, vmax=3)
    k = 5
    lm = oracle.lmax(int(g["vwgt"].sum()), k, 0.03)
    part, _ = oracle.partition(g, k)
    a, sa = oracle.mls(g, part, k, lm, seed=seed)
    b, sb = oracle.mls(g, part, k, lm, seed=seed, batch=1)
    assert np.array_equal(a, b) and sa == sb


@pytest.mark.parametrize("batch", [2, 16, 10 ** 6])
def test_batched_mls_invariants(batch):
    # searches of a batch start from the same state; their prefixes are
    # applied in seed order with recomputed gains, so the reported gain is
    # the exact cut change and no move breaks L_max
    g = graphgen.rgg2d(3000, 4)
    k = 8
    lm = oracle.lmax(3000, k, 0.03)
    part, _ = oracle.partition(g, k)
    c0 = oracle.cut(g, part)
    P, st = oracle.mls(g, part, k, lm, seed=3, batch=batch)
    assert np.bincount(P, minlength=k).max() <= lm
    assert st["gain"] >= 0 and oracle.cut(g, P) == c0 - st["gain"]
    P2, st2 = oracle.mls(g, part, k, lm, seed=3, batch=batch)
    assert np.array_equal(P, P2) and st == st2
    p, r = oracle.partition(g, k, mls=3, mls_batch=batch)
    assert r["balanced"] == 1 and oracle.cut(g, p) == r["cut"]


@pytest.mark.parametrize("q", [1, 8, 64])
def test_mls_queue_bound(q):
    g = graphgen.rmat(11, 5)
    n = len(g["xadj"]) - 1
    k = 8
    lm = oracle.lmax(n, k, 0.03)
    part, _ = oracle.partition(g, k)
    c0 = oracle.cut(g, part)
    # a bound the searches never reach changes nothing
    a, sa = oracle.mls(g, part, k, lm, seed=2)
    b, sb = oracle.mls(g, part, k, lm, seed=2, max_queue=n + 1)
    assert np.array_equal(a, b) and sa == sb
    # bounded searches, alone or in batches: exact gains, L_max kept, and a
    # batch of one is still the sequential search
    for batch in (0, 1, 32):
        P, st = oracle.mls(g, part, k, lm, seed=2, batch=batch, max_queue=q)
        assert np.bincount(P, minlength=k).max() <= lm
        assert st["gain"] >= 0 and oracle.cut(g, P) == c0 - st["gain"]
        if batch == 0:
            seq = (P, st)
        if batch == 1:
            assert np.array_equal(P, seq[0]) and st == seq[1]


@pytest.mark.parametrize("shape", ["clique", "star"])
def test_batched_mls_disjoint_neighbourhoods(shape):
    # every two closed neighbourhoods meet (in a clique directly, in a star
    # through the hub), so every batch holds a single seed and any batch size
    # gives the sequential result
    rng = np.random.default_rng(4)
    if shape == "clique":
        n = 24
        edges = [(a, b) for a in range(n) for b in range(a + 1, n)]
    else:
        n = 40
        edges = [(0, i) for i in range(1, n)]
    w = rng.integers(1, 6, size=len(edges)).tolist()
    g = graphgen.from_edges(n, edges, weights=w)
    k = 4
    part = (np.arange(n) * 5 % k).astype(np.int32)
    lm = oracle.lmax(n, k, 0.25)
    a, sa = oracle.mls(g, part, k, lm, seed=1)
    for batch in (2, 7, 10 ** 6):
        b, sb = oracle.mls(g, part, k, lm, seed=1, batch=batch)
        assert np.array_equal(a, b) and sa == sb, batch
    assert sa["gain"] > 0
