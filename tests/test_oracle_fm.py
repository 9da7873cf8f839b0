"""Pins of the oracle's 2-way FM local search after each initial bisection
(§III-B: the recursive bisection is improved by local search). Gains count
only edges inside the bisected set; the unlocked vertex of largest gain whose
receiving side stays within (blocks it will hold) x L_max moves first (ties to
the lowest id); the shortest best prefix of a pass is kept; passes repeat until
one gains nothing."""
import numpy as np
import pytest

import graphgen
import oracle


def _two_cliques():
    # K4 {0,1,2,3} and K4 {4,5,6,7}, joined by 3-4 and 3-5; the best bisection
    # cuts only those two edges
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    edges += [(a, b) for a in range(4, 8) for b in range(a + 1, 8)] + [(3, 4), (3, 5)]
    return graphgen.from_edges(8, edges)


def _seed_starting_at(v, n):
    # the bisection's start vertex is S[mix4(seed, attempt, base, k_S) % |S|]
    return next(s for s in range(1000) if oracle.mix4(s, 0, 0, 2) % n == v)


def test_fm_worked_two_cliques():
    g = _two_cliques()
    seed = _seed_starting_at(4, 8)
    # BFS from 4 (neighbours 3, 5, 6, 7) takes 4, 3, 5, 6 as the left side:
    # cut 3-0, 3-1, 3-2, 4-7, 5-7, 6-7 = 6
    P = oracle.recursive_bisection(g, 2, seed=seed, lmax_=5, fm=0)
    assert P.tolist() == [1, 1, 1, 0, 0, 0, 0, 1] and oracle.cut(g, P) == 6
    # L_max = 5 (W = 8, eps = 0.25). FM pass 1: 7 (gain +3) moves left, then
    # 3 (gain +1; the right side's 0, 1, 2 would overload the left side)
    # moves right; every later move loses, so the 2-move prefix (gain 4) is
    # kept. Pass 2 gains nothing.
    assert oracle.lmax(8, 2, 0.25) == 5
    for fm in (1, 3):
        P = oracle.recursive_bisection(g, 2, seed=seed, lmax_=5, fm=fm)
        assert P.tolist() == [1, 1, 1, 1, 0, 0, 0, 0] and oracle.cut(g, P) == 2
    # with L_max = 4 both sides are full: no move fits, the bisection stays
    P = oracle.recursive_bisection(g, 2, seed=seed, lmax_=4, fm=3)
    assert P.tolist() == [1, 1, 1, 0, 0, 0, 0, 1]


def _single_move_gains(g, P, lm):
    """Cut reduction of every single move whose receiving side stays <= lm,
    by recomputing the cut (independent of any gain formula)."""
    c0 = oracle.cut(g, P)
    vw = g["vwgt"] if g.get("vwgt") is not None else np.ones(len(P), np.int64)
    B = np.bincount(P, weights=vw, minlength=2)
    out = []
    for v in range(len(P)):
        t = 1 - P[v]
        if B[t] + vw[v] > lm:
            continue
        Q = P.copy()
        Q[v] = t
        out.append(c0 - oracle.cut(g, Q))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_fm_bisection_is_locally_optimal(seed):
    g = graphgen.random_small(40, 0.12, seed, wmax=5, vmax=3)
    n = len(g["xadj"]) - 1
    W = int(g["vwgt"].sum())
    lm = oracle.lmax(W, 2, 0.1)
    P0 = oracle.recursive_bisection(g, 2, seed=seed, lmax_=lm, fm=0)
    P = oracle.recursive_bisection(g, 2, seed=seed, lmax_=lm, fm=1000)
    # passes run until one gains nothing, so no single move that fits reduces
    # the cut; FM only keeps improving prefixes
    assert max(_single_move_gains(g, P, lm), default=0) <= 0
    assert oracle.cut(g, P) <= oracle.cut(g, P0)
    # the receiving side never goes above L_max; a side may only shrink past it
    B0 = np.bincount(P0, weights=g["vwgt"], minlength=2)
    B = np.bincount(P, weights=g["vwgt"], minlength=2)
    assert all(B[s] <= max(B0[s], lm) for s in (0, 1)) and B.sum() == W
    assert set(P.tolist()) <= {0, 1} and len(P) == n


def test_fm_one_pass_gain_is_a_prefix_sum():
    # a single pass changes the cut by exactly the kept prefix's running gain,
    # which is positive or zero; repeated passes never raise the cut again
    g = graphgen.rgg2d(600, 11)
    lm = oracle.lmax(600, 2, 0.03)
    cuts = [oracle.cut(g, oracle.recursive_bisection(g, 2, seed=5, lmax_=lm, fm=p)) for p in range(6)]
    assert all(b <= a for a, b in zip(cuts, cuts[1:]))
    assert cuts[-1] < cuts[0]


@pytest.mark.parametrize("k", [3, 8])
def test_fm_recursive_and_partition(k):
    g = graphgen.rgg2d(3000, 4)
    lm = oracle.lmax(3000, k, 0.03)
    P = oracle.recursive_bisection(g, k, seed=1, lmax_=lm, fm=2)
    assert sorted(set(P.tolist())) == list(range(k))
    # deterministic
    assert np.array_equal(P, oracle.recursive_bisection(g, k, seed=1, lmax_=lm, fm=2))
    p, r = oracle.partition(g, k, init_fm=3)
    assert r["balanced"] == 1 and oracle.cut(g, p) == r["cut"]
    q, _ = oracle.initial_partition(g, k, lm, fm=3)
    assert q.max() < k


def test_partition_with_fm_lower_cut_on_meshes():
    # the quality this local search buys on geometric graphs (rgg16k, k = 2)
    g = graphgen.rgg2d(16384, 1)
    r0 = oracle.partition(g, 2)[1]
    r3 = oracle.partition(g, 2, init_fm=3)[1]
    assert r3["balanced"] == 1 and r3["cut"] < r0["cut"]
