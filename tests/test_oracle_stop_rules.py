"""Pins of the oracle's coarsening stop rules and initial-try selection.

The paper only says coarsening stops once the graph is "small enough" (§III-A)
and that the best of several initial tries is kept (§III-B, §IV-B). The
readings pinned here: coarsen while n > coarsest_per_k * k; a level that does
not shrink is discarded and coarsening stops; after a level with
stall_den * n' > stall_num * n coarsening stops and that level is kept; the
number of levels is not bounded otherwise; the kept try is the minimum of
(imbalanced, cut, try index).

Every expected number below is traced by hand on graphs made of a path of
unit-weight vertices and disjoint pairs of weight-2 vertices (tests/hand_graphs.py),
with one clustering round per level (rounds_coarsen = 1, a round that only
allows moves to smaller labels) and a clustering bound U_c = 2, so that:
  * a weight-2 vertex never joins anything (2 + 1 > 2);
  * on a path whose front holds j weight-2 vertices followed by unit-weight
    ones, the round moves every unit vertex after the first one to its left
    neighbour's label, each target receiving exactly one proposer (admitted:
    1 + 1 <= 2), so the path loses exactly one vertex per level while two or
    more unit vertices remain; then no vertex moves.
"""
import numpy as np
import pytest

import oracle
from hand_graphs import path_and_heavy_pairs, two_cliques

ONE_ROUND = dict(rounds_coarsen=1)


def _ucl(g, k):
    W = oracle.total_vwgt(g)
    cmax = int(np.max(g["vwgt"]))
    return max(cmax, oracle.lmax(W, k, 0.03) - (-(-W // k)))


def test_hand_graphs_have_cluster_bound_two():
    # W = 36: L_max = floor(1.03 * 36) = 37, slack 1, c_max = 2 -> U_c = 2
    g20 = path_and_heavy_pairs(4, 8)
    assert oracle.total_vwgt(g20) == 36 and _ucl(g20, 1) == 2
    # W = 80: L_max = 82, slack 2 -> U_c = 2
    g42 = path_and_heavy_pairs(4, 19)
    assert oracle.total_vwgt(g42) == 80 and _ucl(g42, 1) == 2
    # W = 144, k = 3: ceil(W/k) = 48, L_max = floor(1.03 * 48) = 49, slack 1 -> U_c = 2
    g142 = path_and_heavy_pairs(140, 1)
    assert _ucl(g142, 3) == 2


def test_one_level_removes_one_path_vertex():
    # level 0 -> 1 of a 4-vertex path: labels [0, 0, 1, 2] -> clusters {0,1}, {2}, {3}
    g = path_and_heavy_pairs(4, 8)
    lab, st = oracle.lp_cluster(g, 2, 1)
    assert lab[:4].tolist() == [0, 0, 1, 2]
    assert lab[4:].tolist() == list(range(4, 20))


@pytest.mark.parametrize("cp,levels,coarsest", [(20, 1, 20), (19, 2, 19)])
def test_threshold_is_strict(cp, levels, coarsest):
    # n = 20, k = 1: coarsen only while n > cp * k; with cp = 19 one level (n = 19) and 19 > 19 fails
    g = path_and_heavy_pairs(4, 8)
    _, res = oracle.partition(g, 1, 0.03, coarsest_per_k=cp, **ONE_ROUND)
    assert (res["levels"], res["coarsest_n"]) == (levels, coarsest)


def test_stall_level_is_kept_and_stops():
    # n = 42 -> 41: 20 * 41 = 820 > 19 * 42 = 798, so level 1 is kept and is the last
    # (discarding it would leave 1 level; going on would reach 40)
    g = path_and_heavy_pairs(4, 19)
    _, res = oracle.partition(g, 1, 0.03, coarsest_per_k=1, **ONE_ROUND)
    assert (res["levels"], res["coarsest_n"]) == (2, 41)


def test_stall_boundary_and_discarded_level():
    # n = 20 -> 19: 20 * 19 = 380 is not > 19 * 20 = 380, go on; 19 -> 18: 360 is not > 361, go on;
    # the next level cannot shrink (two weight-2 path vertices) and is discarded: 3 levels, 18 vertices
    g = path_and_heavy_pairs(4, 8)
    _, res = oracle.partition(g, 1, 0.03, coarsest_per_k=1, **ONE_ROUND)
    assert (res["levels"], res["coarsest_n"]) == (3, 18)


def test_more_than_64_levels():
    # stall rule off (stall_num = stall_den: n' > n never holds): the 140-vertex path
    # loses one vertex per level for 70 levels (140 unit vertices -> 70 pairs), the next
    # level cannot shrink and is discarded: 71 graphs, 70 + 2 coarsest vertices
    g = path_and_heavy_pairs(140, 1)
    _, res = oracle.partition(g, 3, 0.03, coarsest_per_k=1, stall_num=1, stall_den=1, **ONE_ROUND)
    assert (res["levels"], res["coarsest_n"]) == (71, 72)
    assert res["balanced"] == 1


def _start_vertex(seed, attempt, n):
    # the first bisection of try `attempt` starts at sorted(V)[mix4(seed, attempt, 0, k) mod n]
    return oracle.mix4(seed, attempt, 0, 2) % n


@pytest.mark.parametrize("seed", range(8))
def test_tied_tries_keep_the_first(seed):
    # two disjoint K5, k = 2: every try cuts 0 and is balanced (the BFS from the start
    # vertex fills its own clique, 5 = ceil(10 * 1 / 2)); the tries differ only in which
    # clique becomes block 0, the start vertex's. Ties go to the lowest try index.
    g = two_cliques(5)
    lm = oracle.lmax(10, 2, 0.03)
    starts = [_start_vertex(seed, a, 10) for a in range(4)]
    P, best = oracle.initial_partition(g, 2, lm, seed=seed, attempts=4)
    assert best == 0
    assert P[starts[0]] == 0
    assert sorted(np.bincount(P, minlength=2).tolist()) == [5, 5]


def test_seeds_whose_tries_disagree_exist():
    # the tie test above would not notice a "last try wins" mistake unless some seed's
    # first and last tries start in different cliques
    side = [[_start_vertex(s, a, 10) // 5 for a in range(4)] for s in range(8)]
    assert any(sd[0] != sd[3] for sd in side)


def test_mix4_from_published_splitmix64_outputs():
    # splitmix64 (Steele, Lea & Flood 2014): next() from state x returns the finaliser of
    # x + gamma; started at state 0 its outputs are E220A8397B1DCDAF (state 0),
    # 6E789E6AA1B965F4 (state gamma) and 06C45D188009454F (state 2 gamma).
    # mix4 chains sm(sm(sm(sm(seed) ^ a) ^ base) ^ ks) with sm = next() from state x, so the
    # arguments below walk through exactly those states.
    M = (1 << 64) - 1
    gamma = 0x9E3779B97F4A7C15
    o0, o1, o2 = 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F
    a = o0 ^ gamma
    base = o1 ^ ((2 * gamma) & M)
    ks = o2 ^ 0
    assert oracle.mix4(0, a, base, ks) == o0
    # a different last word leaves state 0: the chain is order-sensitive
    assert oracle.mix4(0, a, base, ks ^ 1) != o0
    assert oracle.mix4(0, base, a, ks) != o0
