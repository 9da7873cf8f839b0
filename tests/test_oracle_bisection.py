"""Pins of the oracle's breadth-first bisection (initial partitioning, §III-B).

The paper grows each bisection's first side from a start vertex and leaves the
details to the initial partitioner. The reading pinned here: a FIFO search
inside the current vertex set S, neighbours taken in ascending id order,
vertices marked when enqueued and added to the grown side when dequeued; the
search stops as soon as the grown side weighs at least
ceil(c(S) * ceil(k_S / 2) / k_S); if the queue runs dry first, the smallest
unmarked vertex of S is enqueued. The grown side takes the lower block ids.

The start vertex of a bisection is S[mix4(seed, try, first block, k_S) mod |S|]
(S ascending); mix4 itself is pinned by published splitmix64 outputs in
tests/test_oracle_stop_rules.py, so each case below picks a seed whose start is
the vertex it was traced from. Every expected side is traced by hand. A search
that takes neighbours in descending order, a stack instead of a queue, a start
taken from another index, a restart at another vertex than the smallest
unmarked one, or a '>' stop rule gives another side in at least one case.
"""
import numpy as np
import pytest

import oracle
from hand_graphs import path, spider, star, three_parts


def _seed_for(start_index, size, ks, base=0, attempt=0):
    for seed in range(100000):
        if oracle.mix4(seed, attempt, base, ks) % size == start_index:
            return seed
    raise AssertionError("no seed found")


def _side0(g, seed, k=2, attempt=0):
    P = oracle.recursive_bisection(g, k, seed=seed, attempt=attempt)
    return set(np.flatnonzero(P == 0).tolist())


# star: centre 0, leaves 1..7 (unit weights, k = 2: the grown side weighs 4)
STAR = star(7)
# traced: from the centre the leaves are enqueued 1, 2, ..., 7 and 1, 2, 3 follow it;
# from a leaf s the centre comes second, then the smallest leaves other than s
STAR_SIDES = {
    0: {0, 1, 2, 3},
    1: {1, 0, 2, 3},
    3: {3, 0, 1, 2},
    4: {4, 0, 1, 2},
    7: {7, 0, 1, 2},
}


@pytest.mark.parametrize("start", sorted(STAR_SIDES))
def test_star_neighbours_in_ascending_order(start):
    assert _side0(STAR, _seed_for(start, 8, 2)) == STAR_SIDES[start]


# spider: centre 0 with legs 0-1-2-3, 0-4-5-6, 0-7-8-9 (n = 10, the grown side weighs 5)
SPIDER = spider()
# traced (dequeue order):
#   from 0: 0 | 1 4 7 | 2            -> a queue reaches all three legs before going deeper
#   from 3: 3 2 1 0 | 4              -> the first leg, then the lowest next leg
#   from 5: 5 | 4 6 | 0 | 1          -> 4 before 6, then the centre, then leg 1 before leg 7
#   from 8: 8 | 7 9 | 0 | 1
SPIDER_SIDES = {
    0: {0, 1, 4, 7, 2},
    3: {3, 2, 1, 0, 4},
    5: {5, 4, 6, 0, 1},
    8: {8, 7, 9, 0, 1},
}


@pytest.mark.parametrize("start", sorted(SPIDER_SIDES))
def test_spider_is_grown_breadth_first(start):
    assert _side0(SPIDER, _seed_for(start, 10, 2)) == SPIDER_SIDES[start]


# three components: path 0-1-2-3-4, triangle 5-6-7, edge 8-9 (the grown side weighs 5)
PARTS = three_parts()
# traced: a component smaller than the target runs dry and the search restarts at the
# smallest unmarked vertex
PARTS_SIDES = {
    6: {6, 5, 7, 0, 1},   # triangle (3), then 0, 1
    9: {9, 8, 0, 1, 2},   # edge (2), then 0, 1, 2
    2: {2, 1, 3, 0, 4},   # the path alone reaches the target
    8: {8, 9, 0, 1, 2},
}


@pytest.mark.parametrize("start", sorted(PARTS_SIDES))
def test_search_restarts_at_smallest_unmarked_vertex(start):
    assert _side0(PARTS, _seed_for(start, 10, 2)) == PARTS_SIDES[start]


def test_weighted_stop_is_at_least_target():
    # path 0-1-2-3 with vertex weights 3, 1, 1, 3 (c(S) = 8, target 4), started at 1:
    # 1 (weight 1), then 0 (total 4 >= 4): stop. A '>' rule would take 2 as well.
    g = path(4, vwgt=[3, 1, 1, 3])
    assert _side0(g, _seed_for(1, 4, 2)) == {0, 1}
    # started at 2: 2, then 1 (total 2), then 3 (total 5): the lower neighbour 1 is
    # dequeued before 3, so 0 stays out
    assert _side0(g, _seed_for(2, 4, 2)) == {1, 2, 3}


def test_four_blocks_on_a_path_traced():
    # path 0..7, k = 4. First bisection: k_S = 4, the grown side weighs ceil(8 * 2 / 4) = 4
    # and takes blocks 0, 1; the rest takes blocks 2, 3. Each side is then bisected with
    # k_S = 2 (first block 0 and 2): its grown side weighs 2.
    n = 8
    g = path(n)
    # find a seed whose first start is vertex 5: 5 | 4 6 | 3 -> side {3, 4, 5, 6}
    found = 0
    for seed in range(20000):
        if oracle.mix4(seed, 0, 0, 4) % n != 5:
            continue
        left, right = [3, 4, 5, 6], [0, 1, 2, 7]
        sl = left[oracle.mix4(seed, 0, 0, 2) % 4]
        sr = right[oracle.mix4(seed, 0, 2, 2) % 4]
        # traced second-level sides (two vertices each): inside {3,4,5,6} the start's lower
        # neighbour is dequeued next when it is in the set, else the upper one; inside
        # {0,1,2,7}, 7 has no neighbour in the set, so the search restarts at 0
        second_l = {3: {3, 4}, 4: {4, 3}, 5: {5, 4}, 6: {6, 5}}[sl]
        second_r = {0: {0, 1}, 1: {1, 0}, 2: {2, 1}, 7: {7, 0}}[sr]
        expect = np.empty(n, np.int32)
        for v in left:
            expect[v] = 0 if v in second_l else 1
        for v in right:
            expect[v] = 2 if v in second_r else 3
        P = oracle.recursive_bisection(g, 4, seed=seed, attempt=0)
        assert P.tolist() == expect.tolist(), (seed, sl, sr)
        found += 1
        if found == 6:
            break
    assert found == 6


def test_try_index_changes_the_start():
    # the try index is the second word of the start hash: tries of one seed start at
    # different vertices for some seed, and each try's side is the traced one for its start
    hits = 0
    for seed in range(200):
        starts = [oracle.mix4(seed, a, 0, 2) % 8 for a in range(4)]
        if len(set(starts)) < 2:
            continue
        for a, s in enumerate(starts):
            want = STAR_SIDES.get(s, {s, 0, 1, 2} if s >= 3 else {0, 1, 2, 3})
            assert _side0(STAR, seed, attempt=a) == want
        hits += 1
        if hits == 4:
            break
    assert hits == 4
