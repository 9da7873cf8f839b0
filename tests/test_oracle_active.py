"""Pins of the oracle's active-set rounds: the synchronous form of the paper's
queues Q/Q' (§III-A, §IV-A), where only vertices that still owe an evaluation
propose. Owed evaluations: all vertices start with one per direction, each
evaluation pays one, a proposal refused by the admission leaves at least one,
and every neighbour of an admitted mover owes one per direction again."""
import numpy as np
import pytest

import graphgen
import oracle


def _capacity_graph():
    # x = 0 (block 0) has both neighbours 1, 2 in block 1; 1-3 and 2-4 hold 1
    # and 2 in place (ties); y = 5 (block 1) has both neighbours 6, 7 in block
    # 0, and 6-7 holds them in place. Blocks: {0, 6, 7} and {1, .., 5}.
    edges = [(0, 1), (0, 2), (1, 3), (2, 4), (5, 6), (5, 7), (6, 7)]
    g = graphgen.from_edges(8, edges)
    part = np.array([0, 1, 1, 1, 1, 1, 0, 0], np.int32)
    return g, part


def test_active_worked_capacity_freed_elsewhere():
    # lmax = 5, one direction. Round 0: block 1 is full (5 + 1 > 5), so x makes
    # no proposal; y moves to block 0 (3 + 1 <= 5), freeing room in block 1.
    g, part = _capacity_graph()
    # full rounds: round 1 re-evaluates x, which now fits (4 + 1 <= 5) and
    # moves; rounds 2 and 3 are idle. Visits: 4 rounds x 14 entries.
    P, st = oracle.lp_refine(g, part, 2, 5, 25, dir_alternate=0)
    assert P.tolist() == [1, 1, 1, 1, 1, 0, 0, 0]
    assert st == {"rounds_run": 4, "moves": 2, "edge_visits": 56}
    # active-set rounds: after round 0 only y's neighbours 6 and 7 owe an
    # evaluation (x made no proposal and none of its neighbours moved); they
    # stay, round 2 has nobody to evaluate, so x keeps block 0.
    # Visits: 14 (round 0) + deg 6 + deg 7 (round 1) + 0.
    P, st = oracle.lp_refine(g, part, 2, 5, 25, dir_alternate=0, active=True)
    assert P.tolist() == [0, 1, 1, 1, 1, 0, 0, 0]
    assert st == {"rounds_run": 3, "moves": 1, "edge_visits": 14 + 4}


def test_active_worked_two_directions():
    # the same graph with direction alternation (two evaluations owed per
    # direction change). Round 0 (smaller labels only): x cannot look at block
    # 1, y moves to block 0. Round 1 (larger labels): every vertex still owes
    # one evaluation, x moves to block 1. Round 2: 6, 7 (one left) and x's
    # neighbours 1, 2 (two again) stay; round 3: 1 and 2 stay; stop.
    g, part = _capacity_graph()
    P, st = oracle.lp_refine(g, part, 2, 5, 25, dir_alternate=1, active=True)
    assert P.tolist() == [1, 1, 1, 1, 1, 0, 0, 0]
    assert st == {"rounds_run": 4, "moves": 2, "edge_visits": 14 + 14 + 8 + 4}


def test_active_worked_refused_proposal_stays_active():
    # p = 0 and q = 1 (block 0) both want block 1 (two neighbours there); z = 6
    # (block 1) wants block 0. lmax = 6, one direction, W = (4, 5).
    # Round 0: target 1 admits p (5 + 1 <= 6) and refuses q (5 + 2 > 6); z
    # moves to block 0. Round 1: q still owes an evaluation (refused), block 1
    # has room again (W1 = 5) and q moves; p's neighbours 2, 3 and z's
    # neighbours 7, 8 stay. Round 2: q's neighbours 4, 5 stay. Round 3: idle.
    edges = [(0, 2), (0, 3), (1, 4), (1, 5), (2, 3), (4, 5), (6, 7), (6, 8), (7, 8)]
    g = graphgen.from_edges(9, edges)
    part = np.array([0, 0, 1, 1, 1, 1, 1, 0, 0], np.int32)
    P, st = oracle.lp_refine(g, part, 2, 6, 25, dir_alternate=0, active=True)
    assert P.tolist() == [1, 1, 1, 1, 1, 1, 0, 0, 0]
    assert st == {"rounds_run": 4, "moves": 3, "edge_visits": 18 + 10 + 4}
    # round by round against the single-round primitive: q is refused first
    C = part.copy()
    W = np.array([4, 5], np.int64)
    C, W, m, prop = oracle.lp_round(g, C, W, 6, 0, dir_alternate=0)
    assert m == 2 and prop[1] == 1 and C[1] == 0


@pytest.mark.parametrize("dirs", [0, 1])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_active_first_rounds_equal_full_rounds(dirs, seed):
    # every vertex starts owing one evaluation per direction, so the first
    # (1 + dirs) rounds are full rounds
    g = graphgen.random_small(150, 0.05, seed, wmax=5, vmax=3)
    R = 1 + dirs
    a, sa = oracle.lp_cluster(g, 12, R, dirs)
    b, sb = oracle.lp_cluster(g, 12, R, dirs, active=True)
    assert np.array_equal(a, b) and sa == sb
    n = len(g["xadj"]) - 1
    part = (np.arange(n) * 7 % 5).astype(np.int32)
    lm = oracle.lmax(int(g["vwgt"].sum()), 5, 0.03)
    a, sa = oracle.lp_refine(g, part, 5, lm, R, dirs)
    b, sb = oracle.lp_refine(g, part, 5, lm, R, dirs, active=True)
    assert np.array_equal(a, b) and sa == sb


@pytest.mark.parametrize("dirs", [0, 1])
def test_active_invariants(dirs):
    g = graphgen.rmat(11, 6)
    n = len(g["xadj"]) - 1
    nnz = len(g["adjncy"])
    lab, st = oracle.lp_cluster(g, 40, 10, dirs, active=True)
    full, sf = oracle.lp_cluster(g, 40, 10, dirs)
    W = np.bincount(lab, minlength=n)
    assert W.max() <= 40 and W.sum() == n
    # never more visits than full rounds, and at least the first full round(s)
    assert (1 + dirs) * nnz <= st["edge_visits"] <= st["rounds_run"] * nnz
    part = (np.arange(n) * 11 % 8).astype(np.int32)
    lm = oracle.lmax(n, 8, 0.03)
    P, st = oracle.lp_refine(g, part, 8, lm, 25, dirs, active=True)
    B = np.bincount(P, minlength=8)
    assert B.sum() == n and B.max() <= max(lm, np.bincount(part, minlength=8).max())
    assert st["edge_visits"] <= st["rounds_run"] * nnz
    # a partition in active-set mode (coarsening, refinement, both) is valid and balanced
    full = oracle.partition(g, 8)[1]
    for mode in (1, 2, 3):
        p, r = oracle.partition(g, 8, active_set=mode)
        assert r["balanced"] == 1 and oracle.cut(g, p) == r["cut"]
        if mode == 2:  # coarsening unchanged, so the hierarchy is the same
            assert (r["levels"], r["edge_visits_cluster"]) == (full["levels"], full["edge_visits_cluster"])
            assert r["edge_visits_refine"] <= full["edge_visits_refine"]
