"""The identity the refinement's connection rows rest on, checked on the CPU.

Refinement on the GPU keeps, for a vertex v, its connection sums
conn(v, b) = sum of w(v, u) over the neighbours u in block b, from round to
round, and changes them only by the admitted moves: a vertex u moved from a to
b takes w(u, v) off conn(v, a) and adds it to conn(v, b), reading the weight
from u's own list. On a symmetric graph (§II-A) that equals recomputing every
sum from the labels after the round. Here the oracle's rounds (run for r and
r + 1 rounds from the same start) supply the moves, and numpy both recomputes
and updates the sums; the two must agree exactly after every round, and an
asymmetric weight must break the identity (which is why the GPU path takes
symmetric graphs).
"""
import numpy as np

import graphgen
import oracle


def _conn(g, part, k):
    n = len(g["xadj"]) - 1
    rows = np.repeat(np.arange(n), np.diff(g["xadj"]))
    w = g["adjwgt"].astype(np.int64) if "adjwgt" in g else np.ones(len(rows), np.int64)
    c = np.zeros((n, k), np.int64)
    np.add.at(c, (rows, part[g["adjncy"]]), w)
    return c


def _push(g, c, before, after):
    # every moved u pushes w(u, v), read from u's own list, into the rows of its neighbours v
    c = c.copy()
    w_all = g["adjwgt"].astype(np.int64) if "adjwgt" in g else None
    for u in np.nonzero(before != after)[0]:
        e0, e1 = g["xadj"][u], g["xadj"][u + 1]
        nb = g["adjncy"][e0:e1]
        w = w_all[e0:e1] if w_all is not None else np.ones(e1 - e0, np.int64)
        np.add.at(c, (nb, np.full(len(nb), before[u])), -w)
        np.add.at(c, (nb, np.full(len(nb), after[u])), w)
    return c


def _rounds(g, k, seed, rounds):
    n = len(g["xadj"]) - 1
    part = np.array([graphgen.rand_u64(seed, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(oracle.total_vwgt(g), k, 0.03)
    out = [part]
    for r in range(1, rounds + 1):
        p, st = oracle.lp_refine(g, part, k, lm, r)
        out.append(p)
        if st["rounds_run"] < r:
            break
    return out


def test_updated_rows_equal_recomputed_rows():
    g = graphgen.random_small(400, 0.03, 11, wmax=9, vmax=4)
    k = 8
    parts = _rounds(g, k, 3, 12)
    assert len(parts) > 3 and any((a != b).any() for a, b in zip(parts, parts[1:]))
    c = _conn(g, parts[0], k)
    for before, after in zip(parts, parts[1:]):
        c = _push(g, c, before, after)
        assert np.array_equal(c, _conn(g, after, k))


def test_an_asymmetric_weight_breaks_the_identity():
    g = graphgen.random_small(200, 0.05, 5, wmax=9)
    k = 4
    parts = _rounds(g, k, 7, 6)
    before, after = parts[0], parts[1]
    u = int(np.nonzero(before != after)[0][0])
    h = dict(g)
    h["adjwgt"] = g["adjwgt"].copy()
    h["adjwgt"][g["xadj"][u]] += 1  # w(u, v) != w(v, u) for u's first neighbour v
    c = _push(h, _conn(h, before, k), before, after)
    assert not np.array_equal(c, _conn(h, after, k))
