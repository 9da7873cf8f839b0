"""The seeded input generators shared by the oracle and the GPU path produce
what both sides assume: CSR rows sorted strictly ascending (no duplicate
entries, no self-loops), a symmetric graph with equal weights on both
directions of an edge, weights >= 1, and the same arrays for the same seed."""
import numpy as np
import pytest

import graphgen


def _check_csr(g):
    x = np.asarray(g["xadj"], np.int64)
    a = np.asarray(g["adjncy"], np.int64)
    n = len(x) - 1
    assert x[0] == 0 and x[-1] == len(a) and np.all(np.diff(x) >= 0)
    assert len(a) == 0 or (a.min() >= 0 and a.max() < n)
    rows = np.repeat(np.arange(n), np.diff(x))
    assert not np.any(rows == a)  # no self-loops
    # strictly ascending inside every row
    inner = np.diff(a)
    same_row = np.diff(rows) == 0
    assert np.all(inner[same_row] > 0)
    # symmetric, with the same weight both ways
    w = np.ones(len(a), np.int64) if g.get("adjwgt") is None else np.asarray(g["adjwgt"], np.int64)
    assert np.all(w >= 1)
    fwd = rows * n + a
    bwd = a * n + rows
    o1, o2 = np.argsort(fwd), np.argsort(bwd)
    assert np.array_equal(fwd[o1], bwd[o2]) and np.array_equal(w[o1], w[o2])
    if g.get("vwgt") is not None:
        assert len(g["vwgt"]) == n and np.all(np.asarray(g["vwgt"]) >= 1)


def _same(g, h):
    return all(
        (g.get(key) is None and h.get(key) is None) or np.array_equal(g[key], h[key])
        for key in ("xadj", "adjncy", "adjwgt", "vwgt"))


CASES = {
    "rgg": lambda s: graphgen.rgg2d(3000, s),
    "rmat": lambda s: graphgen.rmat(12, s),
    "rmat_m": lambda s: graphgen.rmat_m(11, 20000, s),
    "grid": lambda s: graphgen.grid3d(9, 8, 7, seed=s, wmax=9),
    "random_small": lambda s: graphgen.random_small(150, 0.06, s, wmax=7, vmax=4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_generator_csr_contract_and_seeding(name):
    make = CASES[name]
    g1, g2, g3 = make(5), make(5), make(6)
    _check_csr(g1)
    _check_csr(g3)
    assert _same(g1, g2)
    assert not _same(g1, g3)


def test_from_edges_normalises():
    # duplicates merge, both directions appear once, rows come out sorted
    g = graphgen.from_edges(5, [(3, 1), (1, 3), (0, 4), (2, 0), (4, 0)])
    _check_csr(g)
    assert g["xadj"].tolist() == [0, 2, 3, 4, 5, 6]
    assert g["adjncy"].tolist() == [2, 4, 3, 0, 1, 0]


def test_batch_graphs_are_valid():
    graphs, ks = graphgen.batch(master_seed=3, count=16, log2_min=6, log2_max=10)
    assert len(graphs) == len(ks) == 16
    for g, k in zip(graphs, ks):
        _check_csr(g)
        assert k >= 1
