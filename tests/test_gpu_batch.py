"""GPU parity of the batched form: every graph of a batch gets exactly the
oracle's single-graph partition (labels, cut, balance, levels, edge visits).

The batch mixes random geometric graphs, R-MAT graphs with many vertices
without neighbours, a weighted grid, a tiny graph below the coarsening
threshold, an empty graph and an all-isolated graph, with k in {1, 2, 3, 8, 32}.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

KEYS = ("cut", "max_block_w", "lmax", "ucl", "balanced", "levels", "coarsest_n", "n_isolated",
        "edge_visits_cluster", "edge_visits_refine")


def _check_batch(graphs, ks, eps=0.03, **params):
    u, off = gp.union_graph(graphs)
    part, res, code = gp.partition_batch(gp.to_device(u), off, ks, eps, **params)
    part = part.cpu().numpy()
    any_imb = False
    for q, (g, k) in enumerate(zip(graphs, ks)):
        op, ores = oracle.partition(g, k, eps, **params)
        assert np.array_equal(part[off[q]:off[q + 1]], op), f"graph {q}"
        for key in KEYS:
            assert res[q][key] == ores[key], (q, key)
        any_imb |= ores["code"] != 0
    assert code == (1 if any_imb else 0)


def test_batch_mixed_graphs():
    graphs, ks = graphgen.batch(master_seed=4, count=24, log2_min=6, log2_max=12)
    graphs += [graphgen.grid3d(9, 7, 5, seed=3, wmax=10), graphgen.from_edges(5, [(0, 1), (2, 3)]),
               graphgen.from_edges(0, []), graphgen.from_edges(6, []), graphgen.rgg2d(700, 9)]
    ks += [8, 2, 3, 2, 1]
    _check_batch(graphs, ks)


def test_batch_single_graph_equals_plain():
    g = graphgen.rmat(13, 7)
    _check_batch([g], [16])


@pytest.mark.parametrize("seed", [0, 5])
def test_batch_params(seed):
    graphs, ks = graphgen.batch(master_seed=11, count=10, log2_min=8, log2_max=11)
    _check_batch(graphs, ks, eps=0.05, seed=seed, attempts=3)


def test_batch_rejects_cross_edges():
    u, off = gp.union_graph([graphgen.from_edges(3, [(0, 1)]), graphgen.from_edges(3, [(0, 2)])])
    # join vertex 2 of graph 0 with vertex 3 of graph 1
    bad = graphgen.from_edges(6, [(0, 1), (3, 5), (2, 3)])
    with pytest.raises(gp.GPError):
        gp.partition_batch(gp.to_device(bad), off, [2, 2])


def test_batch_mixed_block_counts_and_hubs():
    # block counts on both sides of the refinement's table switches (64, 256, 300) in one
    # batch, with hubs of 2,049 to 9,000 neighbours and graphs just past 1,024 and 16,384 vertices
    rng = np.random.default_rng(3)
    n = 20000
    edges = [(int(u), int(v)) for u, v in rng.integers(0, n - 3, size=(3 * n, 2)) if u != v]
    for h, d in ((n - 3, 2049), (n - 2, 4097), (n - 1, 9000)):
        edges += [(h, int(u)) for u in rng.choice(n - 3, d, replace=False)]
    hubs = graphgen.from_edges(n, edges)
    graphs = [hubs, graphgen.rgg2d(16385, 12), graphgen.rmat(12, 5), graphgen.grid3d(5, 5, 41, seed=4, wmax=9),
              graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)]), graphgen.rgg2d(1025, 2)]
    _check_batch(graphs, [16, 300, 64, 256, 4, 65])
