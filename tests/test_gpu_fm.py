"""GPU parity of the 2-way FM local search after every initial bisection
(init_fm): whole partitions, bit for bit against the oracle in the same mode,
single graphs and batches."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

KEYS = ("cut", "max_block_w", "balanced", "levels", "coarsest_n", "edge_visits_cluster", "edge_visits_refine")


def _same(g, k, eps=0.03, **params):
    p, r = gp.partition(gp.to_device(g), k, eps, **params)
    op, ores = oracle.partition(g, k, eps, **params)
    assert np.array_equal(p.cpu().numpy(), op)
    for key in KEYS:
        assert r[key] == ores[key], key
    return ores


def test_fm_worked_two_cliques():
    # K4 {0..3} and K4 {4..7} joined by 3-4 and 3-5; L_max = 5 (eps 0.25):
    # the bisections end at the two cliques (cut 2)
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    edges += [(a, b) for a in range(4, 8) for b in range(a + 1, 8)] + [(3, 4), (3, 5)]
    g = graphgen.from_edges(8, edges)
    seed = next(s for s in range(1000) if oracle.mix4(s, 0, 0, 2) % 8 == 4)
    for fm in (0, 1, 3):
        r = _same(g, 2, 0.25, init_fm=fm, seed=seed, attempts=1, rounds_refine=0)
        assert r["cut"] == (6 if fm == 0 else 2)


CASES = {
    "rgg16k": (lambda: graphgen.rgg2d(16384, 1), (2, 16)),
    "rgg32k": (lambda: graphgen.rgg2d(1 << 15, 3), (3, 64)),
    "rmat14": (lambda: graphgen.rmat(14, 4), (2, 16)),
    "grid": (lambda: graphgen.grid3d(24, 20, 16, seed=3, wmax=9), (8, 64)),
    "weighted": (lambda: graphgen.random_small(400, 0.04, 9, wmax=9, vmax=5), (4, 7)),
    "star": (lambda: graphgen.from_edges(3001, [(0, i) for i in range(1, 3001)]), (2, 5)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fm", [1, 3])
def test_fm_partition_matches_oracle(name, fm):
    make, ks = CASES[name]
    g = make()
    for k in ks:
        _same(g, k, init_fm=fm)


@pytest.mark.parametrize("attempts", [1, 6])
def test_fm_attempts_and_seeds(attempts):
    g = graphgen.rgg2d(8000, 7)
    for seed in (0, 5):
        _same(g, 8, init_fm=2, attempts=attempts, seed=seed)


def test_fm_batch_matches_oracle():
    graphs, ks = graphgen.batch(master_seed=6, count=12, log2_min=6, log2_max=12)
    u, off = gp.union_graph(graphs)
    part, res, code = gp.partition_batch(gp.to_device(u), off, ks, 0.03, init_fm=3)
    part = part.cpu().numpy()
    for q, (g, k) in enumerate(zip(graphs, ks)):
        op, ores = oracle.partition(g, k, 0.03, init_fm=3)
        assert np.array_equal(part[off[q]:off[q + 1]], op), q
        assert res[q]["cut"] == ores["cut"], q


def test_fm_rejects_negative_passes():
    g = gp.to_device(graphgen.rgg2d(500, 1))
    with pytest.raises(gp.GPError):
        gp.partition(g, 4, init_fm=-1)


def test_fm_large_set_global_path():
    # n = 17000 <= 60 * 300: the graph is its own coarsest level, so the first
    # bisection's set (17000 vertices) is beyond the LDS search and uses the
    # global-memory one; the deeper, smaller sets use the LDS search
    g = graphgen.rgg2d(17000, 2)
    _same(g, 300, init_fm=2)


def _heavy(g, scale):
    # symmetric edge weights large enough that connection sums need 64 bits
    h = dict(g)
    n = len(g["xadj"]) - 1
    rows = np.repeat(np.arange(n), np.diff(g["xadj"]))
    lo, hi = np.minimum(rows, g["adjncy"]), np.maximum(rows, g["adjncy"])
    h["adjwgt"] = ((((lo.astype(np.int64) * 1000003 + hi) * 2654435761) % scale) + scale // 2).astype(np.int32)
    assert int(h["adjwgt"].astype(np.int64).sum()) >= 2 ** 31
    return h


@pytest.mark.parametrize("k", [2, 8])
def test_fm_heavy_weights_global_path(k):
    # 64-bit connection sums: gains stay in 64-bit words in global memory
    _same(_heavy(graphgen.rgg2d(6000, 5), 1 << 22), k, init_fm=3)
