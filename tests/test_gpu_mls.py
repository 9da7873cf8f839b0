"""GPU parity of the multi-try k-way local search (§III-C; the batched form
of §IV-C's parallel MLS) with the oracle's orc_mls_batched: the same
partition, gain, searches, kept moves and local iterations, for several
batch sizes and queue bounds, standalone (gp_mls_refine) and after every
level's LP refinement inside the multilevel partition (gp_params.mls)."""
import numpy as np
import pytest

import graphgen
import oracle

GRAPHS = {
    "rgg16k": (lambda: graphgen.rgg2d(16384, 1), 2),
    "rgg17_k16": (lambda: graphgen.rgg2d(1 << 15, 6), 16),
    "grid_w": (lambda: graphgen.grid3d(24, 20, 16, seed=3, wmax=10), 64),
    "rmat16": (lambda: graphgen.rmat(16, 16), 16),
}


def _start(g, k):
    # the LP-only multilevel partition, a realistic start for the search
    part, res = oracle.partition(g, k, 0.03)
    return part, res["lmax"]


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("batch,queue", [(1, 64), (64, 64), (1024, 64), (256, 16)])
def test_mls_refine_matches_oracle(name, batch, queue):
    import torch
    import paper_1710_08231_amd as gp
    make, k = GRAPHS[name]
    g = make()
    part, lm = _start(g, k)
    want, ost = oracle.mls(g, part, k, lm, seed=5, global_iters=3, batch=batch, max_queue=queue)
    got, st = gp.mls_refine(gp.to_device(g), torch.from_numpy(part).cuda(), k, lm, seed=5, global_iters=3,
                            batch=batch, queue=queue)
    got = got.cpu().numpy()
    assert (st["gain"], st["searches"], st["moves"], st["local_iters"]) == \
           (ost["gain"], ost["searches"], ost["moves"], ost["local_iters"])
    assert np.array_equal(got, want)
    assert oracle.cut(g, got) == oracle.cut(g, part) - st["gain"]


@pytest.mark.gpu
def test_mls_worked_example_and_lmax():
    # two moves, each losing alone, together gain 6 (see the oracle pins)
    import torch
    import paper_1710_08231_amd as gp
    edges = [(0, 1), (0, 2), (0, 3), (0, 4), (1, 5), (1, 6), (1, 7)] + [(i, 8) for i in range(2, 8)] + [(9, 10)]
    w = [5, 1, 1, 1, 1, 1, 1] + [3] * 6 + [10]
    g = graphgen.from_edges(11, edges, weights=w)
    part = np.array([0, 0, 1, 1, 1, 1, 1, 1, 1, 0, 0], np.int32)
    dg = gp.to_device(g)
    P, st = gp.mls_refine(dg, torch.from_numpy(part).cuda(), 2, 100)
    assert P.cpu().numpy().tolist() == [1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0] and st["gain"] == 6 and st["moves"] == 2
    P, st = gp.mls_refine(dg, torch.from_numpy(part).cuda(), 2, 8)
    assert P.cpu().numpy().tolist() == part.tolist() and st["gain"] == 0


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["rgg16k", "grid_w", "rmat16"])
@pytest.mark.parametrize("batch", [1, 1024])
def test_partition_with_mls_matches_oracle(name, batch):
    import paper_1710_08231_amd as gp
    make, k = GRAPHS[name]
    g = make()
    prm = dict(mls=3, mls_batch=batch, mls_queue=64, seed=2)
    opart, ores = oracle.partition(g, k, 0.03, **prm)
    part, res = gp.partition(gp.to_device(g), k, 0.03, **prm)
    assert np.array_equal(part.cpu().numpy(), opart)
    assert (res["cut"], res["max_block_w"], res["levels"]) == (ores["cut"], ores["max_block_w"], ores["levels"])
    _, plain = oracle.partition(g, k, 0.03, seed=2)
    assert res["balanced"] == 1 and res["cut"] <= plain["cut"] and res["mls_gain"] > 0


@pytest.mark.gpu
def test_partition_with_mls_isolated_vertices():
    # R-MAT graphs have vertices without neighbours: level 0 hashes by rank among the others
    import paper_1710_08231_amd as gp
    g = graphgen.rmat(14, 44)
    assert (np.diff(g["xadj"]) == 0).any()
    prm = dict(mls=2, mls_batch=64, mls_queue=32)
    opart, ores = oracle.partition(g, 8, 0.03, **prm)
    part, res = gp.partition(gp.to_device(g), 8, 0.03, **prm)
    assert np.array_equal(part.cpu().numpy(), opart) and res["cut"] == ores["cut"]


@pytest.mark.gpu
def test_mls_argument_errors():
    import torch
    import paper_1710_08231_amd as gp
    g = graphgen.rgg2d(500, 3)
    dg = gp.to_device(g)
    part = torch.zeros(500, dtype=torch.int32, device="cuda")
    for kw in (dict(queue=0), dict(queue=65), dict(batch=0)):
        with pytest.raises(gp.GPError):
            gp.mls_refine(dg, part, 2, 300, **kw)
    with pytest.raises(gp.GPError):
        gp.mls_refine(dg, part + 5, 2, 300)
    with pytest.raises(gp.GPError):
        gp.partition(dg, 300, 0.03, mls=1)  # k > 256
    u, off = gp.union_graph([g, g])
    with pytest.raises(gp.GPError):
        gp.partition_batch(gp.to_device(u), off, [2, 2], 0.03, mls=1)
