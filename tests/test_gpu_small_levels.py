"""GPU parity on both sides of the small-level bounds of an LP round.

A level of at most 16,384 vertices runs everything of a round after the
proposals (mover compaction, stable sort by target, prefix admission, label and
weight updates, §IV-A's size-constrained moves) in one workgroup, and keeps the
label weights in LDS while there are at most 1,024 labels. Each bound is run
just below, at and just above it, for clustering (labels = vertices) and for
refinement (labels = blocks), on geometric graphs and on weighted grids of odd
shapes, against the oracle."""
import numpy as np
import pytest

import graphgen
import oracle

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

GRAPHS = {
    "rgg1023": graphgen.rgg2d(1023, 11),
    "rgg1024": graphgen.rgg2d(1024, 11),
    "rgg1025": graphgen.rgg2d(1025, 11),
    "grid1025w": graphgen.grid3d(5, 5, 41, seed=4, wmax=9),
    "rgg16383": graphgen.rgg2d(16383, 12),
    "rgg16384": graphgen.rgg2d(16384, 12),
    "rgg16385": graphgen.rgg2d(16385, 12),
    "grid16383w": graphgen.grid3d(3, 43, 127, seed=5, wmax=9),
    "grid16385w": graphgen.grid3d(5, 29, 113, seed=6, wmax=9),
}


@pytest.fixture(scope="module")
def dev():
    return {k: gp.to_device(v) for k, v in GRAPHS.items()}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("U,dirs", [(3, 1), (40, 1), (40, 0)])
def test_lp_cluster_around_small_level_bounds(dev, name, U, dirs):
    g = GRAPHS[name]
    lab, st = gp.lp_cluster(dev[name], U, rounds=10, dir_alternate=dirs)
    olab, ost = oracle.lp_cluster(g, U, 10, dirs)
    assert np.array_equal(lab.cpu().numpy(), olab)
    assert (st["rounds_run"], st["moves"], st["edge_visits"]) == (ost["rounds_run"], ost["moves"], ost["edge_visits"])


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["rgg16383", "rgg16384", "rgg16385", "grid16385w"])
@pytest.mark.parametrize("k", [2, 1023, 1024, 1025])
def test_lp_refine_around_small_level_bounds(dev, name, k):
    g = GRAPHS[name]
    n = len(g["xadj"]) - 1
    part = np.array([graphgen.rand_u64(k + 3, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(oracle.total_vwgt(g), k, 0.03)
    P, st = gp.lp_refine(dev[name], torch.from_numpy(part).cuda(), k, lm, 25)
    oP, ost = oracle.lp_refine(g, part, k, lm, 25)
    assert np.array_equal(P.cpu().numpy(), oP)
    assert (st["rounds_run"], st["moves"]) == (ost["rounds_run"], ost["moves"])
