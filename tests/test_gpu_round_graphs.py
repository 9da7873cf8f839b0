"""GPU parity with LP rounds replayed as HIP graphs (GP_ROUND_GRAPHS=1).

By default every round is launched directly; the replay path records one
round's launch sequence per LP run and replays it. Both must give the
oracle's labels, counters and partitions bit for bit: plain graphs of every
size class (the one-workgroup round tail below 16,385 vertices and the
multi-kernel round above), active sets and the batched form.
"""
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture
def replay():
    old = os.environ.get("GP_ROUND_GRAPHS")
    os.environ["GP_ROUND_GRAPHS"] = "1"
    yield
    if old is None:
        del os.environ["GP_ROUND_GRAPHS"]
    else:
        os.environ["GP_ROUND_GRAPHS"] = old


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", ["rgg16k", "rmat16", "grid"])
def test_replayed_rounds_match_oracle(replay, name):
    g = {"rgg16k": lambda: graphgen.rgg2d(16384, 1), "rmat16": lambda: graphgen.rmat(16, 16),
         "grid": lambda: graphgen.grid3d(20, 17, 9, seed=3, wmax=10)}[name]()
    dg = gp.to_device(g)
    lab, st = gp.lp_cluster(dg, 200, 10)
    olab, ost = oracle.lp_cluster(g, 200, 10)
    assert np.array_equal(_np(lab), olab)
    assert (st["rounds_run"], st["moves"], st["edge_visits"]) == (ost["rounds_run"], ost["moves"], ost["edge_visits"])
    k = 8
    part, res = gp.partition(dg, k, 0.03)
    opart, ores = oracle.partition(g, k, 0.03)
    assert np.array_equal(_np(part), opart) and res["cut"] == ores["cut"]
    part2, res2 = gp.partition(dg, k, 0.03, active_set=3)
    opart2, ores2 = oracle.partition(g, k, 0.03, active_set=3)
    assert np.array_equal(_np(part2), opart2) and res2["cut"] == ores2["cut"]


def test_replayed_rounds_batch(replay):
    graphs, ks = graphgen.batch(master_seed=4, count=12, log2_min=6, log2_max=12)
    u, off = gp.union_graph(graphs)
    part, res, _ = gp.partition_batch(gp.to_device(u), off, ks, 0.03)
    part = part.cpu().numpy()
    for q, (g, k) in enumerate(zip(graphs, ks)):
        op, ores = oracle.partition(g, k, 0.03)
        assert np.array_equal(part[off[q]:off[q + 1]], op), q
        assert res[q]["cut"] == ores["cut"], q
