"""GPU parity of refinement with connection rows.

On levels above 16,384 vertices the refinement keeps, for every vertex above
KT/8 neighbours (KT = 16, 64 or 256 from k), its k connection sums from round
to round and changes them only by the admitted moves. The labels, rounds and
moves must be the oracle's bit for bit, as with the plain rounds
(GP_REFINE_ROWS=0): every row width, unit and weighted edges, vertex weights,
64-bit sums, movers above 256 neighbours (queued as chunks), active sets,
rounds without the direction rule, and whole partitions.
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


def _np(t):
    return t.detach().cpu().numpy()


def _with_vwgt(g, seed):
    h = dict(g)
    n = len(g["xadj"]) - 1
    h["vwgt"] = np.array([1 + graphgen.rand_u64(seed, i) % 5 for i in range(n)], np.int32)
    return h


def _heavy(g, scale):
    """Symmetric edge weights large enough that sums need 64 bits."""
    h = dict(g)
    n = len(g["xadj"]) - 1
    rows = np.repeat(np.arange(n), np.diff(g["xadj"]))
    lo, hi = np.minimum(rows, g["adjncy"]), np.maximum(rows, g["adjncy"])
    w = (((lo.astype(np.int64) * 1000003 + hi) * 2654435761) % scale) + scale // 2
    h["adjwgt"] = w.astype(np.int32)
    assert int(h["adjwgt"].astype(np.int64).sum()) >= 2 ** 31
    return h


GRAPHS = {
    "rmat16": lambda: graphgen.rmat(16, 16),
    "rgg40k": lambda: graphgen.rgg2d(40000, 2),
    "grid_w": lambda: graphgen.grid3d(40, 35, 30, seed=5, wmax=10),
    "rmat15_vw": lambda: _with_vwgt(graphgen.rmat(15, 7), 3),
    "rmat15_heavy": lambda: _heavy(graphgen.rmat(15, 8), 1 << 22),
}
_cache = {}


def _graph(name):
    if name not in _cache:
        g = GRAPHS[name]()
        _cache[name] = (g, gp.to_device(g))
    return _cache[name]


@pytest.fixture(params=["rows", "plain"])
def mode(request):
    old = os.environ.get("GP_REFINE_ROWS")
    if request.param == "plain":
        os.environ["GP_REFINE_ROWS"] = "0"
    else:
        os.environ.pop("GP_REFINE_ROWS", None)
    yield request.param
    if old is None:
        os.environ.pop("GP_REFINE_ROWS", None)
    else:
        os.environ["GP_REFINE_ROWS"] = old


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("k", [2, 16, 64, 200])
def test_refine_matches_oracle(mode, name, k):
    g, dg = _graph(name)
    n = len(g["xadj"]) - 1
    assert n > 16384  # above the one-workgroup round tail
    part = np.array([graphgen.rand_u64(k + 1, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(oracle.total_vwgt(g), k, 0.03)
    P, st = gp.lp_refine(dg, torch.from_numpy(part).cuda(), k, lm, 25)
    oP, ost = oracle.lp_refine(g, part, k, lm, 25)
    assert np.array_equal(_np(P), oP)
    assert (st["rounds_run"], st["moves"]) == (ost["rounds_run"], ost["moves"])


@pytest.mark.parametrize("name", ["rmat16", "grid_w", "rmat15_heavy"])
def test_refine_active_and_undirected_rounds(mode, name):
    g, dg = _graph(name)
    n = len(g["xadj"]) - 1
    k = 16
    part = np.array([graphgen.rand_u64(5, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(oracle.total_vwgt(g), k, 0.03)
    dp = torch.from_numpy(part).cuda()
    P, st = gp.lp_refine(dg, dp, k, lm, 25, active=True)
    oP, ost = oracle.lp_refine(g, part, k, lm, 25, active=True)
    assert np.array_equal(_np(P), oP) and st["moves"] == ost["moves"]
    P, st = gp.lp_refine(dg, dp, k, lm, 12, dir_alternate=0)
    oP, ost = oracle.lp_refine(g, part, k, lm, 12, dir_alternate=0)
    assert np.array_equal(_np(P), oP) and st["moves"] == ost["moves"]


def test_big_movers_are_chunked():
    # hubs above 256 neighbours move in the first rounds from a random start
    g, dg = _graph("rmat16")
    n = len(g["xadj"]) - 1
    deg = np.diff(g["xadj"])
    k = 64
    part = np.array([graphgen.rand_u64(k + 1, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(n, k, 0.03)
    P, _ = gp.lp_refine(dg, torch.from_numpy(part).cuda(), k, lm, 1)
    moved = _np(P) != part
    assert np.count_nonzero(moved & (deg > 256)) > 0
    assert np.count_nonzero(moved & (deg > 4096)) > 0 or deg.max() <= 4096


@pytest.mark.parametrize("name,k", [("rmat16", 16), ("grid_w", 64), ("rmat15_vw", 8)])
def test_partition_matches_oracle(mode, name, k):
    g, dg = _graph(name)
    part, res = gp.partition(dg, k, 0.03)
    opart, ores = oracle.partition(g, k, 0.03)
    assert np.array_equal(_np(part), opart) and res["cut"] == ores["cut"]
