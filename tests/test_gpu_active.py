"""GPU parity of the active-set LP rounds (GP_LP_ACTIVE_SET, gp_params.active_set)
against the oracle, bit-exact: labels, rounds, moves and edge visits, in every
proposal tier (group lanes, workgroup tables, chunked and global-table hubs,
dense refinement tables), with 32- and 64-bit connection sums, and through
the multilevel partition."""
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


def _star(n_leaves, extra=()):
    edges = [(0, i) for i in range(1, n_leaves + 1)] + list(extra)
    return graphgen.from_edges(n_leaves + 1, edges)


def _heavy(g, scale, seed):
    h = dict(g)
    n = len(g["xadj"]) - 1
    rows = np.repeat(np.arange(n), np.diff(g["xadj"]))
    lo, hi = np.minimum(rows, g["adjncy"]), np.maximum(rows, g["adjncy"])
    w = (((lo.astype(np.int64) * 1000003 + hi) * 2654435761) % scale) + scale // 2
    h["adjwgt"] = w.astype(np.int32)
    return h


CASES = {
    "rgg16k": graphgen.rgg2d(16384, 1),
    "rmat12": graphgen.rmat(12, 12),
    "rmat16": graphgen.rmat(16, 16),
    "grid": graphgen.grid3d(20, 17, 9, seed=3, wmax=10),
    "star_hub": _star(20000, extra=[(1, 2), (3, 4), (5, 6)]),
    "weighted": graphgen.random_small(300, 0.05, 9, wmax=9, vmax=5),
    "heavy_rmat13": _heavy(graphgen.rmat(13, 3), 1 << 22, 1),
    "heavy_star": _heavy(_star(20000, extra=[(1, 2), (3, 4)]), 1 << 20, 2),
}


@pytest.fixture(scope="module")
def dev_cases():
    return {k: gp.to_device(v) for k, v in CASES.items()}


def _lp_stats_equal(st, ost):
    for key in ("rounds_run", "moves", "edge_visits"):
        assert st[key] == ost[key], key


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dirs", [0, 1])
def test_active_cluster_matches_oracle(dev_cases, name, dirs):
    g = CASES[name]
    for U in (6, 300):
        lab, st = gp.lp_cluster(dev_cases[name], U, 10, dirs, active=True)
        olab, ost = oracle.lp_cluster(g, U, 10, dirs, active=True)
        assert np.array_equal(_np(lab), olab), U
        _lp_stats_equal(st, ost)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k", [2, 16, 300])
def test_active_refine_matches_oracle(dev_cases, name, k):
    g = CASES[name]
    n = len(g["xadj"]) - 1
    part = np.array([graphgen.rand_u64(k, i) % k for i in range(n)], np.int32)
    W = oracle.total_vwgt(g)
    lm = oracle.lmax(W, k, 0.03)
    for dirs in (0, 1):
        P, st = gp.lp_refine(dev_cases[name], torch.from_numpy(part).cuda(), k, lm, 25, dirs, active=True)
        oP, ost = oracle.lp_refine(g, part, k, lm, 25, dirs, active=True)
        assert np.array_equal(_np(P), oP), dirs
        _lp_stats_equal(st, ost)


def test_active_worked_examples():
    # the oracle's hand-derived examples, through the C ABI
    edges = [(0, 1), (0, 2), (1, 3), (2, 4), (5, 6), (5, 7), (6, 7)]
    g = gp.to_device(graphgen.from_edges(8, edges))
    part = torch.tensor([0, 1, 1, 1, 1, 1, 0, 0], dtype=torch.int32).cuda()
    P, st = gp.lp_refine(g, part, 2, 5, 25, 0, active=True)
    assert _np(P).tolist() == [0, 1, 1, 1, 1, 0, 0, 0]
    assert (st["rounds_run"], st["moves"], st["edge_visits"]) == (3, 1, 18)
    P, st = gp.lp_refine(g, part, 2, 5, 25, 1, active=True)
    assert _np(P).tolist() == [1, 1, 1, 1, 1, 0, 0, 0]
    assert (st["rounds_run"], st["moves"], st["edge_visits"]) == (4, 2, 40)
    edges = [(0, 2), (0, 3), (1, 4), (1, 5), (2, 3), (4, 5), (6, 7), (6, 8), (7, 8)]
    g = gp.to_device(graphgen.from_edges(9, edges))
    part = torch.tensor([0, 0, 1, 1, 1, 1, 1, 0, 0], dtype=torch.int32).cuda()
    P, st = gp.lp_refine(g, part, 2, 6, 25, 0, active=True)
    assert _np(P).tolist() == [1, 1, 1, 1, 1, 1, 0, 0, 0]
    assert (st["rounds_run"], st["moves"], st["edge_visits"]) == (4, 3, 32)


@pytest.mark.parametrize("tuning", [
    {"tier_max": [16, 16, 16, 16], "dense_split": 16, "dense_chunk": 256},
    {"tier_max": [32, 128, 1024, 4096], "dense_split": 1024, "dense_chunk": 8192},
])
def test_active_under_tuning(tuning):
    g = graphgen.rmat(13, 4)
    n = len(g["xadj"]) - 1
    try:
        gp.set_tuning(tuning)
        dg = gp.to_device(g)
        lab, st = gp.lp_cluster(dg, 200, 10, 1, active=True)
        olab, ost = oracle.lp_cluster(g, 200, 10, 1, active=True)
        assert np.array_equal(_np(lab), olab)
        _lp_stats_equal(st, ost)
        part = (np.arange(n) * 7919 % 16).astype(np.int32)
        lm = oracle.lmax(n, 16, 0.03)
        P, st = gp.lp_refine(dg, torch.from_numpy(part).cuda(), 16, lm, 25, 1, active=True)
        oP, ost = oracle.lp_refine(g, part, 16, lm, 25, 1, active=True)
        assert np.array_equal(_np(P), oP)
        _lp_stats_equal(st, ost)
    finally:
        gp.set_tuning(None)


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("name,k", [("rgg16k", 2), ("rmat12", 16), ("rmat16", 16), ("grid", 8), ("weighted", 5),
                                    ("star_hub", 4), ("rgg16k", 64)])
def test_active_partition_matches_oracle(dev_cases, name, k, mode):
    # mode: bit 0 coarsening, bit 1 refinement in active-set rounds
    g = CASES[name]
    p, r = gp.partition(dev_cases[name], k, 0.03, active_set=mode)
    op, ores = oracle.partition(g, k, active_set=mode)
    assert np.array_equal(_np(p), op)
    for key in ("cut", "max_block_w", "levels", "coarsest_n", "edge_visits_cluster", "edge_visits_refine"):
        assert r[key] == ores[key], key


def test_active_set_rejected_by_batch():
    graphs = [graphgen.rmat(10, 3), graphgen.rgg2d(1000, 2)]
    u, off = gp.union_graph(graphs)
    with pytest.raises(gp.GPError):
        gp.partition_batch(gp.to_device(u), off, [4, 4], 0.03, active_set=1)


def test_lp_rejects_unknown_flags(dev_cases):
    import ctypes
    gs = gp._gstruct(dev_cases["rmat12"])
    lab = torch.empty(gs.n, dtype=torch.int32, device="cuda")
    st = gp.LPStats()
    rc = gp.load().gp_lp_cluster(ctypes.byref(gs), 10, 5, 4, gp._ptr(lab), ctypes.byref(st), None, 0, gp._stream())
    assert rc < 0


def test_active_rmat22_refine_rounds_full():
    # level-0 size: dense refinement with chunked big vertices, active sets
    g = graphgen.rmat(22, 22)
    dg = gp.to_device(g)
    n = len(g["xadj"]) - 1
    part = (np.arange(n) * 7919 % 16).astype(np.int32)
    lm = oracle.lmax(n, 16, 0.03)
    P, st = gp.lp_refine(dg, torch.from_numpy(part).cuda(), 16, lm, 4, 1, active=True)
    oP, ost = oracle.lp_refine(g, part, 16, lm, 4, 1, active=True)
    assert np.array_equal(_np(P), oP)
    _lp_stats_equal(st, ost)
