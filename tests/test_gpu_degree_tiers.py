"""GPU parity with a vertex exactly on each side of every degree bound.

The proposal step (§III-A, §IV-A: the strongest eligible neighbouring label)
runs in kernels chosen by degree: lane groups of 4 to 64 lanes, workgroups of
128, 512 and 1024 threads with LDS tables, and the bucketed hub path above;
refinement switches from lane groups to chunked dense tables and keeps
connection rows above KT/8 neighbours. The bounds are tuning values. Here hubs
of exact degrees 1 .. 16,385 straddle every bound that the default tuning and
the committed per-workload tunings use, and clustering, refinement and a whole
partition must equal the oracle's under each of those tunings."""
import glob
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEGREES = [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512,
           513, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 16383, 16384, 16385]
N_PLAIN = 40000


def _hubs_graph(seed=7):
    # vertices 0 .. N_PLAIN-1 are plain (random sparse edges among themselves), then one hub
    # per entry of DEGREES whose neighbours are distinct plain vertices: its degree is exact
    rng = np.random.default_rng(seed)
    n = N_PLAIN + len(DEGREES)
    extra = rng.integers(0, N_PLAIN, size=(4 * N_PLAIN, 2))
    edges = [(int(u), int(v)) for u, v in extra if u != v]
    for i, d in enumerate(DEGREES):
        nbr = rng.choice(N_PLAIN, d, replace=False)
        edges += [(N_PLAIN + i, int(u)) for u in nbr]
    g = graphgen.from_edges(n, edges)
    assert np.diff(g["xadj"])[N_PLAIN:].tolist() == DEGREES
    return g


G = _hubs_graph()
TUNING_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1710_08231_amd",
                          "tuning")
TUNINGS = [("default", None)] + [(os.path.basename(p)[:-5], json.load(open(p))["tuning"])
                                 for p in sorted(glob.glob(os.path.join(TUNING_DIR, "*.json")))]


@pytest.fixture(scope="module")
def dg():
    return gp.to_device(G)


@pytest.fixture
def tuned(request):
    gp.set_tuning(request.param)
    yield request.param
    gp.set_tuning(None)


@pytest.mark.gpu
@pytest.mark.parametrize("tuned", [t for _, t in TUNINGS], ids=[n for n, _ in TUNINGS], indirect=True)
def test_cluster_refine_partition_at_exact_degree_bounds(dg, tuned):
    for U, dirs in [(3, 1), (60, 1), (60, 0), (20000, 1)]:
        lab, st = gp.lp_cluster(dg, U, 6, dirs)
        olab, ost = oracle.lp_cluster(G, U, 6, dirs)
        assert np.array_equal(lab.cpu().numpy(), olab), (U, dirs)
        assert {k: st[k] for k in ost} == ost, (U, dirs)
    n = len(G["xadj"]) - 1
    for k in (16, 64, 300):
        part = np.array([graphgen.rand_u64(k, i) % k for i in range(n)], np.int32)
        lm = oracle.lmax(n, k, 0.03)
        p, st = gp.lp_refine(dg, torch.from_numpy(part).cuda(), k, lm, 12)
        op, ost = oracle.lp_refine(G, part, k, lm, 12)
        assert np.array_equal(p.cpu().numpy(), op), k
        assert {key: st[key] for key in ost} == ost, k
    part, res = gp.partition(dg, 16, 0.03)
    opart, ores = oracle.partition(G, 16, 0.03)
    assert np.array_equal(part.cpu().numpy(), opart)
    assert res["cut"] == ores["cut"] and res["levels"] == ores["levels"]


@pytest.mark.gpu
def test_opt_in_modes_at_exact_degree_bounds(dg):
    # active-set rounds renew the neighbours of movers above 256 neighbours in chunks of 4,096
    # entries (hubs of 255-257, 4,095-4,097, 8,191-8,193 and 16,383-16,385 neighbours straddle
    # both), FM after the bisections and the batched multi-try local search see the same hubs
    n = len(G["xadj"]) - 1
    for U in (3, 60):
        lab, st = gp.lp_cluster(dg, U, 6, 1, active=True)
        olab, ost = oracle.lp_cluster(G, U, 6, 1, active=True)
        assert np.array_equal(lab.cpu().numpy(), olab), U
        assert {k: st[k] for k in ost} == ost, U
    part = np.array([graphgen.rand_u64(16, i) % 16 for i in range(n)], np.int32)
    lm = oracle.lmax(n, 16, 0.03)
    p, st = gp.lp_refine(dg, torch.from_numpy(part).cuda(), 16, lm, 12, 1, active=True)
    op, ost = oracle.lp_refine(G, part, 16, lm, 12, 1, active=True)
    assert np.array_equal(p.cpu().numpy(), op)
    assert {k: st[k] for k in ost} == ost
    for params in (dict(active_set=3), dict(init_fm=2), dict(mls=2, mls_batch=64, mls_queue=64)):
        part, res = gp.partition(dg, 16, 0.03, **params)
        opart, ores = oracle.partition(G, 16, 0.03, **params)
        assert np.array_equal(part.cpu().numpy(), opart), params
        assert res["cut"] == ores["cut"] and res["levels"] == ores["levels"], params
