"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Inputs are seeded synthetic graphs from graphgen (shared input generator);
expected values come from the oracle only. Sizes are small enough for the
oracle to finish in seconds but span several tiles, every degree tier of the
proposal kernels (including the global-table hub tier), ragged tails, empty
inputs and isolated vertices.
"""
import json
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lp_worked_vectors.json")


def _np(t):
    return t.detach().cpu().numpy()


def _star(n_leaves, extra=()):
    edges = [(0, i) for i in range(1, n_leaves + 1)] + list(extra)
    return graphgen.from_edges(n_leaves + 1, edges)


def _cases():
    cases = {
        "rgg2k": graphgen.rgg2d(2000, 3),
        "rgg16k": graphgen.rgg2d(16384, 1),
        "rmat12": graphgen.rmat(12, 12),
        "rmat16": graphgen.rmat(16, 16),
        "grid": graphgen.grid3d(20, 17, 9, seed=3, wmax=10),
        "star_hub": _star(20000),
        "star_wg": _star(3000),
        "star_wg2": _star(6000),
        "weighted": graphgen.random_small(300, 0.05, 9, wmax=9, vmax=5),
    }
    return cases


CASES = _cases()


@pytest.fixture(scope="module")
def dev_cases():
    return {k: gp.to_device(v) for k, v in CASES.items()}


def test_library_exports():
    lib = gp.load()
    for name in gp.EXPORTS:
        assert hasattr(lib, name)


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_worked_vectors_on_gpu(case):
    g = graphgen.from_edges(case["n"], case["edges"], vwgt=case.get("vwgt"))
    dg = gp.to_device(g)
    if case["mode"] == "cluster":
        lab, st = gp.lp_cluster(dg, case["U"], case["rounds"])
    else:
        part = torch.tensor(case["part_in"], dtype=torch.int32, device="cuda")
        lab, st = gp.lp_refine(dg, part, case["k"], case["lmax"], case["rounds"])
    assert _np(lab).tolist() == case["labels"]
    assert st["rounds_run"] == case["rounds_run"] and st["moves"] == case["moves"]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("U", [3, 40, 1000])
def test_lp_cluster_matches_oracle(dev_cases, name, U):
    g = CASES[name]
    vmax = int(g["vwgt"].max()) if "vwgt" in g else 1
    U = max(U, vmax)
    lab, st = gp.lp_cluster(dev_cases[name], U, 10)
    olab, ost = oracle.lp_cluster(g, U, 10)
    assert np.array_equal(_np(lab), olab)
    assert (st["rounds_run"], st["moves"], st["edge_visits"]) == (ost["rounds_run"], ost["moves"], ost["edge_visits"])


@pytest.mark.parametrize("name", ["rgg16k", "rmat12", "grid", "weighted"])
def test_lp_cluster_without_direction_rule(dev_cases, name):
    g = CASES[name]
    lab, st = gp.lp_cluster(dev_cases[name], 30, 7, dir_alternate=0)
    olab, ost = oracle.lp_cluster(g, 30, 7, dir_alternate=0)
    assert np.array_equal(_np(lab), olab) and st["rounds_run"] == ost["rounds_run"]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k", [2, 16, 64])
def test_lp_refine_matches_oracle(dev_cases, name, k):
    g = CASES[name]
    n = len(g["xadj"]) - 1
    part = np.array([graphgen.rand_u64(k, i) % k for i in range(n)], np.int32)
    W = oracle.total_vwgt(g)
    lm = oracle.lmax(W, k, 0.03)
    dp = torch.from_numpy(part).cuda()
    P, st = gp.lp_refine(dev_cases[name], dp, k, lm, 25)
    oP, ost = oracle.lp_refine(g, part, k, lm, 25)
    assert np.array_equal(_np(P), oP)
    assert (st["rounds_run"], st["moves"]) == (ost["rounds_run"], ost["moves"])


@pytest.mark.parametrize("name", list(CASES))
def test_contract_matches_oracle(dev_cases, name):
    g = CASES[name]
    olab, _ = oracle.lp_cluster(g, 50, 10)
    ocg, of2c = oracle.contract(g, olab)
    cg, f2c = gp.contract(dev_cases[name], torch.from_numpy(olab).cuda())
    assert np.array_equal(_np(f2c), of2c)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg[key]), ocg[key]), key


def test_contract_arbitrary_labels():
    g = graphgen.random_small(200, 0.1, 4, wmax=3, vmax=2)
    n = 200
    lab = np.array([graphgen.rand_u64(77, i) % 37 * 5 for i in range(n)], np.int32)
    ocg, of2c = oracle.contract(g, lab)
    cg, f2c = gp.contract(gp.to_device(g), torch.from_numpy(lab).cuda())
    assert np.array_equal(_np(f2c), of2c)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg[key]), ocg[key]), key


def test_contract_label_groups_without_edges():
    # many vertices without neighbours share labels: rows with more members than entries,
    # in each size class (wave, workgroup, global)
    edges = [(i, i + 1) for i in range(0, 400, 2)]
    g = graphgen.from_edges(7000, edges)
    lab = np.zeros(7000, np.int32)
    lab[:400] = np.arange(400) // 2 * 2
    lab[400:500] = 401
    lab[500:3000] = 403
    lab[3000:] = 405
    ocg, of2c = oracle.contract(g, lab)
    cg, f2c = gp.contract(gp.to_device(g), torch.from_numpy(lab).cuda())
    assert np.array_equal(_np(f2c), of2c)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg[key]), ocg[key]), key


def test_contract_large_row_with_members_without_edges():
    # one coarse row of 3000 entries (two hubs of 1500 distinct neighbours) whose
    # 6002 members are mostly vertices without neighbours, listed between the two
    # hubs: a chunk of the row then spans more members than it has entries
    edges = [(0, 6002 + j) for j in range(1500)] + [(6001, 7502 + j) for j in range(1500)]
    g = graphgen.from_edges(9002, edges)
    lab = np.arange(9002, dtype=np.int32)
    lab[:6002] = 0
    ocg, of2c = oracle.contract(g, lab)
    cg, f2c = gp.contract(gp.to_device(g), torch.from_numpy(lab).cuda())
    assert np.array_equal(_np(f2c), of2c)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg[key]), ocg[key]), key


def test_contract_large_rows():
    # a coarse row with > 2048 entries and many distinct columns (global class) next to small rows
    g = graphgen.rmat(14, 3)
    n = len(g["xadj"]) - 1
    lab = np.array([(v // 64) * 64 if v < 4096 else v for v in range(n)], np.int32)
    ocg, of2c = oracle.contract(g, lab)
    cg, f2c = gp.contract(gp.to_device(g), torch.from_numpy(lab).cuda())
    assert np.array_equal(_np(f2c), of2c)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg[key]), ocg[key]), key


def test_contract_rows_above_2048_entries_weighted():
    # many coarse rows of 2,049..8,192 entries and above (chunked, pair-sorted class)
    # beside rows of every other class; then the weighted coarse graph once more
    g = graphgen.rmat(15, 7)
    n = len(g["xadj"]) - 1
    lab = np.array([(v // 256) * 256 if v < 16384 else v for v in range(n)], np.int32)
    D = np.bincount(lab, weights=np.diff(g["xadj"]), minlength=n)
    assert ((D > 2048) & (D <= 8192)).sum() >= 10 and (D > 8192).sum() >= 10
    ocg, of2c = oracle.contract(g, lab)
    cg, f2c = gp.contract(gp.to_device(g), torch.from_numpy(lab).cuda())
    assert np.array_equal(_np(f2c), of2c)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg[key]), ocg[key]), key
    nc = len(ocg["xadj"]) - 1
    lab2 = np.array([(v // 32) * 32 for v in range(nc)], np.int32)
    D2 = np.bincount(lab2, weights=np.diff(ocg["xadj"]), minlength=nc)
    assert ((D2 > 2048) & (D2 <= 8192)).sum() >= 5
    ocg2, of2c2 = oracle.contract(ocg, lab2)
    cg2, f2c2 = gp.contract(gp.to_device(ocg), torch.from_numpy(lab2).cuda())
    assert np.array_equal(_np(f2c2), of2c2)
    for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
        assert np.array_equal(_np(cg2[key]), ocg2[key]), key


def test_contract_weight_overflow_in_large_rows():
    # coarse rows of 3,000 entries to one column of weight 2^30 each: the sum does not
    # fit the int32 coarse weight, so the call fails with GP_ERR_OVERFLOW
    n = 3001
    g = graphgen.from_edges(n, [(v, 3000) for v in range(3000)], weights=[1 << 30] * 3000)
    lab = np.arange(n, dtype=np.int32)
    lab[:3000] = 0
    with pytest.raises(gp.GPError, match="overflow"):
        gp.contract(gp.to_device(g), torch.from_numpy(lab).cuda())


def test_project_and_cut():
    g = graphgen.rmat(12, 5)
    dg = gp.to_device(g)
    olab, _ = oracle.lp_cluster(g, 20, 10)
    ocg, of2c = oracle.contract(g, olab)
    nc = len(ocg["xadj"]) - 1
    pc = np.array([graphgen.rand_u64(3, i) % 7 for i in range(nc)], np.int32)
    pf = gp.project(torch.from_numpy(of2c).cuda(), torch.from_numpy(pc).cuda())
    assert np.array_equal(_np(pf), oracle.project(of2c, pc))
    cut, B = gp.cut_and_blocks(dg, pf, 7)
    assert cut == oracle.cut(g, _np(pf))
    assert np.array_equal(_np(B), oracle.block_weights(g, _np(pf), 7))


PART_CASES = [
    ("rgg16k", 2), ("rgg2k", 8), ("rmat12", 16), ("rmat16", 16), ("grid", 8), ("weighted", 5),
    ("star_hub", 4), ("rgg16k", 64),
]


@pytest.mark.parametrize("name,k", PART_CASES)
def test_partition_matches_oracle(dev_cases, name, k):
    g = CASES[name]
    part, res = gp.partition(dev_cases[name], k, 0.03)
    opart, ores = oracle.partition(g, k, 0.03)
    assert np.array_equal(_np(part), opart)
    for key in ("cut", "max_block_w", "lmax", "ucl", "balanced", "levels", "coarsest_n", "n_isolated",
                "edge_visits_cluster", "edge_visits_refine"):
        assert res[key] == ores[key], key
    assert res["code"] == ores["code"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_partition_seeds_and_attempts(dev_cases, seed):
    g = CASES["rmat12"]
    part, res = gp.partition(dev_cases["rmat12"], 8, 0.05, seed=seed, attempts=3)
    opart, ores = oracle.partition(g, 8, 0.05, seed=seed, attempts=3)
    assert np.array_equal(_np(part), opart) and res["cut"] == ores["cut"]


def test_partition_edge_cases():
    # empty graph, all-isolated, graph smaller than the coarsening threshold, k=1
    for g, k in [(graphgen.from_edges(0, []), 2), (graphgen.from_edges(9, []), 4),
                 (graphgen.from_edges(7, [(0, 1), (1, 2), (4, 5)]), 3),
                 (graphgen.rgg2d(500, 2), 1), (graphgen.random_small(50, 0.1, 2, wmax=4, vmax=7), 3)]:
        n = len(g["xadj"]) - 1
        opart, ores = oracle.partition(g, k, 0.03)
        part, res = gp.partition(gp.to_device(g), k, 0.03)
        assert np.array_equal(_np(part)[:n], opart)
        assert res["cut"] == ores["cut"] and res["code"] == ores["code"]


def test_errors_are_reported():
    g = gp.to_device(graphgen.rgg2d(100, 1))
    with pytest.raises(gp.GPError):
        gp.partition(g, 0, 0.03)
    bad = dict(g)
    bad["adjncy"] = g["adjncy"].clone()
    bad["adjncy"][0] = 1000
    with pytest.raises(gp.GPError):
        gp.lp_cluster(bad, 5)
    with pytest.raises(gp.GPError):
        gp.lp_refine(g, torch.full((100,), 3, dtype=torch.int32, device="cuda"), 2, 60)


def test_repeat_runs_identical(dev_cases):
    a, _ = gp.partition(dev_cases["rmat16"], 16, 0.03)
    b, _ = gp.partition(dev_cases["rmat16"], 16, 0.03)
    assert torch.equal(a, b)


def test_cached_memory_reuse_and_release():
    # successive calls reuse the library's cached device memory; releasing it
    # in between changes nothing
    g1, g2 = graphgen.rmat(12, 8), graphgen.rgg2d(3000, 9)
    d1, d2 = gp.to_device(g1), gp.to_device(g2)
    p1, r1 = gp.partition(d1, 8)
    p2, r2 = gp.partition(d2, 4)
    gp.release_cache()
    q1, s1 = gp.partition(d1, 8)
    q2, s2 = gp.partition(d2, 4)
    assert torch.equal(p1, q1) and torch.equal(p2, q2)
    assert r1["cut"] == s1["cut"] and r2["cut"] == s2["cut"]
    op, _ = oracle.partition(g2, 4)
    assert np.array_equal(q2.cpu().numpy(), op)


@pytest.mark.parametrize("tuning", [
    {"tier_max": [16, 16, 16, 16], "dense_split": 16, "dense_chunk": 256},
    {"tier_max": [32, 128, 1024, 4096], "dense_split": 1024, "dense_chunk": 8192},
    {"tier_max": [64, 64, 2048, 2048], "dense_split": 100000, "dense_chunk": 65536},
])
def test_tuning_changes_no_result(tuning):
    # execution thresholds move vertices between kernels; labels must not change
    gs = [(graphgen.rmat(13, 4), 16), (graphgen.grid3d(14, 12, 10, seed=4, wmax=9), 4),
          (graphgen.rmat_m(12, 60000, 9), 300)]
    try:
        gp.set_tuning(tuning)
        assert gp.get_tuning() == tuning
        for g, k in gs:
            p, r = gp.partition(gp.to_device(g), k)
            op, ores = oracle.partition(g, k)
            assert np.array_equal(p.cpu().numpy(), op)
            assert r["cut"] == ores["cut"]
        g = graphgen.rmat(14, 5)
        lab, _ = gp.lp_cluster(gp.to_device(g), 500, 10)
        olab, _ = oracle.lp_cluster(g, 500, 10)
        assert np.array_equal(lab.cpu().numpy(), olab)
    finally:
        gp.set_tuning(None)


def test_tuning_rejects_values_beyond_table_capacity():
    with pytest.raises(gp.GPError):
        gp.set_tuning({"tier_max": [128, 256, 2048, 8192], "dense_split": 256, "dense_chunk": 2048})
    with pytest.raises(gp.GPError):
        gp.set_tuning({"tier_max": [64, 32, 2048, 8192], "dense_split": 256, "dense_chunk": 2048})
    with pytest.raises(gp.GPError):
        gp.set_tuning({"tier_max": [64, 256, 2048, 8192], "dense_split": 256, "dense_chunk": 1000})
    assert gp.get_tuning()["tier_max"] == [64, 256, 2048, 8192]


def _heavy(g, scale, seed):
    """Same graph with edge weights large enough that sums need 64 bits."""
    rng = np.random.default_rng(seed)
    h = dict(g)
    n = len(g["xadj"]) - 1
    rows = np.repeat(np.arange(n), np.diff(g["xadj"]))
    lo, hi = np.minimum(rows, g["adjncy"]), np.maximum(rows, g["adjncy"])
    # symmetric weights from the undirected edge's ends
    w = (((lo.astype(np.int64) * 1000003 + hi) * 2654435761) % scale) + scale // 2
    h["adjwgt"] = w.astype(np.int32)
    assert int(h["adjwgt"].astype(np.int64).sum()) >= 2 ** 31
    return h


@pytest.mark.parametrize("case", ["rmat13", "star", "grid"])
def test_lp_with_64bit_sums(case):
    if case == "rmat13":
        g = _heavy(graphgen.rmat(13, 3), 1 << 22, 1)
    elif case == "star":
        g = _heavy(_star(20000, extra=[(1, 2), (3, 4)]), 1 << 20, 2)
    else:
        g = _heavy(graphgen.grid3d(16, 15, 14, seed=1, wmax=0), 1 << 24, 3)
    dg = gp.to_device(g)
    for U in (5, 400):
        lab, st = gp.lp_cluster(dg, U, 10)
        olab, ost = oracle.lp_cluster(g, U, 10)
        assert np.array_equal(_np(lab), olab), U
        assert st["moves"] == ost["moves"]
    n = len(g["xadj"]) - 1
    for k in (16, 300):
        part = (np.arange(n) * 7919 % k).astype(np.int32)
        lm = oracle.lmax(n, k, 0.03)
        p, _ = gp.lp_refine(dg, torch.from_numpy(part).cuda(), k, lm, 10)
        op, _ = oracle.lp_refine(g, part, k, lm, 10)
        assert np.array_equal(_np(p), op), k


def test_lp_with_64bit_sums_small_block_tier():
    # a block-tier bound of 1024 selects the 128-thread workgroups with
    # 2048-slot tables, here with 64-bit connection sums
    g = _heavy(graphgen.rmat(13, 3), 1 << 22, 1)
    deg = np.diff(g["xadj"])
    assert np.count_nonzero((deg > 128) & (deg <= 1024)) > 10
    try:
        gp.set_tuning({"tier_max": [32, 128, 1024, 4096], "dense_split": 256, "dense_chunk": 2048})
        for U in (5, 400):
            lab, st = gp.lp_cluster(gp.to_device(g), U, 10)
            olab, ost = oracle.lp_cluster(g, U, 10)
            assert np.array_equal(_np(lab), olab), U
            assert st["moves"] == ost["moves"]
    finally:
        gp.set_tuning(None)


def _fmix32(x):
    # MurmurHash3's 32-bit finaliser, the hub path's bucket hash
    x = x.astype(np.uint64)
    m = np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x85EBCA6B)) & m
    x ^= x >> np.uint64(13)
    x = (x * np.uint64(0xC2B2AE35)) & m
    x ^= x >> np.uint64(16)
    return x


def _colliding_hub(d, n, seed):
    # hub = vertex n - 1 (the largest label, so the direction rule lets it see
    # all its neighbours in even rounds) with d neighbours whose labels (their
    # ids in round 0) all fall into bucket 0 of the hub's ceil(d / 2048)
    # buckets: more pairs than a bucket region holds (4096), so the overflow
    # table is used. A second hub, vertex n - 2, has ordinary neighbours.
    nb = -(-d // 2048)
    ids = np.arange(n - 2, dtype=np.int64)
    b = (_fmix32(ids) * np.uint64(nb)) >> np.uint64(32)
    nbr = ids[b == 0][:d]
    assert len(nbr) == d
    rng = np.random.default_rng(seed)
    other = rng.choice(n - 2, 12000, replace=False)
    extra = rng.integers(0, n - 2, size=(3 * n, 2))
    edges = [(n - 1, int(u)) for u in nbr] + [(n - 2, int(u)) for u in other]
    edges += [(int(u), int(v)) for u, v in extra if u != v]
    return graphgen.from_edges(n, edges)


@pytest.mark.parametrize("dirs", [0, 1])
def test_hub_bucket_overflow(dirs):
    g = _colliding_hub(9000, 60000, 5)
    deg = np.diff(g["xadj"])
    assert deg[-1] >= 9000 and deg[-2] > 8192  # both in the hub tier
    dg = gp.to_device(g)
    for U in (3, 50, 5000):
        lab, st = gp.lp_cluster(dg, U, 6, dirs)
        olab, ost = oracle.lp_cluster(g, U, 6, dirs)
        assert np.array_equal(_np(lab), olab), U
        assert {k: st[k] for k in ost} == ost
    # the same hubs with many labels in refinement (hashed tables, no overflow)
    n = len(deg)
    part = (np.arange(n) * 7919 % 300).astype(np.int32)
    lm = oracle.lmax(n, 300, 0.03)
    p, st = gp.lp_refine(dg, torch.from_numpy(part).cuda(), 300, lm, 6, dirs)
    op, ost = oracle.lp_refine(g, part, 300, lm, 6, dirs)
    assert np.array_equal(_np(p), op) and {k: st[k] for k in ost} == ost


def test_packed_tables_at_every_block_tier_size():
    # degrees 2049-4096 take 512-thread workgroups with 8192-slot packed tables,
    # 4097-8192 1024-thread ones with 16384 slots (bound 8192) or the hub path
    # (bound 4096); R-MAT-17 has vertices in both degree ranges
    g = graphgen.rmat(17, 11)
    deg = np.diff(g["xadj"])
    assert np.count_nonzero((deg > 2048) & (deg <= 4096)) > 5 and np.count_nonzero((deg > 4096) & (deg <= 8192)) > 0
    dg = gp.to_device(g)
    olab, ost = oracle.lp_cluster(g, 300, 10)
    opart, ores = oracle.partition(g, 16)
    try:
        for t3 in (4096, 8192):
            gp.set_tuning({"tier_max": [64, 256, 2048, t3], "dense_split": 256, "dense_chunk": 2048})
            lab, st = gp.lp_cluster(dg, 300, 10)
            assert np.array_equal(_np(lab), olab) and st["moves"] == ost["moves"], t3
            p, r = gp.partition(dg, 16)
            assert np.array_equal(_np(p), opart) and r["cut"] == ores["cut"], t3
    finally:
        gp.set_tuning(None)
