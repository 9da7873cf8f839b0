"""Full-size parity: the GPU multilevel partition against the oracle's, on the
benchmark workloads (§III scheme; single graphs and the batched form).

The expected values are in tests/golden/partition_goldens.json, written by
tests/golden/make_partition_goldens.py, which calls only the oracle and the
input generators. For each workload the GPU partition array must hash to the
oracle's SHA-256 (bit-identical labels, original vertex ids) and every scalar
of the result must be equal: cut, largest block, L_max, U_c, balance flag,
levels, coarsest size, isolated count, clustering and refinement edge visits,
and for the learned initial partition the judge's coarsest-level cuts and
decision. The partitions run with the tuned execution thresholds of the
workload when a tuning file exists (thresholds never change a result).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "partition_goldens.json")
FIELDS = ("cut", "max_block_w", "lmax", "ucl", "balanced", "levels", "coarsest_n", "n_isolated",
          "edge_visits_cluster", "edge_visits_refine", "learned_tried", "learned_kept",
          "plain_cut_coarsest", "learned_cut_coarsest")
TUNING_OF = {"rmat22": "rmat22", "grid256": "grid256", "rmat24": "rmat24", "rmat24_k16": "rmat24",
             "learned24": "rmat24", "batch512": "batch512"}


def _goldens():
    with open(GOLDEN) as f:
        return json.load(f)


def _sha(part_np):
    return hashlib.sha256(np.ascontiguousarray(part_np, dtype="<i4").tobytes()).hexdigest()


def _graph(spec):
    if spec["kind"] == "rgg":
        return graphgen.rgg2d(spec["n"], spec["seed"])
    if spec["kind"] == "rmat":
        return graphgen.rmat(spec["scale"], spec["seed"])
    if spec["kind"] == "grid":
        s = spec["side"]
        return graphgen.grid3d(s, s, s, seed=spec["seed"], wmax=spec["wmax"])
    raise ValueError(spec["kind"])


_CACHE = {}


def _device_graph(spec):
    """One resident copy per input (the rmat24 workloads share a graph)."""
    import paper_1710_08231_amd as gp
    key = json.dumps(spec, sort_keys=True)
    if key not in _CACHE:
        _CACHE.clear()
        g = _graph(spec)
        _CACHE[key] = (g, gp.to_device(g))
    return _CACHE[key]


def _with_tuning(name):
    import paper_1710_08231_amd as gp
    path = os.path.join(ROOT, "paper_1710_08231_amd", "tuning", f"{TUNING_OF.get(name, name)}.json")
    if os.path.exists(path):
        with open(path) as f:
            gp.set_tuning(json.load(f)["tuning"])
    else:
        gp.set_tuning(None)


SINGLE = [w for w, e in sorted(_goldens().items()) if e["graph"]["kind"] != "batch"]


@pytest.mark.gpu
@pytest.mark.parametrize("name", SINGLE)
def test_partition_matches_oracle_golden(name):
    import torch
    import paper_1710_08231_amd as gp
    e = _goldens()[name]
    g, dg = _device_graph(e["graph"])
    assert (len(g["xadj"]) - 1, len(g["adjncy"])) == (e["n"], e["nnz"])
    params = dict(e["params"])
    keep = None
    if "weights" in e:
        path = os.path.join(ROOT, e["weights"])
        with open(path, "rb") as f:
            assert hashlib.sha256(f.read()).hexdigest() == e["weights_sha256"], "weights changed since the golden"
        keep = torch.from_numpy(np.load(path).astype(np.float32)).cuda()
        params["mpnn_params"] = keep
    _with_tuning(name)
    try:
        part, res = gp.partition(dg, e["k"], e["eps"], **params)
    finally:
        gp.set_tuning(None)
    got = {f: int(res[f]) for f in FIELDS}
    want = {f: e[f] for f in FIELDS}
    assert got == want
    assert res["code"] == e["code"]
    assert _sha(part.cpu().numpy()) == e["sha256"]


@pytest.mark.gpu
def test_batch512_matches_oracle_goldens():
    import paper_1710_08231_amd as gp
    e = _goldens()["batch512"]
    graphs, ks = graphgen.batch(master_seed=e["graph"]["master_seed"], count=e["graph"]["count"])
    assert [x["k"] for x in e["graphs"]] == list(ks)
    u, off = gp.union_graph(graphs)
    du = gp.to_device(u)
    _with_tuning("batch512")
    try:
        part, res, code = gp.partition_batch(du, off, ks, e["eps"])
    finally:
        gp.set_tuning(None)
    part = part.cpu().numpy()
    bad = []
    for q, want in enumerate(e["graphs"]):
        got = {f: int(res[q][f]) for f in FIELDS}
        if got != {f: want[f] for f in FIELDS} or _sha(part[off[q]:off[q + 1]]) != want["sha256"]:
            bad.append(q)
    assert not bad, f"graphs differing from the oracle: {bad[:20]} ({len(bad)} of {len(ks)})"
    assert code == (1 if any(x["code"] == 1 for x in e["graphs"]) else 0)
