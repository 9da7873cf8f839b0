"""The stored full-size goldens are the oracle's: re-derive the cheap ones.

tests/golden/partition_goldens.json is written by make_partition_goldens.py
from the oracle alone. Here the small workload (2-D rgg, n = 16384, k = 2) and
the smallest graphs of the 512-graph batch are recomputed with the oracle as it
stands and must match the file, so a change to the oracle's arithmetic that
would invalidate the goldens fails on the CPU."""
import hashlib
import json
import os

import numpy as np

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "partition_goldens.json")
FIELDS = ("cut", "max_block_w", "lmax", "ucl", "balanced", "levels", "coarsest_n", "n_isolated",
          "edge_visits_cluster", "edge_visits_refine", "code")


def _sha(p):
    return hashlib.sha256(np.ascontiguousarray(p, dtype="<i4").tobytes()).hexdigest()


def _goldens():
    with open(GOLDEN) as f:
        return json.load(f)


def test_goldens_cover_every_workload():
    d = _goldens()
    assert {"rgg16k", "rmat22", "grid256", "rmat24", "rmat24_k16", "learned24", "batch512"} <= set(d)
    assert len(d["batch512"]["graphs"]) == 512
    # the plain runs are balanced; R-MAT-24 has 7,905,142 vertices without neighbours
    assert all(d[w]["balanced"] == 1 for w in ("rgg16k", "rmat22", "grid256", "rmat24", "rmat24_k16"))
    assert d["rmat24"]["n_isolated"] == 7_905_142 and d["rmat24"]["nnz"] == 520_761_028


def test_rgg16k_golden_is_the_oracle():
    e = _goldens()["rgg16k"]
    g = graphgen.rgg2d(e["graph"]["n"], e["graph"]["seed"])
    part, res = oracle.partition(g, e["k"], e["eps"])
    assert {f: res[f] for f in FIELDS} == {f: e[f] for f in FIELDS}
    assert _sha(part) == e["sha256"]


def test_smallest_batch_goldens_are_the_oracle():
    e = _goldens()["batch512"]
    graphs, ks = graphgen.batch(master_seed=e["graph"]["master_seed"], count=e["graph"]["count"])
    order = np.argsort([len(g["adjncy"]) for g in graphs], kind="stable")[:6]
    for q in order.tolist():
        part, res = oracle.partition(graphs[q], ks[q], e["eps"])
        want = e["graphs"][q]
        assert {f: res[f] for f in FIELDS} == {f: want[f] for f in FIELDS}
        assert _sha(part) == want["sha256"]
