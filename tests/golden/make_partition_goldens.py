"""Write the oracle's full multilevel partitions of the benchmark workloads to
``tests/golden/partition_goldens.json``.

Calls only ``graphgen`` (the seeded inputs) and ``oracle`` (the plain CPU
definition). For every workload the file records how to regenerate the input,
the partition parameters, and the oracle's result: the SHA-256 of the
partition array (int32, little-endian, original vertex ids), the cut, the
largest block weight, L_max, the balance flag, the number of levels, the
coarsest graph's size, the isolated count and the clustering / refinement edge
visits (§III scheme; the readings are those of the oracle's header). The
learned-init workload also records the judge's coarsest-level cuts and
whether the proposal was kept, and the SHA-256 of the weights it used.

Usage: python tests/golden/make_partition_goldens.py [workload ...]
(default: all). Workloads already in the file and not named are kept.
The proposal loop runs on all host cores (oracle.set_threads); results do not
depend on the thread count.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "partition_goldens.json")
WEIGHTS_K16 = "paper_1710_08231_amd/mpnn_k16.npy"

# input recipe, k and partition parameters of each workload (eps = 0.03 throughout)
WORKLOADS = {
    "rgg16k": {"graph": {"kind": "rgg", "n": 16384, "seed": 1}, "k": 2, "params": {}},
    "rmat22": {"graph": {"kind": "rmat", "scale": 22, "seed": 22}, "k": 16, "params": {}},
    "grid256": {"graph": {"kind": "grid", "side": 256, "seed": 3, "wmax": 10}, "k": 64, "params": {}},
    "rmat24": {"graph": {"kind": "rmat", "scale": 24, "seed": 24}, "k": 64, "params": {}},
    "rmat24_k16": {"graph": {"kind": "rmat", "scale": 24, "seed": 24}, "k": 16, "params": {}},
    "learned24": {"graph": {"kind": "rmat", "scale": 24, "seed": 24}, "k": 16,
                  "params": {"init_mode": 1, "seed": 0, "mpnn_seed": 0}, "weights": WEIGHTS_K16},
    "batch512": {"graph": {"kind": "batch", "master_seed": 4, "count": 512}, "k": None, "params": {}},
}
EPS = 0.03
FIELDS = ("cut", "max_block_w", "lmax", "ucl", "balanced", "levels", "coarsest_n", "n_isolated",
          "edge_visits_cluster", "edge_visits_refine", "learned_tried", "learned_kept",
          "plain_cut_coarsest", "learned_cut_coarsest", "code")


def make_graph(spec):
    kind = spec["kind"]
    if kind == "rgg":
        return graphgen.rgg2d(spec["n"], spec["seed"])
    if kind == "rmat":
        return graphgen.rmat(spec["scale"], spec["seed"])
    if kind == "grid":
        s = spec["side"]
        return graphgen.grid3d(s, s, s, seed=spec["seed"], wmax=spec["wmax"])
    raise ValueError(kind)


def part_sha256(part):
    return hashlib.sha256(np.ascontiguousarray(part, dtype="<i4").tobytes()).hexdigest()


def file_sha256(path):
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def run(name):
    w = WORKLOADS[name]
    entry = {"graph": w["graph"], "k": w["k"], "eps": EPS, "params": w["params"]}
    t0 = time.time()
    if w["graph"]["kind"] == "batch":
        graphs, ks = graphgen.batch(master_seed=w["graph"]["master_seed"], count=w["graph"]["count"])
        per = []
        for i, (g, k) in enumerate(zip(graphs, ks)):
            part, res = oracle.partition(g, k, EPS)
            per.append({"k": k, "n": len(g["xadj"]) - 1, "nnz": len(g["adjncy"]), "sha256": part_sha256(part),
                        **{f: int(res[f]) for f in FIELDS}})
        entry["graphs"] = per
    else:
        g = make_graph(w["graph"])
        params = dict(w["params"])
        if "weights" in w:
            params["mpnn_params"] = np.load(os.path.join(ROOT, w["weights"])).astype(np.float32)
            entry["weights"] = w["weights"]
            entry["weights_sha256"] = file_sha256(w["weights"])
        part, res = oracle.partition(g, w["k"], EPS, **params)
        entry.update({"n": len(g["xadj"]) - 1, "nnz": len(g["adjncy"]), "sha256": part_sha256(part),
                      **{f: int(res[f]) for f in FIELDS}})
    entry["oracle_seconds"] = round(time.time() - t0, 1)
    return entry


def main(names):
    oracle.set_threads(os.cpu_count() or 1)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names or list(WORKLOADS):
        print(f"[goldens] {name} ...", flush=True)
        data[name] = run(name)
        print(f"[goldens] {name}: {json.dumps({k: v for k, v in data[name].items() if k != 'graphs'})}",
              flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
