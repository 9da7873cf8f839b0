"""Autotuner of the LP execution thresholds (``gp_set_tuning``).

The thresholds decide which kernel serves a vertex (the degree bounds of the
hashed-table tiers) and how high-degree rows are split in refinement with
dense tables (split degree, chunk size). They never change a result, only
the time, so the tuner simply times whole partitions of the workload graph
(plain or batched form) for each candidate, by coordinate descent: first the
tier bounds with the dense settings at their defaults, then the dense
settings with the best bounds. Each candidate is timed `reps` times after one
warm-up call; the minimum device time (``ms_total``) counts.

    python -m paper_1710_08231_amd.autotune --workload rmat22 --out paper_1710_08231_amd/tuning/rmat22.json
"""
import argparse
import itertools
import json
import os
import sys

import paper_1710_08231_amd as gp

TIER_CANDIDATES = list(itertools.product((32, 64), (128, 256), (1024, 2048), (2048, 4096, 8192)))
DENSE_CANDIDATES = list(itertools.product((128, 256, 512, 1024), (1024, 2048, 4096, 8192)))
DEFAULT = {"tier_max": [64, 256, 2048, 8192], "dense_split": 256, "dense_chunk": 2048}


def _time(run, tuning, reps):
    gp.set_tuning(tuning)
    run()  # warm-up: the scratch cache and the code paths of this setting
    return min(run() for _ in range(reps))


def tune(run, reps=2, log=print):
    """run() -> device ms of one partition under the current tuning. Returns the
    chosen tuning and every measurement."""
    rows = []
    best = dict(DEFAULT)
    best_ms = _time(run, best, reps)
    rows.append({"tuning": dict(best), "ms": best_ms})
    log(f"[tune] default {best_ms:.2f} ms")
    for tm in TIER_CANDIDATES:
        cand = dict(best, tier_max=list(tm))
        if cand == best:
            continue
        ms = _time(run, cand, reps)
        rows.append({"tuning": cand, "ms": ms})
        if ms < best_ms:
            best, best_ms = cand, ms
    log(f"[tune] tiers {best['tier_max']} {best_ms:.2f} ms")
    for split, chunk in DENSE_CANDIDATES:
        cand = dict(best, dense_split=split, dense_chunk=chunk)
        if cand == best:
            continue
        ms = _time(run, cand, reps)
        rows.append({"tuning": cand, "ms": ms})
        if ms < best_ms:
            best, best_ms = cand, ms
    log(f"[tune] dense split {best['dense_split']} chunk {best['dense_chunk']} {best_ms:.2f} ms")
    gp.set_tuning(best)
    return best, best_ms, rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench  # the workload recipes
    w = bench.WORKLOADS[a.workload]
    g = bench.make_graph(w)
    if w["kind"] == "batch":
        du = gp.to_device(g["union"])

        def run():
            _, res, _ = gp.partition_batch(du, g["off"], g["ks"], 0.03)
            return res[0]["ms_total"]
    else:
        dg = gp.to_device(g)

        def run():
            return gp.partition(dg, w["k"], 0.03)[1]["ms_total"]

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    best, best_ms, rows = tune(run, a.reps, log)
    default_ms = rows[0]["ms"]
    out = {"workload": a.workload, "tuning": best, "ms": best_ms, "default_ms": default_ms, "candidates": rows}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"workload": a.workload, "tuning": best, "ms": best_ms, "default_ms": default_ms}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
