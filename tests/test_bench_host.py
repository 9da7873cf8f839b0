"""Host-side checks of the benchmark driver and the committed tuning files
(no GPU: the refusal of several GPUs happens before any device work, and
gp_set_tuning only validates and stores the thresholds)."""
import glob
import json
import os
import subprocess
import sys

import pytest

import paper_1710_08231_amd as gp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_bench_refuses_more_than_one_gpu(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_tuning_files_are_valid_and_round_trip():
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1710_08231_amd", "tuning", "*.json")))
    assert {os.path.basename(f)[:-5] for f in files} >= {"rmat22", "rmat24", "grid256", "batch512"}
    try:
        for f in files:
            rec = json.load(open(f))
            t = rec["tuning"]
            gp.set_tuning(t)
            assert gp.get_tuning() == t, f
            # the chosen candidate is the fastest one the tuner recorded
            assert rec["ms"] == min(c["ms"] for c in rec["candidates"]), f
    finally:
        gp.set_tuning(None)


def test_workload_table():
    # every workload partitions into k >= 2 blocks, except the batch, whose
    # graphs carry their own k
    for name, w in bench.WORKLOADS.items():
        assert (w["k"] is None) if w["kind"] == "batch" else (w["k"] >= 2), name
    assert "rmat22" in bench.WORKLOADS


def test_level_tables_group_by_phase_and_level():
    calls = [{"name": "cluster L0|lp_cluster", "launches": 1, "ms": 2.0, "bytes": 8e9},
             {"name": "cluster L1|lp_cluster", "launches": 1, "ms": 1.0, "bytes": 1e9},
             {"name": "refine L0|lp_refine", "launches": 1, "ms": 4.0, "bytes": 16e9},
             {"name": "contract L0|contract", "launches": 1, "ms": 1.0, "bytes": 2e9}]
    kern = [{"name": "cluster L0|k_a", "launches": 10, "ms": 1.5, "bytes": 6e9},
            {"name": "cluster L0|k_b", "launches": 10, "ms": 0.2, "bytes": 1e9},
            {"name": "refine L0|k_c", "launches": 25, "ms": 3.0, "bytes": 12e9},
            {"name": "init|k_d", "launches": 3, "ms": 0.1, "bytes": 1e6}]
    rows, fam = bench.level_tables(calls, kern)
    assert [(r["phase"], r["level"]) for r in rows] == [("cluster", 0), ("cluster", 1), ("contract", 0),
                                                        ("refine", 0)]
    # 8 GB in 2 ms = 4000 GB/s = half of the 8 TB/s peak
    assert rows[0]["lp_frac"] == 0.5 and rows[0]["top_kernel"] == "k_a"
    assert rows[0]["top_kernel_frac"] == 0.5 and "top_kernel" not in rows[1]
    assert fam["lp_cluster"]["ms"] == 3.0 and fam["lp_cluster"]["frac"] == round(9e9 / 3e-3 / 1e9 / 8000, 4)
    assert fam["lp_refine"]["frac"] == 0.5 and fam["contract"]["frac"] == 0.25


def test_default_workload_is_rmat24():
    assert bench.WORKLOADS["rmat24"] == dict(kind="rmat", scale=24, seed=24, k=64)
    import argparse  # noqa: F401
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'default="rmat24"' in src
