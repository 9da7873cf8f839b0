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
    # graphs carry their own k; rmat22 is the default workload
    for name, w in bench.WORKLOADS.items():
        assert (w["k"] is None) if w["kind"] == "batch" else (w["k"] >= 2), name
    assert "rmat22" in bench.WORKLOADS
