"""The C ABI used from plain C (tests/c_caller.c): no Python binding, no torch.

Without a GPU the program is only compiled against include/gp.h with a C
compiler and linked against libgp.so, which checks that the header is plain C
and self-contained. On a GPU it runs as a child process: it partitions graphs
written by the seeded generators, once on the library's scratch and once on a
caller workspace of the reported size, and its partition must equal the
oracle's (the multilevel scheme of §III)."""
import os
import subprocess

import numpy as np
import pytest

import graphgen
import oracle
import paper_1710_08231_amd as gp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(out_dir):
    if not os.path.exists(gp.LIB_PATH):
        gp.build()
    exe = os.path.join(str(out_dir), "c_caller")
    lib_dir = os.path.dirname(gp.LIB_PATH)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_caller.c"), "-o", exe,
           "-L", lib_dir, "-lgp", "-Wl,-rpath," + lib_dir,
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=120)
    return exe


def test_c_caller_compiles_and_links(tmp_path):
    try:
        exe = _compile(tmp_path)
    except subprocess.CalledProcessError as e:
        pytest.fail(e.stderr)
    assert os.path.exists(exe)


def _write_graph(path, g):
    n = len(g["xadj"]) - 1
    with open(path, "wb") as f:
        np.array([n, len(g["adjncy"])], np.int32).tofile(f)
        np.asarray(g["xadj"], np.int32).tofile(f)
        np.asarray(g["adjncy"], np.int32).tofile(f)


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,k", [
    ("rgg30k", lambda: graphgen.rgg2d(30000, 4), 8),
    ("rmat15", lambda: graphgen.rmat(15, 3), 16),
    ("grid", lambda: graphgen.grid3d(30, 20, 10, seed=2, wmax=0), 64),
])
def test_c_caller_partition_equals_oracle(tmp_path, name, make, k):
    exe = _compile(tmp_path)
    g = make()
    gfile, pfile = os.path.join(str(tmp_path), "g.bin"), os.path.join(str(tmp_path), "p.bin")
    _write_graph(gfile, g)
    run = subprocess.run([exe, gfile, str(k), pfile], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    part = np.fromfile(pfile, dtype=np.int32)
    opart, ores = oracle.partition(g, k, 0.03)
    assert np.array_equal(part, opart)
    fields = dict(kv.split("=") for kv in run.stdout.split()[1:])
    assert int(fields["cut"]) == ores["cut"] and int(fields["max_block_w"]) == ores["max_block_w"]
    assert int(fields["levels"]) == ores["levels"]
