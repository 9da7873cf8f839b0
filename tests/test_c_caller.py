"""The C ABI used from plain C (tests/c_caller.c): no Python binding, no torch.

Without a GPU the program is only compiled against include/gp.h with a C
compiler and linked against libgp.so, which checks that the header is plain C
and self-contained. On a GPU it runs as a child process on graphs written by
the seeded generators:
  * partition mode: the whole multilevel scheme (§III), once on the library's
    scratch and once on a caller workspace of the reported size, must equal the
    oracle's partition;
  * steps mode: one level by hand on one caller workspace sized by
    gp_workspace_bytes (clustering §III-A, contraction, coarse refinement
    §III-C, projection, fine refinement, cut and block weights §II-A), each
    result equal to the oracle's step on the same input."""
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
    run = subprocess.run([exe, "partition", gfile, str(k), pfile], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    part = np.fromfile(pfile, dtype=np.int32)
    opart, ores = oracle.partition(g, k, 0.03)
    assert np.array_equal(part, opart)
    fields = dict(kv.split("=") for kv in run.stdout.split()[1:])
    assert int(fields["cut"]) == ores["cut"] and int(fields["max_block_w"]) == ores["max_block_w"]
    assert int(fields["levels"]) == ores["levels"]


def _ints(path):
    return np.fromfile(path, dtype=np.int32)


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,k,U", [
    ("rgg30k", lambda: graphgen.rgg2d(30000, 4), 8, 40),
    ("rmat15", lambda: graphgen.rmat(15, 3), 16, 300),
    ("rmat14_k300", lambda: graphgen.rmat(14, 9), 300, 20),
])
def test_c_caller_steps_equal_oracle(tmp_path, name, make, k, U):
    exe = _compile(tmp_path)
    g = make()
    n = len(g["xadj"]) - 1
    gfile = os.path.join(str(tmp_path), "g.bin")
    _write_graph(gfile, g)
    run = subprocess.run([exe, "steps", gfile, str(k), str(U), str(tmp_path)], capture_output=True, text=True,
                         timeout=120)
    assert run.returncode == 0, run.stderr
    fields = dict(kv.split("=") for kv in run.stdout.split()[1:])

    labels = _ints(os.path.join(str(tmp_path), "labels.bin"))
    olab, ost = oracle.lp_cluster(g, U, 10, 1)
    assert np.array_equal(labels, olab) and int(fields["moves_c"]) == ost["moves"]

    coarse = _ints(os.path.join(str(tmp_path), "coarse.bin"))
    n_c, nnz_c = int(coarse[0]), int(coarse[1])
    parts = np.split(coarse[2:], np.cumsum([n_c + 1, nnz_c, nnz_c]))
    ocg, of2c = oracle.contract(g, olab)
    for got, key in zip(parts, ("xadj", "adjncy", "adjwgt", "vwgt")):
        assert np.array_equal(got, ocg[key]), key
    assert np.array_equal(_ints(os.path.join(str(tmp_path), "f2c.bin")), of2c)

    lm = oracle.lmax(n, k, 0.03)
    opc, osc = oracle.lp_refine(ocg, np.arange(n_c, dtype=np.int32) % k, k, lm, 25, 1)
    assert np.array_equal(_ints(os.path.join(str(tmp_path), "partc.bin")), opc)
    assert int(fields["moves_rc"]) == osc["moves"]

    opf, osf = oracle.lp_refine(g, oracle.project(of2c, opc), k, lm, 25, 1)
    assert np.array_equal(_ints(os.path.join(str(tmp_path), "partf.bin")), opf)
    assert int(fields["moves_rf"]) == osf["moves"]
    assert int(fields["cut"]) == oracle.cut(g, opf)
    assert [int(b) for b in fields["B"].split(",")] == oracle.block_weights(g, opf, k).tolist()
