"""Pins of the learned initial partition's oracle (CPU only).

The binary32 inference (oracle/mpnn.c) is checked against the independent
binary64 matrix form (oracle/mpnn.py); the binary64 gradient is checked by
central finite differences; bfloat16 rounding against torch's conversion; the
probe stream against splitmix64's published test vectors; the judge by forced
rejection and forced acceptance.
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import mpnn


def test_param_count():
    # 3 layers (18->64, 64->64, 64->64, self and neighbour matrices plus bias) and a 64->k head
    assert oracle.mpnn_param_count(16) == 19920 == mpnn.param_count(16)
    for k in (1, 2, 8, 64):
        assert oracle.mpnn_param_count(k) == 2 * 64 * 18 + 64 + 2 * (2 * 64 * 64 + 64) + 65 * k


def test_splitmix_published_vectors():
    # splitmix64 started from state 0: the first outputs are the published reference values
    gamma = 0x9E3779B97F4A7C15
    assert mpnn._splitmix(0) == 0xE220A8397B1DCDAF
    assert mpnn._splitmix(gamma) == 0x6E789E6AA1B965F4
    assert mpnn._splitmix((2 * gamma) & ((1 << 64) - 1)) == 0x06C45D188009454F


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 3000), rng.normal(0, 1e-30, 200), rng.normal(0, 1e30, 200)])
    x = x.astype(np.float32)
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -126 * (1 + 2.0 ** -8)],
                    dtype=np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.finfo(np.float32).max, 1e-45], dtype=np.float32)
    x = np.concatenate([x, ties, special])
    ours = oracle.bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
    # ties go to the even neighbour
    assert oracle.bf16(np.float32(1.0 + 2.0 ** -8)) == np.float32(1.0)
    assert oracle.bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)
    assert math.isnan(float(oracle.bf16(np.float32(np.nan))))


def test_probes_on_edgeless_graph():
    # without edges the walk keeps every probe: the features are the raw +-1 stream
    g = graphgen.from_edges(40, [])
    X = oracle.mpnn_features(g, seed=123)
    assert np.array_equal(X[:, 2:], mpnn.probes(40, 123).astype(np.float32))
    assert np.all(X[:, 0] == 1.0) and np.all(X[:, 1] == 0.0)
    # both signs appear in every probe column of a larger graph
    Y = mpnn.probes(300, 5)
    assert np.all(np.abs(Y.sum(axis=0)) < 300)


@pytest.mark.parametrize("case", ["rgg", "weighted", "rmat"])
def test_features_match_binary64(case):
    if case == "rgg":
        g = graphgen.rgg2d(1500, 4)
    elif case == "weighted":
        g = graphgen.random_small(60, 0.1, 9, wmax=50, vmax=7)
    else:
        g = graphgen.rmat(10, 2)
    X = oracle.mpnn_features(g, seed=77)
    R = mpnn.features(g, 77)
    # ratio features are one binary64 division rounded once: bit-equal to numpy's
    assert np.array_equal(X[:, :2], R[:, :2].astype(np.float32))
    assert np.abs(X[:, 2:] - R[:, 2:]).max() < 2e-6


def test_walk_preserves_weighted_mean_direction():
    # the lazy walk's stationary direction: sum_v d(v) y(v) is invariant under
    # y <- (y + D^-1 A y)/2 for symmetric A (d = weighted degree)
    g = graphgen.grid3d(6, 5, 4, seed=1, wmax=9)
    X = mpnn.features(g, 3)
    Y0 = mpnn.probes(len(g["xadj"]) - 1, 3)
    A = mpnn.adjacency(g)
    d = np.asarray(A.sum(axis=1)).ravel()
    assert np.allclose(d @ X[:, 2:], d @ Y0, rtol=0, atol=1e-9)


@pytest.mark.parametrize("k", [2, 8, 16])
def test_inference_matches_binary64(k):
    g = graphgen.rgg2d(1200, 8)
    rng = np.random.default_rng(k)
    w = rng.normal(0, 0.25, mpnn.param_count(k)).astype(np.float32)
    Z, P = oracle.mpnn_infer(g, k, w, seed=4)
    c = mpnn.forward(g, k, oracle.bf16(w).astype(np.float64), seed=4)
    scale = np.abs(c["Z"]).max()
    assert np.abs(Z - c["Z"]).max() <= 1e-5 * max(scale, 1.0)
    # where the binary64 margin is clear, the argmax agrees
    srt = np.sort(c["Z"], axis=1)
    clear = srt[:, -1] - srt[:, -2] > 1e-3 if k > 1 else np.ones(len(P), bool)
    assert np.array_equal(P[clear], c["Z"].argmax(axis=1)[clear])


def test_inference_uses_bf16_weights():
    g = graphgen.rgg2d(300, 1)
    rng = np.random.default_rng(3)
    w = rng.normal(0, 0.25, mpnn.param_count(4)).astype(np.float32)
    Z1, _ = oracle.mpnn_infer(g, 4, w)
    Z2, _ = oracle.mpnn_infer(g, 4, oracle.bf16(w))
    assert np.array_equal(Z1, Z2)


def test_argmax_ties_to_lowest():
    g = graphgen.rgg2d(200, 2)
    k = 5
    w = np.zeros(mpnn.param_count(k), np.float32)
    w[-k:] = [0.5, 2.0, 2.0, -1.0, 2.0]  # head bias only
    Z, P = oracle.mpnn_infer(g, k, w)
    assert np.all(P == 1)


@pytest.mark.parametrize("case", ["weighted", "isolated"])
def test_gradient_finite_differences(case):
    if case == "weighted":
        g = graphgen.random_small(24, 0.2, 3, wmax=5, vmax=4)
    else:
        g = graphgen.from_edges(9, [(0, 1), (1, 2), (2, 0), (3, 4), (5, 6), (6, 7), (4, 6)], weights=[1, 2, 3, 1, 4, 1, 2])
    n = len(g["xadj"]) - 1
    k = 4
    rng = np.random.default_rng(1)
    w = rng.normal(0, 0.3, mpnn.param_count(k))
    t = rng.integers(0, k, n)
    _, _, gr = mpnn.loss_and_grad(g, k, w, t, seed=7, lam=0.5)
    idx = np.concatenate([rng.choice(w.size - 64 * k - k, 60, replace=False), np.arange(w.size - 64 * k - k, w.size)])
    h = 1e-5
    fd = np.empty(len(idx))
    for j, i in enumerate(idx):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[j] = (mpnn.loss(g, k, wp, t, 7, 0.5) - mpnn.loss(g, k, wm, t, 7, 0.5)) / (2 * h)
    assert np.linalg.norm(fd - gr[idx]) <= 1e-6 * np.linalg.norm(fd)


def test_loss_limits():
    # uniform softmax: p = 1/k on every edge, Q = 1/k -> balance term 0, edge loss closed form
    g = graphgen.rgg2d(400, 6)
    k = 4
    w = np.zeros(mpnn.param_count(k))
    t = np.zeros(400, np.int64)  # every edge inside one block: y = 1
    e, b, _ = mpnn.loss_and_grad(g, k, w, t)
    assert b == pytest.approx(0.0, abs=1e-15)
    assert e == pytest.approx(-math.log(1.0 / k), rel=1e-12)
    # all mass in class 0: Q = e_0 -> balance term k * ((1 - 1/k)^2 + (k-1)/k^2) = k - 1
    w[-k:] = [60.0, 0, 0, 0]
    _, b, _ = mpnn.loss_and_grad(g, k, w, t)
    assert b == pytest.approx(k - 1.0, rel=1e-9)


def _rgg_for_judge():
    return graphgen.rgg2d(4000, 21)


def test_judge_forced_rejection_nan_weights():
    g = _rgg_for_judge()
    P0, r0 = oracle.partition(g, 4)
    w = np.full(mpnn.param_count(4), np.nan, np.float32)
    P1, r1 = oracle.partition(g, 4, init_mode=1, mpnn_params=w)
    assert r1["learned_tried"] == 1 and r1["learned_kept"] == 0 and r1["learned_cut_coarsest"] == -1
    assert np.array_equal(P0, P1) and r0["cut"] == r1["cut"]


def test_judge_forced_acceptance_k1():
    # one block: the proposal equals the plain partition, a tie keeps the proposal
    g = _rgg_for_judge()
    w = np.random.default_rng(0).normal(0, 0.2, mpnn.param_count(1)).astype(np.float32)
    P0, r0 = oracle.partition(g, 1)
    P1, r1 = oracle.partition(g, 1, init_mode=1, mpnn_params=w)
    assert r1["learned_tried"] == 1 and r1["learned_kept"] == 1
    assert r1["learned_cut_coarsest"] == r1["plain_cut_coarsest"] == 0
    assert np.array_equal(P0, P1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_judge_rule(seed):
    g = graphgen.rgg2d(3000, 30 + seed)
    k = 8
    w = np.random.default_rng(seed).normal(0, 0.3, mpnn.param_count(k)).astype(np.float32)
    P0, r0 = oracle.partition(g, k)
    P1, r1 = oracle.partition(g, k, init_mode=1, mpnn_params=w, mpnn_seed=seed)
    assert r1["learned_tried"] == 1
    assert r1["plain_cut_coarsest"] >= 0
    if r1["learned_kept"]:
        assert r1["learned_cut_coarsest"] <= r1["plain_cut_coarsest"]
    else:
        assert np.array_equal(P0, P1)
    assert r1["balanced"] == 1
    # coarsening is untouched by the learned mode
    for key in ("levels", "coarsest_n", "edge_visits_cluster", "lmax", "ucl"):
        assert r0[key] == r1[key]


def test_size_limit_skips_learned():
    g = _rgg_for_judge()
    w = np.zeros(mpnn.param_count(4), np.float32)
    P0, r0 = oracle.partition(g, 4)
    P1, r1 = oracle.partition(g, 4, init_mode=1, mpnn_params=w, mpnn_max_n=r0["coarsest_n"] - 1)
    assert r1["learned_tried"] == 0 and np.array_equal(P0, P1)


def test_coarsest_graph_and_partition():
    g = graphgen.rmat(12, 5)
    k = 8
    cg, pc = oracle.coarsest(g, k)
    P, r = oracle.partition(g, k)
    nc = len(cg["xadj"]) - 1
    assert nc == r["coarsest_n"]
    deg = np.diff(g["xadj"])
    # vertex weight is conserved (vertices without neighbours are set aside)
    assert cg["vwgt"].sum() == np.count_nonzero(deg)
    rows = np.repeat(np.arange(nc), np.diff(cg["xadj"]))
    assert np.all(rows != cg["adjncy"])  # no self-loops
    B = oracle.block_weights(cg, pc, k)
    assert B.max() <= r["lmax"]
    # same plain cut as the learned mode reports for the coarsest level
    w = np.full(mpnn.param_count(k), np.nan, np.float32)
    _, r1 = oracle.partition(g, k, init_mode=1, mpnn_params=w)
    assert oracle.cut(cg, pc) == r1["plain_cut_coarsest"]


def test_decode_worked_examples():
    # hand-derived: five unit vertices, k=2, L_max=3; four prefer block 0.
    # round 0 admits v0, v1, v2 to block 0 (v3 would make it 4) and v4 to block 1;
    # round 1 offers v3 its second choice, block 1 (weight 2 <= 3).
    g = graphgen.from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    Z = np.array([[1, 0], [1, 0], [1, 0], [1, 0], [0, 1]], np.float32)
    assert oracle.mpnn_decode(g, 2, Z, 3).tolist() == [0, 0, 0, 1, 1]
    # equal logits rank the lower block first
    assert oracle.mpnn_decode(g, 2, np.zeros((5, 2), np.float32), 3).tolist() == [0, 0, 0, 1, 1]
    # weights 3,3,3, L_max=4: v0 -> 0; v1 -> 1 in round 1; v2 fits nowhere and
    # goes to the lighter block, a tie between 3 and 3 -> block 0
    g3 = graphgen.from_edges(3, [(0, 1), (1, 2)], vwgt=[3, 3, 3])
    assert oracle.mpnn_decode(g3, 2, np.array([[1, 0]] * 3, np.float32), 4).tolist() == [0, 1, 0]
    # an early heavy offer that is rejected still counts against the later ones:
    # weights 1,5,1, L_max=5, all prefer block 0. Round 0: v0 in (1), v1 out (6),
    # v2 out (7 > 5 although 1+1 would fit). Round 1: v1 -> block 1 (5), v2 out
    # (6). Leftover v2 -> lighter block 0 (1 < 5).
    g4 = graphgen.from_edges(3, [(0, 1), (1, 2)], vwgt=[1, 5, 1])
    assert oracle.mpnn_decode(g4, 2, np.array([[1, 0]] * 3, np.float32), 5).tolist() == [0, 1, 0]


def test_decode_reduces_to_argmax_within_capacity():
    g = graphgen.rgg2d(800, 3)
    rng = np.random.default_rng(0)
    Z = rng.normal(0, 1, (800, 8)).astype(np.float32)
    # a bound no block can reach: decoding is the argmax (ties -> lowest)
    assert np.array_equal(oracle.mpnn_decode(g, 8, Z, 10 ** 9), Z.argmax(axis=1))


@pytest.mark.parametrize("k", [2, 7, 16])
def test_decode_unit_weights_always_balanced(k):
    # unit weights and k * L_max >= n: every vertex is placed within k rounds,
    # no block exceeds L_max, and a vertex only sits outside its first choice
    # when that block is full
    g = graphgen.rgg2d(1500, k)
    rng = np.random.default_rng(k)
    Z = np.round(rng.normal(0, 1, (1500, k)), 1).astype(np.float32)  # many ties
    lm = oracle.lmax(1500, k, 0.03)
    P = oracle.mpnn_decode(g, k, Z, lm)
    B = np.bincount(P, minlength=k)
    assert B.max() <= lm and B.sum() == 1500
    first = np.array([min(range(k), key=lambda c: (-z[c], c)) for z in Z])
    assert np.all(B[first[P != first]] == lm)
