"""What the trained network gains, on the evaluation workload: R-MAT scale 24
(seed 24), k = 16, eps = 0.03, partition seeds 0..9 (the bisection start hash
and the probe seed), with the committed k = 16 weights.

The judge guarantees the learned mode never ends the coarsest level with a
larger cut or an imbalance. The evaluation coarsest graph (54,681 vertices)
lies far outside the training pairs (at most 3,252 vertices); over the ten
seeds the proposal is kept several times and the geometric mean of the final
cuts is below the plain one. Seed 0's outcome is also pinned by the oracle's
golden (tests/golden/partition_goldens.json, learned24).
"""
import math
import os

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_learned_init_gain_rmat24_k16():
    g = gp.to_device(graphgen.rmat(24, 24))
    w = torch.from_numpy(np.load(os.path.join(ROOT, "paper_1710_08231_amd", "mpnn_k16.npy"))).cuda()
    ratios, kept = [], []
    for seed in range(10):
        _, r0 = gp.partition(g, 16, 0.03, seed=seed)
        _, r1 = gp.partition(g, 16, 0.03, seed=seed, init_mode=1, mpnn_params=w, mpnn_seed=seed)
        assert r1["learned_tried"] == 1 and r0["balanced"] and r1["balanced"]
        # the judge: a kept proposal never cuts more at the coarsest level
        if r1["learned_kept"]:
            assert r1["learned_cut_coarsest"] <= r1["plain_cut_coarsest"]
        else:
            assert r1["cut"] == r0["cut"]
        # coarsening is the same in both modes
        assert r1["coarsest_n"] == r0["coarsest_n"] and r1["levels"] == r0["levels"]
        kept.append(r1["learned_kept"])
        ratios.append(r1["cut"] / r0["cut"])
    assert kept[0] == 1 and sum(kept) >= 3
    geo = math.exp(sum(math.log(x) for x in ratios) / len(ratios))
    print(f"learned/plain final cut, seeds 0..9: {[round(x, 4) for x in ratios]}; kept {kept}; geomean {geo:.4f}")
    assert geo < 1.0
