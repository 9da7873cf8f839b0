"""GPU parity at the block counts where the refinement kernels change form.

LP refinement (§III-C) keeps one connection sum per block: up to 16, 64 or 256
sums per table (the table width switches between k = 16 and 17 and between
k = 64 and 65), block ids fit a byte mirror of the labels up to k = 256, and
from k = 257 on the refinement uses the hashed tables of clustering. Each side
of each switch runs against the oracle: single LP refinements from a seeded
random partition on a mesh-like and a skewed graph, and whole partitions."""
import numpy as np
import pytest

import graphgen
import oracle

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

KS = [15, 16, 17, 63, 64, 65, 255, 256, 257, 1024]
GRAPHS = {
    "rgg16k": graphgen.rgg2d(16384, 5),
    "rmat14": graphgen.rmat(14, 16),
    "weighted": graphgen.random_small(3000, 0.01, 4, wmax=9, vmax=5),
}


@pytest.fixture(scope="module")
def dev():
    return {k: gp.to_device(v) for k, v in GRAPHS.items()}


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("k", KS)
def test_lp_refine_at_k_boundaries(dev, name, k):
    g = GRAPHS[name]
    n = len(g["xadj"]) - 1
    part = np.array([graphgen.rand_u64(k + 7, i) % k for i in range(n)], np.int32)
    lm = oracle.lmax(oracle.total_vwgt(g), k, 0.03)
    P, st = gp.lp_refine(dev[name], torch.from_numpy(part).cuda(), k, lm, 25)
    oP, ost = oracle.lp_refine(g, part, k, lm, 25)
    assert np.array_equal(P.cpu().numpy(), oP)
    assert (st["rounds_run"], st["moves"]) == (ost["rounds_run"], ost["moves"])


@pytest.mark.gpu
@pytest.mark.parametrize("k", [16, 17, 64, 65, 256, 257])
def test_partition_at_k_boundaries(dev, k):
    g = GRAPHS["rmat14"]
    part, res = gp.partition(dev["rmat14"], k, 0.03)
    opart, ores = oracle.partition(g, k, 0.03)
    assert np.array_equal(part.cpu().numpy(), opart)
    for key in ("cut", "max_block_w", "balanced", "levels", "coarsest_n", "edge_visits_refine"):
        assert res[key] == ores[key], key


@pytest.mark.gpu
@pytest.mark.parametrize("k", [256, 257])
def test_partition_with_coarsening_at_the_byte_label_bound(k):
    # 65,536 vertices > 60 k: coarse levels are built and refined on both sides of the switch
    g = graphgen.rmat(16, 16)
    part, res = gp.partition(gp.to_device(g), k, 0.03)
    opart, ores = oracle.partition(g, k, 0.03)
    assert ores["levels"] > 1
    assert np.array_equal(part.cpu().numpy(), opart)
    for key in ("cut", "max_block_w", "balanced", "levels", "coarsest_n", "edge_visits_refine"):
        assert res[key] == ores[key], key


@pytest.mark.gpu
def test_partition_at_the_largest_block_count():
    # the initial partitioner supports up to 2,048 blocks: 2,048 equals the oracle (one level and,
    # on the larger graph, two), 2,049 is an argument error
    for n in (40000, 300000):
        g = graphgen.rgg2d(n, 8)
        part, res = gp.partition(gp.to_device(g), 2048, 0.03)
        opart, ores = oracle.partition(g, 2048, 0.03)
        assert np.array_equal(part.cpu().numpy(), opart), n
        assert (res["cut"], res["max_block_w"], res["levels"]) == (ores["cut"], ores["max_block_w"], ores["levels"])
    with pytest.raises(gp.GPError, match="2048"):
        gp.partition(gp.to_device(graphgen.rgg2d(40000, 8)), 2049, 0.03)
