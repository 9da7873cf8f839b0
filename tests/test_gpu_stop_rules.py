"""GPU parity of the coarsening stop rules and the initial-try selection on the
hand-traced graphs of tests/test_oracle_stop_rules.py (§III-A "small enough",
§III-B best of the tries): same levels, coarsest size and partition as the
oracle, and the hand-derived level counts."""
import numpy as np
import pytest

import oracle
from hand_graphs import path_and_heavy_pairs, two_cliques

CASES = [
    # (light path, heavy pairs, k, params, hand-derived (levels, coarsest_n))
    (4, 8, 1, dict(coarsest_per_k=20), (1, 20)),
    (4, 8, 1, dict(coarsest_per_k=19), (2, 19)),
    (4, 19, 1, dict(coarsest_per_k=1), (2, 41)),
    (4, 8, 1, dict(coarsest_per_k=1), (3, 18)),
    (140, 1, 3, dict(coarsest_per_k=1, stall_num=1, stall_den=1), (71, 72)),
]


@pytest.mark.gpu
@pytest.mark.parametrize("light,pairs,k,params,expect", CASES)
def test_stop_rules_match_oracle(light, pairs, k, params, expect):
    import paper_1710_08231_amd as gp
    g = path_and_heavy_pairs(light, pairs)
    params = dict(params, rounds_coarsen=1)
    opart, ores = oracle.partition(g, k, 0.03, **params)
    part, res = gp.partition(gp.to_device(g), k, 0.03, **params)
    assert (ores["levels"], ores["coarsest_n"]) == expect
    assert (res["levels"], res["coarsest_n"]) == expect
    assert np.array_equal(part.cpu().numpy(), opart)
    assert res["cut"] == ores["cut"] and res["max_block_w"] == ores["max_block_w"]


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(8))
def test_tied_tries_keep_the_first(seed):
    import paper_1710_08231_amd as gp
    g = two_cliques(5)
    # 10 vertices <= 60 k: no coarsening, the tries run on the input graph itself
    opart, ores = oracle.partition(g, 2, 0.03, seed=seed)
    part, res = gp.partition(gp.to_device(g), 2, 0.03, seed=seed)
    start0 = oracle.mix4(seed, 0, 0, 2) % 10
    assert ores["levels"] == 1 and opart[start0] == 0
    assert np.array_equal(part.cpu().numpy(), opart)
