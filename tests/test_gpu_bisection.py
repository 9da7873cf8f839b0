"""GPU parity of the initial bisection (§III-B) on the hand-traced graphs of
tests/test_oracle_bisection.py.

These graphs are below 60 k vertices, so the partition runs the initial
partitioner on the input itself. With one try and no refinement rounds, and
sides that fit L_max, the partition is the bisection alone: it must equal the
oracle's and the side traced by hand. With the default tries and rounds it must
still equal the oracle's."""
import numpy as np
import pytest

import oracle
from hand_graphs import path, spider, star, three_parts
from test_oracle_bisection import PARTS_SIDES, SPIDER_SIDES, STAR_SIDES, _seed_for

TRACED = [("star", star, STAR_SIDES), ("spider", spider, SPIDER_SIDES), ("three_parts", three_parts, PARTS_SIDES)]
BARE = dict(attempts=1, rounds_refine=0)


def _run(g, k, **params):
    import paper_1710_08231_amd as gp
    opart, ores = oracle.partition(g, k, 0.03, **params)
    part, res = gp.partition(gp.to_device(g), k, 0.03, **params)
    part = part.cpu().numpy()
    assert ores["levels"] == 1 and res["levels"] == 1
    assert np.array_equal(part, opart)
    assert res["cut"] == ores["cut"] and res["max_block_w"] == ores["max_block_w"]
    return part


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,sides", TRACED, ids=[t[0] for t in TRACED])
def test_bisection_equals_traced_side(name, make, sides):
    g = make()
    n = len(g["xadj"]) - 1
    for start, side in sides.items():
        part = _run(g, 2, seed=_seed_for(start, n, 2), **BARE)
        assert set(np.flatnonzero(part == 0).tolist()) == side, (name, start)


@pytest.mark.gpu
def test_four_blocks_on_a_path():
    g = path(8)
    seeds = [s for s in range(20000) if oracle.mix4(s, 0, 0, 4) % 8 == 5][:6]
    for seed in seeds:
        part = _run(g, 4, seed=seed, **BARE)
        # first bisection from 5: {3, 4, 5, 6} takes blocks 0 and 1
        assert sorted(np.flatnonzero(part <= 1).tolist()) == [3, 4, 5, 6]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,k", [("star", star, 2), ("spider", spider, 3), ("three_parts", three_parts, 2),
                                         ("three_parts", three_parts, 4), ("path16", lambda: path(16), 4),
                                         ("path9w", lambda: path(9, vwgt=[3, 1, 1, 3, 2, 1, 1, 2, 1]), 3)])
def test_default_tries_match_oracle(name, make, k):
    g = make()
    for seed in range(16):
        _run(g, k, seed=seed)
