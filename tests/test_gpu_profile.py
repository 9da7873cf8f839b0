"""GPU tests of the library's HIP-event instrumentation (gp_profile_*).

Profiling never changes a result; GP_PROFILE_KERNELS brackets every proposal
launch, GP_PROFILE_EAGER only the first round of every LP run (the sample the
benchmark takes inside its timed steps), GP_PROFILE_CALLS whole LP runs, and
GP_PROFILE_BY_LEVEL prefixes each name with its phase and level.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

G = graphgen.rmat(15, 15)


@pytest.fixture(scope="module")
def dg():
    return gp.to_device(G)


@pytest.fixture(scope="module")
def expected():
    return oracle.partition(G, 16, 0.03)


def _run(dg, mode, select=None):
    gp.profile_select(select)
    gp.profile_enable(mode)
    try:
        part, res = gp.partition(dg, 16, 0.03)
        entries = gp.profile_entries()
    finally:
        gp.profile_enable(0)
        gp.profile_select(None)
    return part.cpu().numpy(), res, entries


def test_kernels_mode_brackets_every_launch(dg, expected):
    part, res, entries = _run(dg, gp.PROFILE_KERNELS)
    assert np.array_equal(part, expected[0])
    assert entries and all(e["launches"] > 0 and e["ms"] > 0 and e["bytes"] > 0 for e in entries)


def test_eager_mode_samples_first_rounds_only(dg, expected):
    _, _, every = _run(dg, gp.PROFILE_KERNELS)
    top = max(every, key=lambda e: e["ms"])
    part, res, first = _run(dg, gp.PROFILE_EAGER, select=top["name"])
    assert np.array_equal(part, expected[0]) and res["cut"] == expected[1]["cut"]
    assert [e["name"] for e in first] == [top["name"]]
    # every LP run contributes its first round only
    assert 0 < first[0]["launches"] < top["launches"] and first[0]["bytes"] > 0


def test_calls_by_level(dg, expected):
    part, res, entries = _run(dg, gp.PROFILE_CALLS | gp.PROFILE_BY_LEVEL)
    assert np.array_equal(part, expected[0])
    names = {e["name"] for e in entries}
    assert "cluster L0|lp_cluster" in names and "refine L0|lp_refine" in names
    assert all(e["launches"] == 1 for e in entries)
