"""The allocation-free entry point gp_lp_refine_static, through the C ABI.

For callers that cannot allocate: its temporaries live in the library's
static per-GPU scratch array. Its output must equal gp_lp_refine's (the
existing entry point, which takes its scratch from the library cache) bit for
bit, on two calls in a row, the second on a smaller graph (the array keeps
the first call's contents, so whatever must start at zero is cleared by the
call itself). Sizes beyond the array are rejected before any device work.
"""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle


def _case(g, k, seed):
    n = len(g["xadj"]) - 1
    rng = np.random.default_rng(seed)
    part = rng.integers(0, k, n).astype(np.int32)
    lm = oracle.lmax(n if g.get("vwgt") is None else int(g["vwgt"].sum()), k, 0.03)
    return part, lm


@pytest.mark.gpu
def test_static_refine_matches_refine_twice_second_smaller():
    import torch
    import paper_1710_08231_amd as gp
    cases = [(graphgen.rmat(16, 21), 16, 1, 3), (graphgen.grid3d(20, 16, 9, seed=2, wmax=10), 8, 2, 1)]
    for g, k, seed, flags in cases:
        dg = gp.to_device(g)
        part, lm = _case(g, k, seed)
        P = torch.from_numpy(part).cuda()
        want, st_w = gp.lp_refine(dg, P, k, lm, 25, active=bool(flags & 2))
        got, st_g = gp.lp_refine_static(dg, P, k, lm, 25, active=bool(flags & 2))
        assert np.array_equal(want.cpu().numpy(), got.cpu().numpy())
        assert (st_g["rounds_run"], st_g["moves"], st_g["edge_visits"]) == \
               (st_w["rounds_run"], st_w["moves"], st_w["edge_visits"])
        assert 0 < st_g["workspace_bytes"] <= 64 << 20
        # and both equal the oracle's refinement
        opart, ost = oracle.lp_refine(g, part, k, lm, 25, active=bool(flags & 2))
        assert np.array_equal(got.cpu().numpy(), opart)


@pytest.mark.gpu
def test_static_refine_rejects_sizes_beyond_the_array():
    import paper_1710_08231_amd as gp
    lib = gp.load()
    # 8M vertices, 128M entries: beyond 64 MiB; rejected from the sizes alone
    fake = ctypes.c_void_p(1 << 40)
    g = gp.Graph(1 << 23, 1 << 27, fake, fake, None, None)
    st = gp.LPStats()
    rc = lib.gp_lp_refine_static(ctypes.byref(g), 16, 10, 25, 1, fake, ctypes.byref(st), None)
    assert rc == -3 and b"static scratch" in lib.gp_last_error()


@pytest.mark.gpu
@pytest.mark.parametrize("flags", [1, 3])
def test_static_refine_just_below_the_array_limit(flags):
    # the largest geometric graph (in steps of 5,000 vertices) whose workspace bound fits
    # the 64 MiB array: the bound must suffice there too, and the result equal gp_lp_refine's
    # and the oracle's
    import torch
    import paper_1710_08231_amd as gp
    limit, k = 64 << 20, 64

    def bound(n):
        g = graphgen.rgg2d(n, 31)
        return g, gp.workspace_bytes(2, n, len(g["adjncy"]), k, flags)

    # the bound grows about linearly with the size: start near the limit
    n = int(700000 * limit / bound(700000)[1]) // 5000 * 5000
    g, b = bound(n)
    while b > limit:
        n -= 5000
        assert n > 5000, "the workspace bound does not shrink with the graph"
        g, b = bound(n)
    best = (g, b)
    while True:
        n += 5000
        assert n < 4_000_000, "the workspace bound does not grow with the graph"
        g, b = bound(n)
        if b > limit:
            break
        best = (g, b)
    g, b = best
    assert b > 0.97 * limit
    dg = gp.to_device(g)
    part, lm = _case(g, k, 5)
    P = torch.from_numpy(part).cuda()
    got, st_g = gp.lp_refine_static(dg, P, k, lm, 25, active=bool(flags & 2))
    assert 0 < st_g["workspace_bytes"] <= b
    want, st_w = gp.lp_refine(dg, P, k, lm, 25, active=bool(flags & 2))
    assert np.array_equal(want.cpu().numpy(), got.cpu().numpy())
    assert (st_g["rounds_run"], st_g["moves"]) == (st_w["rounds_run"], st_w["moves"])
    opart, ost = oracle.lp_refine(g, part, k, lm, 25, active=bool(flags & 2))
    assert np.array_equal(got.cpu().numpy(), opart)
