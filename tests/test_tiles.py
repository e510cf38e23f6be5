"""Host checks of the update tiles (no GPU): the stored ranges of one span
partition the grid, each lies in its window's owned range (gluing rule,
Sec. 2.5 Eq. (15)), and every stored node is at least S nodes away from any
region end whose data is not exact, so the cut cannot reach it in S levels."""
import numpy as np
import pytest

import paper_2203_10477_amd as rs

LAYOUTS = [
    dict(n_points=1001, n_sub=2, overlap=20),
    dict(n_points=2 ** 24, n_sub=4096, overlap=64),          # large plain case
    dict(n_points=2 ** 20, n_sub=64, overlap=64),            # plain 2^20 case
    dict(n_points=2 ** 18, n_sub=128, overlap=64),           # adjoint case
    dict(n_points=301, n_sub=20, overlap=20),
    dict(n_points=257, n_sub=1, overlap=2, span=40),
    dict(n_points=6000, n_sub=3, overlap=40, tile=(64, 8)),
    dict(n_points=20001, n_sub=16, overlap=64, tile=(256, 16)),
    dict(n_points=1201, n_sub=4, overlap=24, span_mode=rs.QUIET),
    dict(n_points=400, n_sub=4, overlap=0, windows=([0, 90, 200, 260], [110, 230, 290, 399])),
    dict(n_points=101, n_sub=2, overlap=0, windows=([0, 5], [30, 100])),
    dict(n_points=301, n_sub=20, overlap=20, span_mode=rs.QUIET, tile=(64, 8)),
]


def test_narrow_windows_under_long_spans_use_general_tiles():
    plan = rs.Plan(301, 20, 20, span_mode=rs.QUIET, tile=(64, 8))
    assert plan.tiles()[:, 7].sum() > 0


def check_plan(plan):
    M = plan.M
    lo, hi, olo, ohi = plan.layout()
    t = plan.tiles()
    S = plan.info["span"]
    TM = plan.info["tile_threads"] * plan.info["tile_per_thread"]
    assert TM >= 2 * S + 2
    assert np.all(t[:, 1] - t[:, 0] + 1 == TM)
    order = np.argsort(t[:, 2])
    st = t[order]
    assert st[0, 2] == 0 and st[-1, 3] == M - 1
    assert np.all(st[1:, 2] == st[:-1, 3] + 1)     # contiguous, disjoint
    assert np.all(st[:, 3] >= st[:, 2])
    for a, b, s_lo, s_hi, w, lm, rm, gen in t:
        assert olo[w] <= s_lo and s_hi <= ohi[w]
        lb0 = 1 if w == 0 else lo[w]
        rb0 = M - 2 if w == plan.N - 1 else hi[w]
        w0 = 0 if w == 0 else lo[w]          # window's left special node
        w1 = M - 1 if w == plan.N - 1 else hi[w]
        # left end: exact at the window's left end, the window's left end
        # strictly inside (general tile), or every stored node at least S
        # from the first node that is treated wrongly
        if lm == 1:
            assert w > 0 and a == lo[w]
        elif lm == 2:
            assert w == 0 and a == 1
        elif gen:
            assert a < lb0
        else:
            first_wrong = a if a > lb0 else w0
            assert s_lo >= first_wrong + S
        if rm == 1:
            assert w < plan.N - 1 and b == hi[w]
        elif rm == 2:
            assert w == plan.N - 1 and b == M - 2
        else:
            last_wrong = b if b < rb0 else w1
            assert s_hi <= last_wrong - S
        assert s_lo >= a or (lm == 2 and s_lo == 0)
        assert s_hi <= b or (rm == 2 and s_hi == M - 1)


@pytest.mark.parametrize("kw", LAYOUTS)
def test_tiles_partition_and_margins(kw):
    plan = rs.Plan(**kw)
    check_plan(plan)


def test_random_layouts():
    g = np.random.default_rng(0)
    for _ in range(60):
        P = 2 * int(g.integers(1, 70))
        N = int(g.integers(1, 40))
        M = int(g.integers((N + 1) * (P + 2), (N + 1) * (P + 2) + 5000))
        for dtype in ("f32", "f64"):
            import torch
            plan = rs.Plan(M, N, P, dtype=torch.float32 if dtype == "f32" else torch.float64)
            check_plan(plan)


def test_large_case_shape():
    plan = rs.Plan(2 ** 24, 4096, 64, dtype=__import__("torch").float32)
    assert plan.span == 35
    # the default shape is the one-wave 64x33 (wider or multi-wave shapes
    # run fewer waves per SIMD or a barrier per step): two tiles per window,
    # one carrying each input's frame; no general tiles
    assert (plan.info["tile_threads"], plan.info["tile_per_thread"]) == (64, 33)
    assert plan.info["n_tiles"] == 2 * 4096
    assert plan.tiles()[:, 7].sum() == 0
    # the widest shape: one tile per window, plus one for window 0 (narrower
    # than a tile: its nodes next to the Dirichlet node come from a second,
    # left-anchored tile)
    wide = rs.Plan(2 ** 24, 4096, 64, dtype=__import__("torch").float32, tile=(64, 65))
    assert wide.info["n_tiles"] == 4097
    assert wide.tiles()[:, 7].sum() == 0
