"""The redo loop of Sec. 2.6 as one launch (plans built with one_launch,
plain fused, whose tiles all fit on the device at once): every tile waits
only for the tiles it reads from or feeds, between spans, instead of a
launch boundary.  Bitwise equal to the span-by-span launches of the same
layout and to the oracle, with and without checkpoints, through rswr_solve
and rswr_solve_noalloc, on layouts from one window to many, FP64 and
FP32."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_10477_amd as rs
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print("[case]", *a, flush=True)


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def lay_of(plan):
    lo, hi, _, _ = plan.layout()
    return oracle.explicit_layout(plan.M, lo, hi)


def busy(M, n_steps, seed):
    g = np.random.default_rng(seed)
    st = workloads.smooth_state(M, g, shift=2e-3)
    t = np.arange(n_steps + 1) * 0.9 / (M - 1)
    return st, np.sin(2 * np.pi * 7 * t) + 0.3, np.cos(2 * np.pi * 5 * t)


def solve(plan, st0, fa, fb, n, n0=0, ck=None):
    st = st0.clone()
    rs.rswr_solve(plan, st, fa, fb, n, n0=n0, checkpoints=ck)
    torch.cuda.synchronize()
    return st


CASES = [
    # M, N, P, tile, n_steps, n0
    (1001, 2, 20, None, 2000, 0),          # 182 spans, the smallest layout
    (4097, 8, 64, None, 301, 3),           # odd span count, restart level
    (2 ** 16 + 1, 16, 64, (64, 8), 700, 0),  # several tiles per window
    (20001, 1, 2, (256, 16), 170, 0),      # one window: cut ends only
    (2 ** 18, 128, 64, None, 1000, 0),     # the adjoint case's layout
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_one_launch_equals_span_launches_and_oracle(dtype, case):
    M, N, P, tile, n, n0 = CASES[case]
    say("one launch", dtype, CASES[case])
    plan = rs.Plan(M, N, P, tile=tile, dtype=dtype, one_launch=True)
    span_plan = rs.Plan(M, N, P, tile=tile, dtype=dtype)
    assert plan.info["one_launch"] == 1 and span_plan.info["one_launch"] == 0
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n0 + n, case)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    fa_d, fb_d, s_d = dev(fa, dtype), dev(fb, dtype), dev(st0, dtype)
    one = solve(plan, s_d, fa_d, fb_d, n, n0)
    per_span = solve(span_plan, s_d, fa_d, fb_d, n, n0)
    assert torch.equal(one, per_span)
    ref, _, _ = oracle.rswr(lay_of(plan), plan.info["lambda"], plan.info["dx"], fa, fb, n,
                            span=plan.span, state=st0, n0=n0)
    assert np.array_equal(one.cpu().numpy(), ref)
    # a second call replays the recorded launch with fresh counters
    again = solve(plan, s_d, fa_d, fb_d, n, n0)
    assert torch.equal(again, one)
    if case in (1, 4):
        # checkpoints: every span-boundary state and flux row as span by span
        cks = []
        for pl in (plan, span_plan):
            ck = pl.checkpoint_buffer(n)
            out = solve(pl, s_d, fa_d, fb_d, n, n0, ck=ck)
            assert torch.equal(out, one)
            cks.append(ck)
        assert torch.equal(cks[0], cks[1])
        # and the no-allocation solve (its workspace holds the counters too)
        st = s_d.clone()
        rs.rswr_solve_noalloc(plan, st, fa_d, fb_d, n, n0=n0)
        torch.cuda.synchronize()
        assert torch.equal(st, one)


def test_one_launch_not_taken_where_it_does_not_apply():
    # sources, general tiles, two-launch and QUIET plans keep the span launches
    assert rs.Plan(301, 20, 20, span_mode=rs.QUIET, one_launch=True).info["one_launch"] == 0
    assert rs.Plan(1001, 2, 20, fuse=False, one_launch=True).info["one_launch"] == 0
    amp = torch.zeros(1, 100, dtype=torch.float64, device=DEV)
    assert rs.Plan(4097, 8, 64, sources=([100], amp),
                   one_launch=True).info["one_launch"] == 0
