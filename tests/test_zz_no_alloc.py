"""rswr_solve_noalloc, the solve whose workspace is the library's own device
array (no allocation), through the C-ABI: bitwise equal to rswr_solve on the
same plan and inputs for two calls in a row, the second on a smaller problem
(FIXED FP64 with an even span count, then FIXED FP32 with an odd one), a
QUIET plan, launches captured into a graph and replayed; and its
rejections."""
import numpy as np
import pytest
import torch

import paper_2203_10477_amd as rs
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)


def inputs(M, n_steps, dtype, seed):
    g = np.random.default_rng(seed)
    st = workloads.smooth_state(M, g, shift=2e-3)
    t = np.arange(n_steps + 1) * 0.9 / (M - 1)
    fa = np.sin(2 * np.pi * 7 * t) + 0.3
    fb = np.cos(2 * np.pi * 5 * t)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)
    return dev(st), dev(fa), dev(fb)


def reference(plan, st0, fa, fb, n_steps, n0=0):
    st = st0.clone()
    rs.rswr_solve(plan, st, fa, fb, n_steps, n0=n0)
    torch.cuda.synchronize()
    return st


def test_noalloc_equals_solve_two_calls_in_a_row():
    cases = [  # M, N, P, dtype, n_steps, n0; the second problem is the smaller
        (2 ** 20, 64, 64, torch.float64, 35 * 12, 0),
        (4097, 8, 64, torch.float32, 301, 4),
    ]
    prepared = []
    for i, (M, N, P, dtype, n, n0) in enumerate(cases):
        plan = rs.Plan(M, N, P, dtype=dtype)
        st0, fa, fb = inputs(M, n0 + n, dtype, i)
        ref = reference(plan, st0, fa, fb, n, n0)  # also puts the plan's tables on the GPU
        prepared.append((plan, st0, fa, fb, n, n0, ref))
    for plan, st0, fa, fb, n, n0, ref in prepared:
        say("noalloc", plan.M, plan.N, plan.dtype, n, n0)
        st = st0.clone()
        rs.rswr_solve_noalloc(plan, st, fa, fb, n, n0=n0)
        torch.cuda.synchronize()
        assert torch.equal(st, ref)


def test_noalloc_quiet_plan():
    M, N, P, n = 1201, 4, 24, 500
    say("noalloc quiet")
    plan = rs.Plan(M, N, P, span_mode=rs.QUIET, dtype=torch.float64)
    st0, fa, fb = inputs(M, n, torch.float64, 7)
    ref = reference(plan, st0, fa, fb, n)
    for _ in range(2):
        st = st0.clone()
        rs.rswr_solve_noalloc(plan, st, fa, fb, n)
        torch.cuda.synchronize()
        assert torch.equal(st, ref)


def test_noalloc_under_graph_capture():
    """The launches of one call recorded into a graph by the caller and
    replayed several times, with eager work and synchronisations between
    the replays; every replay equals the eager solve."""
    M, N, P, n = 40001, 16, 64, 35 * 9
    say("noalloc capture")
    plan = rs.Plan(M, N, P, dtype=torch.float32)
    st0, fa, fb = inputs(M, n, torch.float32, 11)
    ref = reference(plan, st0, fa, fb, n)
    st = st0.clone()
    rs.rswr_solve_noalloc(plan, st, fa, fb, n)  # first call on this device, outside capture
    torch.cuda.synchronize()
    assert torch.equal(st, ref)
    g = torch.cuda.CUDAGraph()
    st.copy_(st0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        rs.rswr_solve_noalloc(plan, st, fa, fb, n)
    for rep in range(3):
        st.copy_(st0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(st, ref), rep
        (st0 * 2).sum().item()  # eager work between replays


def test_noalloc_rejections():
    big = rs.Plan(2 ** 24, 4096, 64, dtype=torch.float32)  # 134 MB of workspace
    x = torch.zeros(8, dtype=torch.float32, device=DEV)
    st = torch.zeros(2, 2 ** 24, dtype=torch.float32, device=DEV)
    with pytest.raises(rs.RSWRError) as e:
        rs.rswr_solve_noalloc(big, st, x, x, 7)
    assert e.value.status == 5  # NOMEM
    fresh = rs.Plan(3001, 5, 16, dtype=torch.float32)  # tables never uploaded
    s2 = torch.zeros(2, 3001, dtype=torch.float32, device=DEV)
    with pytest.raises(rs.RSWRError) as e:
        rs.rswr_solve_noalloc(fresh, s2, x, x, 7)
    assert e.value.status == 8  # UNSUPPORTED
