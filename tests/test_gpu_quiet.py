"""The adaptive (QUIET) loop of Sec. 2.6 inside rswr_solve: every span is
chosen on the device (predict -> select -> update, the level and the next
predictive span kept in a device control block), the whole loop recorded
as one graph.  The spans the device takes are those of the oracle's adaptive
loop, so states and receiver traces are bit-identical to it."""
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


def host(t):
    return t.detach().cpu().numpy()


def lay_of(plan):
    lo, hi, _, _ = plan.layout()
    return oracle.explicit_layout(plan.M, lo, hi)


def quiet_problem(M, n_steps, seed, smooth):
    """A pulse entering at X_A over a resting field (the spans grow while the
    overlaps are quiet, then shrink to the cone), or a busy smooth field."""
    g = np.random.default_rng(seed)
    t = np.arange(n_steps + 1) * 0.9 / (M - 1)
    fa = np.exp(-((t - 0.1) / 0.02) ** 2)
    fb = np.zeros(n_steps + 1)
    st = workloads.smooth_state(M, g) if smooth else np.zeros((2, M))
    return st, fa, fb


CASES = [
    # M, N, P, n_steps, n0, smooth, tile
    (1001, 2, 20, 2000, 0, False, None),
    (2001, 5, 20, 900, 0, False, (64, 8)),
    (3001, 10, 64, 700, 11, False, None),
    (2001, 3, 40, 400, 0, True, None),      # busy: every span at the cone
    (1001, 2, 20, 7, 0, False, None),       # fewer steps than one span
    (40001, 600, 20, 300, 0, False, None),  # 1198 flux rows: the select spans 75 work-groups
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_quiet_solve_matches_oracle(dtype, case):
    M, N, P, n_steps, n0, smooth, tile = CASES[case]
    say("quiet-solve", dtype, CASES[case])
    npdt = NP[dtype]
    plan = rs.Plan(M, N, P, span_mode=rs.QUIET, dtype=dtype, tile=tile)
    lay = lay_of(plan)
    st0, fa, fb = quiet_problem(M, n0 + n_steps, case, smooth)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    rec = np.array([0, 1, M // 3, M // 2, M - 2, M - 1], np.int64)
    ref, tr_ref, spans = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb,
                                     n_steps, mode=oracle.QUIET, state=st0, n0=n0, rec=rec)
    if case == 0:
        assert len(set(spans.tolist())) > 2  # the spans do vary
    fa_d, fb_d = dev(fa, dtype), dev(fb, dtype)
    for rep in range(2):  # the second call replays the recorded graph
        st = dev(st0, dtype)
        tr = rs.rswr_solve(plan, st, fa_d, fb_d, n_steps, n0=n0, receivers=rec)
        torch.cuda.synchronize()
        assert np.array_equal(host(st), ref), rep
        assert np.array_equal(host(tr), tr_ref), rep


def test_quiet_solve_rejects_checkpoints():
    plan = rs.Plan(1001, 2, 20, span_mode=rs.QUIET)
    st = torch.zeros(2, 1001, dtype=torch.float64, device=DEV)
    f = torch.zeros(101, dtype=torch.float64, device=DEV)
    fixed = rs.Plan(1001, 2, 20)
    ck = fixed.checkpoint_buffer(100)
    with pytest.raises(rs.RSWRError):
        rs.rswr_solve(plan, st, f, f, 100, checkpoints=ck)
