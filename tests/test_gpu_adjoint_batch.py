"""A batch of same-shape adjoint solves with chunked checkpoints
(rswr_solve_adjoint_batch): every problem's dJ/df_A, dJ/df_B and dJ/dlam are
bit-identical to its own forward solve with span checkpoints followed by
rswr_solve_adjoint, for any group size and segment length; one problem also
against the oracle's reverse mode in the same precision (FP64: 1e-12
relative; FP32: 1e-5, dJ/dlam against the magnitude sum of its terms)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_10477_amd as rs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print("[case]", *a, flush=True)


def sources(n_prob, n_steps, ld, M, seed):
    g = np.random.default_rng(seed)
    t = np.arange(ld) * 0.9 / (M - 1)
    fa = np.zeros((n_prob, ld))
    fb = np.zeros((n_prob, ld))
    for i in range(n_prob):
        c, w = g.uniform(0.05, 0.2) * n_steps * 0.9 / (M - 1), g.uniform(5, 20) / (M - 1)
        fa[i] = g.uniform(0.5, 2) * np.exp(-((t - c) / w) ** 2)
        fb[i] = 0.3 * np.sin(2 * np.pi * (i + 1) * t / t[-1])
    return fa, fb


CASES = [
    # M, N, P, windows, n_steps, receivers
    (4097, 8, 64, None, 300, [0, 1, 100, 1500, 2048, 3000, 4095, 4096]),
    (2001, 3, 0, ([0, 5, 1970], [30, 1995, 2000]), 200, [1, 3, 17, 1000, 1998, 1999]),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_batch_equals_single_solves(dtype, case):
    M, N, P, win, n_steps, rec = CASES[case]
    say("adjoint-batch", dtype, CASES[case][:5])
    plan = rs.Plan(M, N, P, windows=win, dtype=dtype)
    assert plan.info["fused"] == 1
    n_prob, ld = 3, n_steps + 4
    fa_np, fb_np = sources(n_prob, n_steps, ld, M, case)
    fa = torch.as_tensor(fa_np, dtype=dtype, device=DEV)
    fb = torch.as_tensor(fb_np, dtype=dtype, device=DEV)
    g = np.random.default_rng(10 + case)
    gtr = torch.as_tensor(g.standard_normal((n_prob, len(rec), n_steps)), dtype=dtype,
                          device=DEV)
    single = []
    for i in range(n_prob):
        ck = plan.checkpoint_buffer(n_steps)
        st = torch.zeros(2, M, dtype=dtype, device=DEV)
        fai = fa[i, :n_steps + 1].contiguous()
        fbi = fb[i, :n_steps + 1].contiguous()
        rs.rswr_solve(plan, st, fai, fbi, n_steps, checkpoints=ck)
        single.append(rs.rswr_solve_adjoint(plan, ck, fai, fbi, n_steps, rec,
                                            gtr[i].contiguous()))
    torch.cuda.synchronize()
    for group, seg in ((2, 2), (3, 0), (1, 4), (3, 50)):
        ga, gb, gl = rs.rswr_solve_adjoint_batch(plan, fa, fb, n_steps, rec, gtr,
                                                 group=group, seg=seg)
        torch.cuda.synchronize()
        for i in range(n_prob):
            sa, sb, sl = single[i]
            assert torch.equal(ga[i], sa), (group, seg, i)
            assert torch.equal(gb[i], sb), (group, seg, i)
            assert torch.equal(gl[i], sl), (group, seg, i)
    # one problem against the oracle's reverse mode in the same precision
    npdt = NP[dtype]
    ra, rb, rl, sa = oracle.adjoint(M, plan.info["lambda"], plan.info["dx"],
                                    fa_np[1, :n_steps + 1].astype(npdt),
                                    fb_np[1, :n_steps + 1].astype(npdt), n_steps, rec,
                                    gtr[1].cpu().numpy(), dtype=npdt, terms=True)
    a = ga[1].cpu().numpy().astype(np.float64)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert np.linalg.norm(a - ra) <= tol * np.linalg.norm(ra)
    if dtype == torch.float64:
        assert abs(gl[1].item() - rl) <= 1e-12 * abs(rl)
    assert abs(gl[1].item() - rl) <= tol * sa


def test_adjoint_batch_rejections():
    amp = torch.zeros(1, 100, dtype=torch.float64, device=DEV)
    f = torch.zeros(2, 60, dtype=torch.float64, device=DEV)
    gtr = torch.zeros(2, 1, 50, dtype=torch.float64, device=DEV)
    with pytest.raises(rs.RSWRError):  # plan with sources
        rs.rswr_solve_adjoint_batch(rs.Plan(4097, 8, 64, sources=([100], amp)), f, f, 50,
                                    [300], gtr)
    with pytest.raises(rs.RSWRError):  # two-launch plan
        rs.rswr_solve_adjoint_batch(rs.Plan(4097, 8, 64, fuse=False), f, f, 50, [300], gtr)
    with pytest.raises(rs.RSWRError):  # samples shorter than n_steps + 1
        rs.rswr_solve_adjoint_batch(rs.Plan(4097, 8, 64), f, f, 60, [300],
                                    torch.zeros(2, 1, 60, dtype=torch.float64, device=DEV))
