"""Parity on the full benchmark workloads, at their own sizes, in the launch
configurations the benchmark times.

* 2^20 nodes, 64 windows, overlap 64, 10^4 steps, FP64 and FP32: the whole
  final state and receiver traces bitwise against the oracle's RSWR.
* 512 batched problems (2^12..2^18 nodes, 4096 steps): every final state of
  the FP32 batch bitwise against the FP32 oracle, every state of the FP64
  batch bitwise against the FP64 oracle, FP32 against FP64 within FP32
  accuracy.
* 2^24 nodes, 4096 windows, 2*10^4 steps, FP32, at the autotuned tile: the
  whole final state and receiver traces bitwise against the FP32 oracle RSWR
  (572 spans); the state at every 100th span boundary, advanced one span in
  FP32 and by the oracle in FP64 from the same FP32 state, within 1e-5
  (relative L2): the per-span exactness of the Prediction Validation Theorem
  holds in FP32 up to rounding.
* 2^18 nodes, 128 windows, 8192 steps, FP64, 16 receivers: the gradient of
  the misfit against central differences (h = 1e-6) in a, in 16 random and
  the last 8 samples of f_A, and along 4 random directions.
* the 2^24-node batch of adjoint solves (FP32): two problems against the
  oracle's reverse mode in FP32 and FP64.
The oracle's CPU time dominates these tests (about a minute each on 16
threads for the 2^24-node and the 512-problem cases)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_10477_amd as rs
import workloads
from paper_2203_10477_amd.autotune import autotune, autotune_batch, batch_plans

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print("[case]", *a, flush=True)


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def rel_l2(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)


def lay_of(plan):
    lo, hi, _, _ = plan.layout()
    return oracle.explicit_layout(plan.M, lo, hi)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2p20_whole_run_bitwise(dtype):
    prob = workloads.config2(NP[dtype])
    say("2^20 whole run", dtype)
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=dtype)
    assert plan.span == 35 and plan.info["fused"]
    fa, fb = prob.sources()
    rec = np.array([0, 1, 1000, 4000, 8000, 9100, 500000, prob.M - 1], np.int64)
    ref, tr_ref, spans = oracle.rswr(lay_of(plan), prob.lam, prob.dx, fa, fb, prob.n_steps,
                                     span=plan.span, rec=rec)
    assert len(spans) == 286 and np.count_nonzero(ref[1]) > 5000
    st = torch.zeros(2, prob.M, dtype=dtype, device=DEV)
    fa_d, fb_d = dev(fa, dtype), dev(fb, dtype)
    rs.rswr_solve(plan, st, fa_d, fb_d, prob.n_steps)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    st.zero_()
    tr = rs.rswr_solve(plan, st, fa_d, fb_d, prob.n_steps, receivers=rec)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)


def _batch_states(plans, probs, dtype):
    b = rs.Batch(plans)
    st = [torch.zeros(2, p.M, dtype=dtype, device=DEV) for p in plans]
    fa = [dev(q.fa, dtype) for q in probs]
    fb = [dev(q.fb, dtype) for q in probs]
    rs.rswr_batch_solve(b, st, fa, fb, [q.n_steps for q in probs])
    torch.cuda.synchronize()
    return [host(s) for s in st]


def _batch_oracle(plans, probs, npdt):
    return oracle.rswr_many([lay_of(p) for p in plans], [p.info["lambda"] for p in plans],
                            [p.info["dx"] for p in plans],
                            [q.fa.astype(npdt) for q in probs],
                            [q.fb.astype(npdt) for q in probs],
                            [q.n_steps for q in probs], [p.span for p in plans])


@pytest.mark.timeout(900)
def test_batched_512_problems_bitwise_fp32_and_fp64():
    probs, _ = workloads.config3()
    assert len(probs) == 512
    out = {}
    for dtype in (torch.float32, torch.float64):
        say("batch 512", dtype)
        tiles, spans, _ = autotune_batch(probs, dtype=dtype, measure=False)
        plans = batch_plans(probs, dtype, tiles=tiles, spans=spans)
        got = _batch_states(plans, probs, dtype)
        say("oracle 512", dtype)
        ref = _batch_oracle(plans, probs, NP[dtype])
        bad = [i for i in range(len(probs)) if not np.array_equal(got[i], ref[i])]
        assert not bad, bad[:10]
        out[dtype] = got
    # FP32 against FP64 (same spans, same operation order): a 4096-step FP32
    # leapfrog carries FP32 rounding of a few 1e-4; on the eight problems
    # where the batch's FP32 result lies farthest from its FP64 result it is
    # no worse than twice the FP32 single-domain solve's own error
    err = np.array([rel_l2(a, b) for a, b in zip(out[torch.float32], out[torch.float64])])
    say("batch 512: FP32 vs FP64 relative L2, median / max", np.median(err), err.max())
    for i in np.argsort(-err)[:8]:
        q = probs[i]
        r64, _ = oracle.single(q.M, q.lam, q.dx, q.fa, q.fb, q.n_steps)
        s32, _ = oracle.single(q.M, q.lam, q.dx, q.fa.astype(np.float32),
                               q.fb.astype(np.float32), q.n_steps)
        assert rel_l2(out[torch.float64][i], r64) <= 1e-12, i
        assert err[i] <= 2 * rel_l2(s32, r64) + 1e-7, (i, err[i], rel_l2(s32, r64))


@pytest.mark.timeout(900)
def test_2p24_fp32_whole_run_bitwise_and_fp64_spot_checks():
    prob = workloads.config5(np.float32)
    say("2^24 fp32: autotune")
    tile, _ = autotune(prob.M, prob.N, prob.P, dtype=torch.float32, reps=5)
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32, tile=tile)
    S = plan.span
    assert S == 35 and plan.info["fused"]
    lay = lay_of(plan)
    fa, fb = prob.sources()
    fa_d, fb_d = dev(fa, torch.float32), dev(fb, torch.float32)
    n = prob.n_steps
    K = -(-n // S)
    assert K == 572
    # the solve the benchmark times: from rest, no receivers, one graph
    st = torch.zeros(2, prob.M, dtype=torch.float32, device=DEV)
    ws = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device=DEV)
    rs.rswr_solve(plan, st, fa_d, fb_d, n, workspace=ws)
    torch.cuda.synchronize()
    bench_state = host(st)
    # receivers on nodes the wave reaches (it travels about 18000 nodes)
    rec = np.array([0, 1, 64, 2080, 2112, 4160, 9000, 17000], np.int64)
    st.zero_()
    tr = rs.rswr_solve(plan, st, fa_d, fb_d, n, receivers=rec)
    torch.cuda.synchronize()
    say("2^24 fp32: oracle (572 spans)")
    ref, tr_ref, spans = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, n, span=S, rec=rec)
    assert len(spans) == K
    assert np.count_nonzero(ref[1]) > 10000
    assert np.array_equal(bench_state, ref)
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)
    assert np.count_nonzero(tr_ref[-2]) > 0
    # FP64 spot checks on 1% of the spans: the run's own FP32 state at span
    # boundary k (k = 0, 100, ..., 500; the run restarted at level k S gives
    # the same bits as the whole run), one span in FP32 on the GPU and in
    # FP64 by the oracle (literal predict + update) from that state with the
    # same boundary samples
    st.zero_()
    lev = 0
    fa64, fb64 = fa.astype(np.float64), fb.astype(np.float64)
    worst = 0.0
    for k in range(0, K, 100):
        if k * S > lev:
            rs.rswr_solve(plan, st, fa_d, fb_d, k * S - lev, n0=lev)
            lev = k * S
        s32 = host(st)
        one = min(S, n - lev)
        out32 = host(rs.rswr_span(plan, st, fa_d, fb_d, lev, span=one))
        say("2^24 spot check span", k)
        x64 = s32.astype(np.float64)
        fl = oracle.predict(lay, prob.lam, prob.dx, fa64, fb64, lev, one, x64)
        out64, _ = oracle.update(lay, prob.lam, prob.dx, fa64, fb64, lev, one, x64, fl)
        assert np.linalg.norm(out64) > 0
        e = rel_l2(out32, out64)
        worst = max(worst, e)
        assert e <= 1e-5, (k, e)
    say("2^24 spot checks: worst relative L2", worst)
    rs.rswr_solve(plan, st, fa_d, fb_d, n - lev, n0=lev)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)


@pytest.mark.timeout(600)
def test_2p18_adjoint_finite_differences():
    """dJ/da and dJ/df_A of the 2^18-node, 8192-step FP64 case (misfit
    against data from a run at a = 1.1) by the adjoint, against central
    differences with h = 1e-6 of the GPU forward solve.  J is quadratic in
    f_A, so its central differences are exact up to rounding (about
    eps J / h); in a they carry an O(h^2) error as well."""
    prob = workloads.config4()
    say("2^18 adjoint FD")
    M, n, rec = prob.M, prob.n_steps, prob.rec
    fa_np, _ = prob.sources()
    spec = rs.ProblemSpec(M, prob.N, prob.P, n, rec, dtype=torch.float64)
    with torch.no_grad():
        d = rs.RSWRFunction.apply(dev(fa_np, torch.float64),
                                  torch.tensor(1.1, dtype=torch.float64), spec)
    fa = dev(fa_np, torch.float64).requires_grad_(True)
    a = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    J = ((rs.RSWRFunction.apply(fa, a, spec) - d) ** 2).sum()
    J.backward()
    ga = host(fa.grad)
    gA = float(a.grad.item())
    J0 = float(J.item())
    assert J0 > 0 and abs(gA) > 0 and np.abs(ga).max() > 0

    def J_at(f, av):
        with torch.no_grad():
            tr = rs.RSWRFunction.apply(dev(f, torch.float64),
                                       torch.tensor(av, dtype=torch.float64), spec)
            return float(((tr - d) ** 2).sum().item())

    h = 1e-6
    fd_a = (J_at(fa_np, 1 + h) - J_at(fa_np, 1 - h)) / (2 * h)
    assert abs(fd_a - gA) <= 1e-6 * abs(gA), (fd_a, gA)
    g = np.random.default_rng(44)
    idx = list(np.sort(g.choice(np.arange(1, n - 8), 16, replace=False))) + \
        list(range(n - 7, n + 1))
    gmax = np.abs(ga).max()
    for i in idx:
        e = np.zeros(n + 1)
        e[i] = h
        fd = (J_at(fa_np + e, 1.0) - J_at(fa_np - e, 1.0)) / (2 * h)
        if i > n - min(rec):
            # no receiver sees f_A[i] within the run: both are exactly zero
            assert fd == 0.0 and ga[i] == 0.0, i
        else:
            assert abs(fd - ga[i]) <= 1e-6 * gmax, (i, fd, ga[i])
    for _ in range(4):
        v = g.standard_normal(n + 1)
        v[0] = 0.0
        v /= np.linalg.norm(v)
        fd = (J_at(fa_np + h * v, 1.0) - J_at(fa_np - h * v, 1.0)) / (2 * h)
        assert abs(fd - float(ga @ v)) <= 1e-6 * np.linalg.norm(ga), (fd, float(ga @ v))


@pytest.fixture(scope="module")
def adjoint_batch_2p24():
    """Two problems of the 2^24-node batch of adjoint solves (FP32, random
    Ricker sources, 16 receivers on nodes the wave reaches, random dJ/dtrace)
    and the oracle's reverse mode of each in FP32 and FP64.  From rest,
    driven at node 0, nothing beyond node n_steps + 2 reaches any value the
    gradient reads, so the oracle runs on the first n_steps + 3 nodes
    (dJ/df_A bit for bit the whole domain's)."""
    prob = workloads.config5(np.float32)
    n = prob.n_steps
    say("2^24 adjoint batch (2 problems)")
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32, tile=(64, 33))
    fa_np = workloads.adjoint_batch_sources(prob.M, n, 64)[:2].astype(np.float32)
    fa = dev(fa_np, torch.float32)
    fb = torch.zeros_like(fa)
    g = workloads.rng(56)
    rec = workloads.receivers(g, 16, min(prob.M - 2, int(0.8 * 0.9 * n)))
    gtr_np = g.standard_normal((2, len(rec), n)).astype(np.float32)
    ga, _, gl = rs.rswr_solve_adjoint_batch(plan, fa, fb, n, rec, dev(gtr_np, torch.float32),
                                            group=2)
    torch.cuda.synchronize()
    out = []
    for y in range(2):
        say("oracle reverse mode, problem", y)
        refs = [oracle.adjoint(n + 3, prob.lam, prob.dx, fa_np[y].astype(t),
                               np.zeros(n + 1, t), n, rec, gtr_np[y].astype(t), ck=200,
                               dtype=t, terms=True) for t in (np.float32, np.float64)]
        out.append((host(ga[y]), float(gl[y].item()), refs[0], refs[1]))
    return out


@pytest.mark.timeout(600)
def test_2p24_adjoint_batch_dJdf(adjoint_batch_2p24):
    """dJ/df_A of a 20000-level FP32 reverse sweep carries FP32 rounding of
    order 1e-4; the batch's is as accurate as the FP32 oracle's (within
    twice its distance from the FP64 oracle)."""
    for ga, _, r32, r64 in adjoint_batch_2p24:
        e_ref = rel_l2(r32[0], r64[0])
        assert rel_l2(ga, r64[0]) <= 2 * e_ref + 1e-6, (rel_l2(ga, r64[0]), e_ref)


@pytest.mark.timeout(600)
def test_2p24_adjoint_batch_dJdlam(adjoint_batch_2p24):
    """dJ/dlam sums about 10^10 terms W Lap U that cancel to 1/80..1/800 of
    their magnitudes; FP32 rounding over 20000 levels then moves it by an
    amount that varies from problem to problem (the FP32 oracle itself lands
    1e-6..2e-5 of the magnitude sum from the FP64 one on these two).  The
    bound: the relative accuracy the FP32 oracle reaches on dJ/df_A of the
    same run, against the magnitude sum, and never tighter than 1e-5."""
    for _, gl, r32, r64 in adjoint_batch_2p24:
        e32 = max(rel_l2(r32[0], r64[0]), 1e-5)
        assert abs(gl - r64[2]) <= e32 * r64[3], (gl, r64[2], r64[3], e32)
