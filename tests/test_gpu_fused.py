"""GPU parity of the fused span: each span as one launch, the prediction of
every input end (Sec. 2.3) carried by the wave that holds the end.

Against the CPU oracle (literal predict + update, the same operation order)
the results are bit-identical; against the two-launch path on the GPU the
states, traces and the predicted flux rows kept for the adjoint are too."""
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


def busy(M, n_steps, seed):
    g = np.random.default_rng(seed)
    st = workloads.smooth_state(M, g, shift=2e-3)
    t = np.arange(n_steps + 1) * 0.9 / (M - 1)
    fa = np.sin(2 * np.pi * 7 * t) + 0.3
    fb = np.cos(2 * np.pi * 5 * t)
    return st, fa, fb


def lay_of(plan):
    lo, hi, _, _ = plan.layout()
    return oracle.explicit_layout(plan.M, lo, hi)


def used_rows(plan):
    """Flux rows (2 i + side) that some tile reads: side 0 feeds the left
    input of window i+1, side 1 the right input of window i."""
    rows = set()
    for _, _, _, _, w, lm, rm, _ in plan.tiles():
        if lm == 1:
            rows.add(2 * (w - 1))
        if rm == 1:
            rows.add(2 * w + 1)
    return sorted(rows)


FUSE_CASES = [
    # M, N, P, windows, tile, n_steps, n0, span
    (1001, 2, 20, None, None, 211, 5, 0),
    (4097, 8, 64, None, None, 400, 0, 0),
    (4097, 8, 64, None, (128, 8), 300, 0, 0),       # two waves per tile
    (6000, 3, 40, None, (64, 8), 190, 0, 0),        # several tiles per window
    (20001, 16, 64, None, (256, 16), 177, 2, 0),    # four waves per tile
    # a window exactly one region wide: both inputs in one tile
    (2001, 3, 0, ([0, 400, 800], [700, 911, 2000]), (64, 8), 150, 0, 0),  # one wave, S 61
    (2501, 3, 0, ([0, 400, 1300], [700, 1423, 2500]), (128, 8), 150, 0, 50),  # two waves
    (4097, 8, 64, None, (64, 33), 100, 0, 63),      # the largest fused span
    # frames holding the Dirichlet nodes: node 0 in the frame of window 1's
    # left input, node M-1 in the frame of its right input
    (2001, 3, 0, ([0, 5, 1970], [30, 1995, 2000]), (64, 8), 160, 0, 0),
    (2001, 3, 0, ([0, 5, 1970], [30, 1995, 2000]), (128, 8), 120, 3, 0),
    (2001, 2, 0, ([0, 5], [30, 2000]), None, 140, 0, 0),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(FUSE_CASES)))
def test_fused_solve_bitwise(dtype, case):
    M, N, P, win, tile, n_steps, n0, span = FUSE_CASES[case]
    if dtype == torch.float64 and tile is not None and tile[1] > 22:
        tile = (64, 16)  # the shape holds no FP64 kernel: the widest FP64 one-wave shape
    say("fused-solve", dtype, FUSE_CASES[case])
    plan = rs.Plan(M, N, P, windows=win, tile=tile, span=span, dtype=dtype)
    two = rs.Plan(M, N, P, windows=win, tile=tile, span=span, dtype=dtype, fuse=False)
    assert plan.info["fused"] == 1 and two.info["fused"] == 0
    lay = lay_of(plan)
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n0 + n_steps, seed=case)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    g = np.random.default_rng(case)
    rec = np.unique(np.concatenate([[0, 1, M - 2, M - 1], g.integers(0, M, 6)]))
    ref, tr_ref, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb,
                                 n_steps, span=plan.span, state=st0, n0=n0, rec=rec)
    fa_d, fb_d = dev(fa, dtype), dev(fb, dtype)
    st = dev(st0, dtype)
    tr = rs.rswr_solve(plan, st, fa_d, fb_d, n_steps, n0=n0, receivers=rec)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)

    # checkpoints: span states and the used flux rows match the two-launch path
    K = plan.n_spans(n_steps)
    cks = []
    for p in (plan, two):
        ck = p.checkpoint_buffer(n_steps)
        s = dev(st0, dtype)
        rs.rswr_solve(p, s, fa_d, fb_d, n_steps, n0=n0, checkpoints=ck)
        torch.cuda.synchronize()
        assert np.array_equal(host(s), ref)
        cks.append(ck)
    st_f = host(plan.checkpoint_states(cks[0], n_steps))
    st_t = host(two.checkpoint_states(cks[1], n_steps))
    assert np.array_equal(st_f, st_t)
    off = (K + 1) * 2 * M
    fl_f = host(cks[0].reshape(-1)[off:]).reshape(K, max(N - 1, 1) * 2, plan.flux_ld)
    fl_t = host(cks[1].reshape(-1)[off:]).reshape(K, max(N - 1, 1) * 2, plan.flux_ld)
    rows = used_rows(plan)
    assert rows
    for k in range(K):
        S_k = min(plan.span, n_steps - k * plan.span)
        assert np.array_equal(fl_f[k][rows, :S_k], fl_t[k][rows, :S_k]), k


GRID_CASES = [
    # M, N, P, tile, n_steps: one to four waves per tile, and grids of
    # several thousand tiles
    (4097, 8, 64, (64, 8), 300),
    (20001, 16, 64, (256, 16), 177),
    (2001, 3, 20, (128, 8), 150),
    (3000001, 64, 64, (64, 8), 90),
    (3000001, 96, 64, (64, 16), 75),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(GRID_CASES)))
def test_fused_grids_bitwise(dtype, case):
    """Fused solves on small and large grids: the state bitwise equal to the
    oracle's RSWR and to the two-launch path, with and without checkpoints
    (checkpoint states equal too)."""
    M, N, P, tile, n_steps = GRID_CASES[case]
    say("fused-grid", dtype, GRID_CASES[case])
    plan = rs.Plan(M, N, P, tile=tile, dtype=dtype)
    two = rs.Plan(M, N, P, tile=tile, dtype=dtype, fuse=False)
    assert plan.info["fused"] == 1 and two.info["fused"] == 0
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n_steps, seed=100 + case)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    fa_d, fb_d = dev(fa, dtype), dev(fb, dtype)
    outs, cks = [], []
    for p in (plan, two):
        s = dev(st0, dtype)
        rs.rswr_solve(p, s, fa_d, fb_d, n_steps)
        ck = p.checkpoint_buffer(n_steps)
        s2 = dev(st0, dtype)
        rs.rswr_solve(p, s2, fa_d, fb_d, n_steps, checkpoints=ck)
        torch.cuda.synchronize()
        outs.append(host(s))
        assert np.array_equal(host(s2), outs[-1])
        cks.append(host(p.checkpoint_states(ck, n_steps)))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(cks[0], cks[1])
    lay = lay_of(plan)
    ref, _, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n_steps,
                            span=plan.span, state=st0)
    assert np.array_equal(outs[0], ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_span_entry_point(dtype):
    """rswr_span: one whole span, fused and two-launch, against the oracle's
    predict + update; the fused call's flux rows against the oracle's
    prediction; a short last span."""
    M, N, P = 1001, 2, 20
    say("span", dtype)
    plan = rs.Plan(M, N, P, dtype=dtype)
    two = rs.Plan(M, N, P, dtype=dtype, fuse=False)
    lay = lay_of(plan)
    npdt = NP[dtype]
    st0, fa, fb = busy(M, 300, seed=4)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    n0 = 17
    fa_d, fb_d, st_d = dev(fa, dtype), dev(fb, dtype), dev(st0, dtype)
    for S in (plan.span, 4, 1):
        ref_flux = oracle.predict(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n0, S,
                                  st0, ld=plan.flux_ld)
        ref, _ = oracle.update(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n0, S, st0,
                               ref_flux)
        fl = plan.flux_buffer()
        out = rs.rswr_span(plan, st_d, fa_d, fb_d, n0, span=S, flux=fl)
        out2 = rs.rswr_span(two, st_d, fa_d, fb_d, n0, span=S, flux=two.flux_buffer())
        out3 = rs.rswr_span(plan, st_d, fa_d, fb_d, n0, span=S)
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref), S
        assert np.array_equal(host(out2), ref), S
        assert np.array_equal(host(out3), ref), S
        rows = used_rows(plan)
        got = host(fl).reshape(-1, plan.flux_ld)
        want = ref_flux.reshape(-1, plan.flux_ld)
        assert np.array_equal(got[rows, :S], want[rows, :S]), S
    with pytest.raises(rs.RSWRError):
        rs.rswr_span(plan, st_d, fa_d, fb_d, n0, span=plan.span + 1)
    with pytest.raises(rs.RSWRError):
        rs.rswr_span(two, st_d, fa_d, fb_d, n0)  # two launches need a flux buffer


def test_large_fp32_fused_span_every_shape():
    """The 2^24-node FP32 case (4096 windows, overlap 64, span 35) as the
    benchmark runs it: one fused span from a smooth state in every built
    kernel shape, sampled windows bitwise against the oracle's literal
    predict + update in FP32, the whole state bitwise against the two-launch
    path, and the input ends' flux rows against the oracle's prediction."""
    prob = workloads.config5(np.float32)
    say("large-2^24-fp32-fused")
    g = np.random.default_rng(78)
    st32 = workloads.smooth_state(prob.M, g, shift=prob.lam * prob.dx).astype(np.float32)
    fa, fb = prob.sources()
    n0 = 1000
    st_d = dev(st32, torch.float32)
    fa_d, fb_d = dev(fa, torch.float32), dev(fb, torch.float32)
    base = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32, fuse=False)
    S = base.span
    assert S == 35
    lay = lay_of(base)
    ref_flux = oracle.predict(lay, prob.lam, prob.dx, fa, fb, n0, S, st32, ld=base.flux_ld)
    wins = [0, 1, 2, 777, 2048, 4000, prob.N - 2, prob.N - 1]
    ref, _ = oracle.update(lay, prob.lam, prob.dx, fa, fb, n0, S, st32, ref_flux,
                           windows=wins)
    two = host(rs.rswr_span(base, st_d, fa_d, fb_d, n0, flux=base.flux_buffer()))
    for w in wins:
        sl = slice(lay.own_lo[w], lay.own_hi[w] + 1)
        assert np.array_equal(two[:, sl], ref[:, sl]), w
    from paper_2203_10477_amd.autotune import kernel_shapes
    n_fused = 0
    for th, pt, _ in kernel_shapes():
        try:
            plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32, tile=(th, pt))
        except rs.RSWRError:
            continue
        say("shape", th, pt)
        assert plan.info["fused"] == 1
        n_fused += 1
        fl = plan.flux_buffer()
        got = host(rs.rswr_span(plan, st_d, fa_d, fb_d, n0, flux=fl))
        assert np.array_equal(got, two), (th, pt)
        rows = used_rows(plan)
        gf = host(fl).reshape(-1, plan.flux_ld)
        assert np.array_equal(gf[rows, :S], ref_flux.reshape(-1, base.flux_ld)[rows, :S])
    assert n_fused >= 8


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_many_receivers_in_one_tile(dtype):
    """Eleven receivers inside one tile (the tile is launched once per group
    of four), a repeated receiver and both Dirichlet nodes: traces and state
    bitwise against the oracle."""
    M, N, P, n_steps = 4097, 8, 64, 300
    say("many-receivers", dtype)
    plan = rs.Plan(M, N, P, dtype=dtype)
    assert plan.info["fused"] == 1
    lay = lay_of(plan)
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n_steps, seed=21)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    rec = np.array([0, 100, 101, 102, 103, 104, 105, 106, 107, 108, 109, 104, 2500,
                    M - 1], np.int64)
    ref, tr_ref, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n_steps,
                                 span=plan.span, state=st0, rec=rec)
    st = dev(st0, dtype)
    tr = rs.rswr_solve(plan, st, dev(fa, dtype), dev(fb, dtype), n_steps, receivers=rec)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_receivers_large_grid(dtype):
    """A grid of more tiles than two waves per SIMD (4542 tiles of 64x2), where
    a tile recording several receivers is launched once per group of four
    (small grids launch one copy per receiver): six receivers in one tile,
    one repeated, and others spread out; traces and state bitwise against
    the oracle."""
    M, N, P, n_steps = 2 ** 18 + 1, 64, 64, 120
    say("receivers-large-grid", dtype)
    plan = rs.Plan(M, N, P, tile=(64, 2), dtype=dtype)
    assert plan.info["fused"] == 1 and plan.info["n_tiles"] > 2 * 1024
    lay = lay_of(plan)
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n_steps, seed=23)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    rec = np.array([7, 50000, 50001, 50002, 50003, 50001, 50004, 131072, M - 2], np.int64)
    ref, tr_ref, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n_steps,
                                 span=plan.span, state=st0, rec=rec)
    st = dev(st0, dtype)
    tr = rs.rswr_solve(plan, st, dev(fa, dtype), dev(fb, dtype), n_steps, receivers=rec)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)
