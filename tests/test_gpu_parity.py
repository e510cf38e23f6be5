"""GPU parity of the RSWR hot path against the CPU oracle.

Both sides run the same operation sequence, so the predict trapezoid equals
the oracle's whole-window prediction and the register-tiled update equals the
oracle's literal update bit for bit; the tests assert bitwise equality there
and the benchmark spec's tolerances (1e-12 relative in FP64, 1e-5 in FP32) where a
different algorithm is compared (RSWR against the single-domain solve)."""
import os

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


def rel_l2(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)


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


CASES = [
    # (M, N, P, windows, tile)
    (1001, 2, 20, None, None),
    (4097, 8, 64, None, None),
    (301, 20, 20, None, None),          # cores narrower than the overlap
    (101, 2, 0, ([0, 5], [30, 100]), None),  # trapezoid reaches node 0
    (6000, 3, 40, None, (64, 8)),        # several tiles per window
    (3001, 5, 16, None, (128, 8)),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_predict_bitwise(dtype, case):
    M, N, P, win, tile = CASES[case]
    say("predict", dtype, M, N, P, win, tile)
    plan = rs.Plan(M, N, P, windows=win, tile=tile, dtype=dtype)
    lay = lay_of(plan)
    S = plan.span
    st, fa, fb = busy(M, 50 + S, seed=case)
    n0 = 7
    npdt = NP[dtype]
    ref = oracle.predict(lay, plan.info["lambda"], plan.info["dx"], fa.astype(npdt),
                         fb.astype(npdt), n0, S, st.astype(npdt))
    fl = rs.rswr_predict(plan, dev(st, dtype), dev(fa, dtype), dev(fb, dtype), n0, S)
    got = host(fl)[:, :, :S]
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_predict_every_frame_width(dtype):
    """The predict runs on register frames of 2..5 nodes per lane for spans up
    to 159 levels and on the LDS trapezoid beyond: spans on both sides of
    every width change, reaching the predicting windows' input ghosts and
    node 0 / M-1, bitwise against the oracle's whole-window prediction."""
    M, N, P = 1201, 8, 128
    say("predict-widths", dtype)
    plan = rs.Plan(M, N, P, span_mode=rs.QUIET, dtype=dtype)
    lay = lay_of(plan)
    cap = plan.info["span"]
    assert cap >= 200, cap
    npdt = NP[dtype]
    st, fa, fb = busy(M, cap + 20, seed=11)
    st, fa, fb = st.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    st_d, fa_d, fb_d = dev(st, dtype), dev(fa, dtype), dev(fb, dtype)
    n0 = 9
    for shat in (1, 2, 40, 63, 64, 95, 96, 127, 128, 159, 160, 200, cap):
        ref = oracle.predict(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n0, shat, st)
        fl = rs.rswr_predict(plan, st_d, fa_d, fb_d, n0, shat)
        got = host(fl)[:, :, :shat]
        assert np.array_equal(got, ref[:, :, :shat]), shat


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_predict_beyond_cone_reaches_window_ends(dtype):
    """QUIET plans predict up to twice the light-cone span; the trapezoid then
    reaches the windows' own input boundaries (zero-flux ghosts)."""
    M, N, P = 1201, 4, 24
    say("predict-quiet", dtype)
    plan = rs.Plan(M, N, P, span_mode=rs.QUIET, dtype=dtype)
    lay = lay_of(plan)
    shat = plan.info["span"]
    assert shat == 2 * plan.info["span_cone"]
    st, fa, fb = busy(M, shat + 5, seed=3)
    npdt = NP[dtype]
    ref = oracle.predict(lay, plan.info["lambda"], plan.info["dx"], fa.astype(npdt),
                         fb.astype(npdt), 0, shat, st.astype(npdt))
    fl = rs.rswr_predict(plan, dev(st, dtype), dev(fa, dtype), dev(fb, dtype), 0, shat)
    assert np.array_equal(host(fl)[:, :, :shat], ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_update_bitwise(dtype, case):
    M, N, P, win, tile = CASES[case]
    plan = rs.Plan(M, N, P, windows=win, tile=tile, dtype=dtype)
    lay = lay_of(plan)
    npdt = NP[dtype]
    for S in sorted({1, max(1, plan.span // 2), plan.span}):
        say("update", dtype, M, N, P, win, tile, "S", S)
        st, fa, fb = busy(M, 40 + S, seed=case + S)
        st, fa, fb = st.astype(npdt), fa.astype(npdt), fb.astype(npdt)
        n0 = 3
        flux = oracle.predict(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n0, S, st,
                              ld=plan.flux_ld)
        ref, _ = oracle.update(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n0, S,
                               st, flux)
        out = rs.rswr_update(plan, dev(st, dtype), dev(fa, dtype), dev(fb, dtype), n0,
                             dev(flux, dtype), span=S)
        assert np.array_equal(host(out), ref), S


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_update_general_tiles_bitwise(dtype):
    """Spans up to twice the light-cone limit (QUIET plans) over windows
    narrower than that reach both window ends: general tiles with the left
    input ghost and node 0 strictly inside the register region."""
    M, N, P = 301, 20, 20
    plan = rs.Plan(M, N, P, span_mode=rs.QUIET, tile=(64, 8), dtype=dtype)
    assert plan.tiles()[:, 7].sum() > 0
    lay = lay_of(plan)
    npdt = NP[dtype]
    for S in (plan.info["span_cone"], plan.info["span"]):
        say("update-general", dtype, "S", S)
        st, fa, fb = busy(M, 40 + S, seed=S)
        st, fa, fb = st.astype(npdt), fa.astype(npdt), fb.astype(npdt)
        flux = oracle.predict(lay, plan.info["lambda"], plan.info["dx"], fa, fb, 2, S, st,
                              ld=plan.flux_ld)
        ref, _ = oracle.update(lay, plan.info["lambda"], plan.info["dx"], fa, fb, 2, S, st,
                               flux)
        out = rs.rswr_update(plan, dev(st, dtype), dev(fa, dtype), dev(fb, dtype), 2,
                             dev(flux, dtype), span=S)
        assert np.array_equal(host(out), ref), S


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_quiet_loop_matches_oracle(dtype):
    """predict -> select (QUIET, on the device) -> update, span by span; the
    chosen spans and the state equal the oracle's adaptive loop."""
    prob = workloads.config1(NP[dtype])
    say("quiet-loop", dtype)
    plan = rs.Plan(prob.M, prob.N, prob.P, span_mode=rs.QUIET, dtype=dtype)
    lay = lay_of(plan)
    fa, fb = prob.sources()
    ref, _, spans_ref = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, prob.n_steps,
                                    mode=oracle.QUIET)
    cap = plan.info["span"]
    st = torch.zeros(2, prob.M, dtype=dtype, device=DEV)
    other = torch.empty_like(st)
    fa_d, fb_d = dev(fa, dtype), dev(fb, dtype)
    flux = plan.flux_buffer()
    sd = torch.zeros(1, dtype=torch.int32, device=DEV)
    n0, S_prev, spans = 0, 0, []
    while n0 < prob.n_steps:
        shat = plan.info["span_cone"] if not spans else int(np.ceil(1.1 * S_prev))
        shat = min(shat, cap, prob.n_steps - n0)
        rs.rswr_predict(plan, st, fa_d, fb_d, n0, shat, flux)
        rs.rswr_select(plan, flux, shat, sd)
        rs.rswr_update(plan, st, fa_d, fb_d, n0, flux, span_dev=sd, out=other)
        S = int(sd.item())
        spans.append(S)
        st, other = other, st
        n0 += S
        S_prev = S
    assert spans == list(spans_ref)
    assert np.array_equal(host(st), ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_select_fixed(dtype):
    plan = rs.Plan(1001, 2, 20, dtype=dtype)
    flux = plan.flux_buffer()
    for shat, want in ((5, 5), (11, 11)):
        assert int(rs.rswr_select(plan, flux, shat).item()) == want


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_solve_config1_bitwise(dtype):
    """The N=2 pulse case: 1001 nodes, overlap 20, span 11, 2000 steps."""
    prob = workloads.config1(NP[dtype])
    say("solve-config1", dtype)
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=dtype)
    assert plan.span == 11
    lay = lay_of(plan)
    fa, fb = prob.sources()
    rec = [0, 100, 489, 490, 500, 510, 511, 999, 1000]
    ref, tr_ref, spans = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, prob.n_steps, span=11,
                                     rec=rec)
    st = torch.zeros(2, prob.M, dtype=dtype, device=DEV)
    tr = rs.rswr_solve(plan, st, dev(fa, dtype), dev(fb, dtype), prob.n_steps, receivers=rec)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)
    if dtype == torch.float64:
        s1, t1 = oracle.single(prob.M, prob.lam, prob.dx, fa, fb, prob.n_steps, rec=rec)
        assert rel_l2(host(st), s1) <= 1e-12 and rel_l2(host(tr), t1) <= 1e-12


SOLVE_CASES = [
    # M, N, P, windows, tile, n_steps, n0, span
    (1001, 2, 20, None, None, 200, 0, 0),
    (1001, 2, 20, None, None, 211, 5, 7),      # odd span count, restart level
    (4097, 8, 64, None, None, 400, 0, 0),
    (301, 20, 20, None, None, 333, 0, 0),
    (257, 1, 2, None, None, 300, 0, 40),       # one window: plain leapfrog
    (400, 4, 0, ([0, 90, 200, 260], [110, 230, 290, 399]), None, 250, 0, 0),
    (6000, 3, 40, None, (64, 8), 190, 0, 0),
    (20001, 16, 64, None, (256, 16), 177, 2, 0),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(SOLVE_CASES)))
def test_solve_bitwise(dtype, case):
    M, N, P, win, tile, n_steps, n0, span = SOLVE_CASES[case]
    say("solve", dtype, SOLVE_CASES[case])
    plan = rs.Plan(M, N, P, windows=win, tile=tile, span=span, dtype=dtype)
    lay = lay_of(plan)
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n0 + n_steps, seed=case)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    g = np.random.default_rng(case)
    rec = np.unique(np.concatenate([[0, M - 1], g.integers(0, M, 6)]))
    ref, tr_ref, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb,
                                 n_steps, span=plan.span, state=st0, n0=n0, rec=rec)
    st = dev(st0, dtype)
    tr = rs.rswr_solve(plan, st, dev(fa, dtype), dev(fb, dtype), n_steps, n0=n0,
                       receivers=rec)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    assert np.array_equal(host(tr), tr_ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_solve_graph_replay_and_checkpoints(dtype):
    """Replaying the recorded graph gives the eager result, every time; the
    checkpoints are the states at the span boundaries."""
    M, N, P, n_steps = 4097, 8, 64, 300
    say("graph", dtype)
    plan = rs.Plan(M, N, P, dtype=dtype)
    lay = lay_of(plan)
    npdt = NP[dtype]
    st0, fa, fb = busy(M, n_steps, seed=9)
    st0, fa, fb = st0.astype(npdt), fa.astype(npdt), fb.astype(npdt)
    fa_d, fb_d = dev(fa, dtype), dev(fb, dtype)
    ws = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device=DEV)
    ref, _, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb, n_steps,
                            span=plan.span, state=st0)
    os.environ["RSWR_NO_GRAPH"] = "1"
    try:
        st_e = dev(st0, dtype)
        rs.rswr_solve(plan, st_e, fa_d, fb_d, n_steps, workspace=ws)
        torch.cuda.synchronize()
    finally:
        del os.environ["RSWR_NO_GRAPH"]
    assert np.array_equal(host(st_e), ref)
    st = dev(st0, dtype)
    for rep in range(4):
        st.copy_(dev(st0, dtype))
        torch.cuda.synchronize()
        rs.rswr_solve(plan, st, fa_d, fb_d, n_steps, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(host(st), ref), rep
    K = plan.n_spans(n_steps)
    ck = plan.checkpoint_buffer(n_steps)
    st = dev(st0, dtype)
    rs.rswr_solve(plan, st, fa_d, fb_d, n_steps, checkpoints=ck, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(host(st), ref)
    ckh = host(plan.checkpoint_states(ck, n_steps))
    assert np.array_equal(ckh[0], st0)
    for k in (1, K // 2, K):
        nk = min(k * plan.span, n_steps)
        r_k, _, _ = oracle.rswr(lay, plan.info["lambda"], plan.info["dx"], fa, fb, nk,
                                span=plan.span, state=st0)
        assert np.array_equal(ckh[k], r_k), k


def test_plain_2p20_fp64_sampled():
    """Full-size plain case in FP64: 2^20 nodes, 64 windows, overlap 64,
    10^4 steps, Ricker source; sampled nodes and receiver traces against the
    single-domain solve (1e-12 relative)."""
    prob = workloads.config2(np.float64)
    say("plain-2^20-fp64")
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float64)
    assert plan.span == 35
    fa, fb = prob.sources()
    rec = np.array([1, 1000, 4000, 8000, 16000, 500000], np.int64)
    st = torch.zeros(2, prob.M, dtype=torch.float64, device=DEV)
    tr = rs.rswr_solve(plan, st, dev(fa, torch.float64), dev(fb, torch.float64),
                       prob.n_steps, receivers=rec)
    got = host(st)
    nodes = np.concatenate([np.arange(0, 9600, 97), [20000, 400000, prob.M - 2,
                                                      prob.M - 1]])
    ref = oracle.point_values(prob.M, prob.lam, prob.dx, fa, fb, prob.n_steps,
                              prob.state0(), nodes)
    scale = np.abs(ref).max()
    assert scale > 0.1 and np.count_nonzero(ref) > 100
    assert np.abs(got[:, nodes] - ref).max() <= 1e-12 * scale
    # traces: from rest and driven at node 0 only, U^n_j = 0 for j >= n, so
    # cutting the domain at node n_steps + 1 changes no value before it
    Ms = prob.n_steps + 2
    keep = rec < Ms
    _, tr_ref = oracle.single(Ms, prob.lam, prob.dx, fa, np.zeros_like(fb), prob.n_steps,
                              rec=rec[keep])
    trh = host(tr)
    assert keep.sum() >= 4
    assert rel_l2(trh[keep], tr_ref) <= 1e-12
    assert np.all(trh[~keep] == 0.0)


def test_large_fp32_span_bitwise_and_fp64_spot():
    """The 2^24-node FP32 case (4096 windows, overlap 64, span 35) in the
    launch shape the benchmark times: one span from a smooth state, sampled
    windows bitwise against the oracle's literal predict + update in FP32, and
    within 1e-5 (relative) of the same span in FP64."""
    prob = workloads.config5(np.float32)
    say("large-2^24-fp32-span")
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32)
    assert plan.span == 35
    lay = lay_of(plan)
    g = np.random.default_rng(77)
    st64 = workloads.smooth_state(prob.M, g, shift=prob.lam * prob.dx)
    fa, fb = prob.sources()
    n0 = 1000
    S = plan.span
    st32 = st64.astype(np.float32)
    st_d = dev(st32, torch.float32)
    fa_d, fb_d = dev(fa, torch.float32), dev(fb, torch.float32)
    flux = rs.rswr_predict(plan, st_d, fa_d, fb_d, n0, S)
    out = rs.rswr_update(plan, st_d, fa_d, fb_d, n0, flux, span=S)
    got_flux = host(flux)[:, :, :S]
    got = host(out)
    ref_flux = oracle.predict(lay, prob.lam, prob.dx, fa, fb, n0, S, st32,
                              ld=plan.flux_ld)
    assert np.array_equal(got_flux, ref_flux[:, :, :S])
    wins = [0, 1, 2, 777, 2048, 4000, prob.N - 2, prob.N - 1]
    ref, _ = oracle.update(lay, prob.lam, prob.dx, fa, fb, n0, S, st32, ref_flux,
                           windows=wins)
    f64 = oracle.predict(lay, prob.lam, prob.dx, fa.astype(np.float64),
                         fb.astype(np.float64), n0, S, st32.astype(np.float64))
    ref64, _ = oracle.update(lay, prob.lam, prob.dx, fa.astype(np.float64),
                             fb.astype(np.float64), n0, S, st32.astype(np.float64), f64,
                             windows=wins)
    for w in wins:
        sl = slice(lay.own_lo[w], lay.own_hi[w] + 1)
        assert np.array_equal(got[:, sl], ref[:, sl]), w
        assert rel_l2(got[:, sl], ref64[:, sl]) <= 1e-5, w
