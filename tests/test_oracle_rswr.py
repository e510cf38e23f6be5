"""Pins of the oracle's RSWR (Sec. 2.2-2.6 and Sec. 3 of the paper).

The method reaches the single-domain solution when every span stays inside
the light cone of the overlap (Decomposition Theorem, Sec. 2.2; Prediction
Validation Theorem, Sec. 2.4; Sec. 3 for N > 2).  So the oracle's RSWR is
pinned to the oracle's single-domain solve, which is itself pinned to
d'Alembert (test_oracle_single.py), and the span rule is pinned from both
sides: exact at the cone limit, wrong one step beyond it.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rel_l2(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)


def busy_problem(M, n_steps, seed=0):
    """Non-zero smooth state and both ends driven: every overlap sees signal
    from the first level on."""
    g = np.random.default_rng(seed)
    st = workloads.smooth_state(M, g, shift=2e-3)
    t = np.arange(n_steps + 1) * 0.9 / (M - 1)
    fa = np.sin(2 * np.pi * 7 * t) + 0.3
    fb = np.cos(2 * np.pi * 5 * t)
    return st, fa, fb


def test_golden_layout():
    gold = json.load(open(os.path.join(GOLD, "layout_1001_N2_P20.json")))
    lay = oracle.layout(gold["M"], gold["N"], gold["P"])
    assert list(lay.lo) == gold["lo"] and list(lay.hi) == gold["hi"]
    assert list(lay.own_lo) == gold["own_lo"] and list(lay.own_hi) == gold["own_hi"]
    assert lay.span_cone == gold["span_cone"]


def test_golden_span_table():
    gold = json.load(open(os.path.join(GOLD, "span_table.json")))
    num, den = gold["courant"]
    for P, S in gold["rows"]:
        assert oracle.span_paper(P, num / den, (num, den)) == S
        assert oracle.span_paper(P, num / den) == S


def test_config1_rswr_equals_single():
    prob = workloads.config1(np.float64)
    lay = oracle.layout(prob.M, prob.N, prob.P)
    S = min(lay.span_cone, oracle.span_paper(prob.P, prob.lam, prob.courant_frac))
    assert S == 11
    fa, fb = prob.sources()
    rec = [0, 100, 489, 490, 500, 510, 511, 999, 1000]
    st_r, tr_r, spans = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, prob.n_steps,
                                    span=S, rec=rec)
    st_s, tr_s = oracle.single(prob.M, prob.lam, prob.dx, fa, fb, prob.n_steps, rec=rec)
    assert len(spans) == 182 and spans[-1] == 2000 - 181 * 11
    assert rel_l2(st_r, st_s) <= 1e-12
    assert rel_l2(tr_r, tr_s) <= 1e-12
    # the wave has crossed the interface and come back
    assert np.abs(st_s[1]).max() > 1e-3 and np.abs(tr_s[6]).max() > 0.1


def test_config1_fp32_rswr_as_accurate_as_fp32_single():
    """In FP32 the flux/ghost exchange rounds differently from the plain
    stencil (q*r is not exactly 1), so RSWR and the single-domain solve part
    at the level of FP32 rounding.  Measured against FP64 the two FP32 runs
    must be equally accurate."""
    p64 = workloads.config1(np.float64)
    p32 = workloads.config1(np.float32)
    lay = oracle.layout(p64.M, p64.N, p64.P)
    rec = [100, 490, 500, 510, 999]
    ref, tr_ref = oracle.single(p64.M, p64.lam, p64.dx, *p64.sources(), p64.n_steps,
                                rec=rec)
    s32, tr_s32 = oracle.single(p32.M, p32.lam, p32.dx, *p32.sources(), p32.n_steps,
                                rec=rec)
    r32, tr_r32, _ = oracle.rswr(lay, p32.lam, p32.dx, *p32.sources(), p32.n_steps,
                                 span=11, rec=rec)
    e_single = rel_l2(tr_s32, tr_ref)
    e_rswr = rel_l2(tr_r32, tr_ref)
    assert 1e-7 < e_single < 1e-4
    assert e_rswr <= 2.0 * e_single, (e_rswr, e_single)
    assert rel_l2(r32, ref) <= 2.0 * rel_l2(s32, ref) + 1e-7


@pytest.mark.parametrize("N,P", [(2, 2), (3, 8), (5, 20), (10, 20), (7, 12)])
def test_rswr_equals_single_any_span_inside_cone(N, P):
    M, n_steps = 401, 700
    st0, fa, fb = busy_problem(M, n_steps, seed=N * 100 + P)
    lay = oracle.layout(M, N, P)
    cone = lay.span_cone
    ref, _ = oracle.single(M, 0.9, 1.0 / (M - 1), fa, fb, n_steps, state=st0)
    for S in sorted({1, max(1, cone // 2), cone}):
        st, _, _ = oracle.rswr(lay, 0.9, 1.0 / (M - 1), fa, fb, n_steps, span=S,
                               state=st0)
        assert rel_l2(st, ref) <= 1e-12, (S, cone)


@pytest.mark.parametrize("N,P", [(2, 20), (4, 16), (20, 20)])
def test_span_one_beyond_cone_deviates(N, P):
    M, n_steps = 301, 500
    st0, fa, fb = busy_problem(M, n_steps, seed=7)
    lay = oracle.layout(M, N, P)
    cone = lay.span_cone
    if N == 20:
        assert cone == 15  # cores of 15 nodes are narrower than the overlap
    ref, _ = oracle.single(M, 0.9, 1.0 / (M - 1), fa, fb, n_steps, state=st0)
    good, _, _ = oracle.rswr(lay, 0.9, 1.0 / (M - 1), fa, fb, n_steps, span=cone,
                             state=st0)
    bad, _, _ = oracle.rswr(lay, 0.9, 1.0 / (M - 1), fa, fb, n_steps, span=cone + 1,
                            state=st0)
    assert rel_l2(good, ref) <= 1e-12
    assert rel_l2(bad, ref) > 1e-6


def test_one_window_is_bitwise_single():
    M, n_steps = 257, 400
    st0, fa, fb = busy_problem(M, n_steps)
    lay = oracle.layout(M, 1, 2)
    ref, tr_ref = oracle.single(M, 0.9, 1 / (M - 1), fa, fb, n_steps, state=st0,
                                rec=[3, 100])
    for S in (1, 17, n_steps):
        st, tr, _ = oracle.rswr(lay, 0.9, 1 / (M - 1), fa, fb, n_steps, span=S,
                                state=st0, rec=[3, 100])
        assert np.array_equal(st, ref) and np.array_equal(tr, tr_ref)


def test_explicit_uneven_layout():
    M, n_steps = 400, 600
    st0, fa, fb = busy_problem(M, n_steps, seed=3)
    lo = [0, 90, 200, 260]
    hi = [110, 230, 290, 399]
    lay = oracle.explicit_layout(M, lo, hi)
    cone = lay.span_cone
    assert cone == 20  # hi_0 - lo_1 = 20 is the narrowest input/output gap
    ref, _ = oracle.single(M, 0.9, 1 / (M - 1), fa, fb, n_steps, state=st0)
    st, _, _ = oracle.rswr(lay, 0.9, 1 / (M - 1), fa, fb, n_steps, span=cone,
                           state=st0)
    assert rel_l2(st, ref) <= 1e-12
    bad, _, _ = oracle.rswr(lay, 0.9, 1 / (M - 1), fa, fb, n_steps, span=cone + 1,
                            state=st0)
    assert rel_l2(bad, ref) > 1e-6


def test_prediction_validation_theorem():
    """The zero-flux prediction's output flux equals the single-domain flux
    for exactly span_cone levels (Prediction Validation Theorem, Sec. 2.4)."""
    M, N, P = 301, 3, 20
    st0, fa, fb = busy_problem(M, 100, seed=11)
    lay = oracle.layout(M, N, P)
    cone = lay.span_cone
    shat = cone + 5
    dx = 1 / (M - 1)
    flux = oracle.predict(lay, 0.9, dx, fa, fb, 0, shat, st0)
    outs = []
    for i in range(N - 1):
        outs += [(i, 0, lay.lo[i + 1]), (i, 1, lay.hi[i])]
    nodes = sorted({o + d for _, _, o in outs for d in (-1, 1)})
    _, tr = oracle.single(M, 0.9, dx, fa, fb, shat, state=st0, rec=nodes)
    lev = np.hstack([st0[1][nodes][:, None], tr])  # levels 0..shat
    r = 1.0 / (2 * dx)
    for i, side, o in outs:
        true = (lev[nodes.index(o + 1)] - lev[nodes.index(o - 1)]) * r
        f = flux[i, side]
        assert np.array_equal(f[:cone], true[:cone]), (i, side)
        assert f[cone] != true[cone], (i, side)


def test_quiet_select_is_exact_and_grows():
    prob = workloads.config1()
    lay = oracle.layout(prob.M, prob.N, prob.P)
    fa, fb = prob.sources()
    ref, tr_ref = oracle.single(prob.M, prob.lam, prob.dx, fa, fb, prob.n_steps,
                                rec=[250, 500, 750])
    st, tr, spans = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, prob.n_steps,
                                mode=oracle.QUIET, beta=0.1, rec=[250, 500, 750])
    assert rel_l2(st, ref) <= 1e-12 and rel_l2(tr, tr_ref) <= 1e-12
    cone = lay.span_cone
    assert spans.max() > cone and spans.max() <= 2 * cone
    assert len(spans) < 2000 / 11


def test_paper_select_exact_on_generic_data():
    """On the asymmetric pulse problem the literal rule of Sec. 2.4 picks
    spans beyond the cone only while the overlap is quiet, and stays exact."""
    prob = workloads.config1()
    lay = oracle.layout(prob.M, prob.N, prob.P)
    fa, fb = prob.sources()
    ref, _ = oracle.single(prob.M, prob.lam, prob.dx, fa, fb, prob.n_steps)
    st, _, spans = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, prob.n_steps,
                               mode=oracle.PAPER)
    assert spans.max() > lay.span_cone
    assert rel_l2(st, ref) <= 1e-12


def test_paper_select_unsafe_under_mirror_symmetry():
    """The literal rule (largest agreement time over the overlap nodes) is
    fooled by data that is mirror-symmetric about the overlap midpoint: both
    predictions are mirror images, so they agree bitwise at the midpoint
    while both are wrong.  Negative pin of the paper's own rule; the derived
    QUIET rule stays exact on the same data."""
    M, n = 1001, 400
    dx = 1 / (M - 1)
    x = np.arange(M) * dx
    st = np.zeros((2, M))
    st[1] = np.exp(-((x - 0.5) / 0.03) ** 2)
    st[1, 501:] = st[1, 499::-1]  # exact mirror about node 500
    st[0] = st[1]
    z = np.zeros(n + 1)
    lay = oracle.layout(M, 2, 20)
    ref, _ = oracle.single(M, 0.9, dx, z, z, n, state=st)
    bad, _, spans = oracle.rswr(lay, 0.9, dx, z, z, n, mode=oracle.PAPER, state=st)
    assert spans.max() > lay.span_cone
    assert rel_l2(bad, ref) > 1e-3
    worse, _, _ = oracle.rswr(lay, 0.9, dx, z, z, n, mode=oracle.PAPER, state=st,
                              tau_hat=60)
    assert rel_l2(worse, ref) > 0.1
    good, _, _ = oracle.rswr(lay, 0.9, dx, z, z, n, mode=oracle.QUIET, state=st)
    assert rel_l2(good, ref) <= 1e-12


def test_update_windows_subset_matches_full():
    M, N, P = 500, 5, 20
    st0, fa, fb = busy_problem(M, 50, seed=5)
    lay = oracle.layout(M, N, P)
    dx = 1 / (M - 1)
    S = lay.span_cone
    flux = oracle.predict(lay, 0.9, dx, fa, fb, 0, S, st0)
    full, _ = oracle.update(lay, 0.9, dx, fa, fb, 0, S, st0, flux)
    part, _ = oracle.update(lay, 0.9, dx, fa, fb, 0, S, st0, flux, windows=[1, 3])
    for w in (1, 3):
        sl = slice(lay.own_lo[w], lay.own_hi[w] + 1)
        assert np.array_equal(part[:, sl], full[:, sl])


def test_rswr_many_equals_each_problem():
    """The batch entry point runs each problem's own span loop: the states
    equal oracle.rswr of every problem alone, bitwise, in both precisions."""
    cases = [(601, 4, 32, 300, 1.0), (257, 2, 16, 137, 0.7), (1025, 8, 40, 211, 1.6)]
    for dtype in (np.float64, np.float32):
        lays, lams, dxs, fas, fbs, ns, spans = [], [], [], [], [], [], []
        for M, N, P, n, a in cases:
            lay = oracle.layout(M, N, P)
            lam, dx = 0.9, 1.0 / (M - 1)
            t = np.arange(n + 1) * lam * dx / a
            fas.append(np.exp(-((t - 40 * dx / a) / (8 * dx / a)) ** 2).astype(dtype))
            fbs.append((0.2 * np.sin(2 * np.pi * t / t[-1])).astype(dtype))
            lays.append(lay)
            lams.append(lam)
            dxs.append(dx)
            ns.append(n)
            spans.append(min(lay.span_cone, oracle.span_paper(P, lam, (9, 10))))
        out = oracle.rswr_many(lays, lams, dxs, fas, fbs, ns, spans)
        for i in range(len(cases)):
            ref, _, _ = oracle.rswr(lays[i], lams[i], dxs[i], fas[i], fbs[i], ns[i],
                                    span=spans[i])
            assert out[i].dtype == dtype
            assert np.array_equal(out[i], ref), (dtype, i)
