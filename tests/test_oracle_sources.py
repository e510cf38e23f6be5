"""Pins of the oracle's interior point sources (the pulse sources of the
paper's experiments, Sec. 4): the step from level n to n+1 adds amp[q, n]
at node nodes[q] after the leapfrog update.

* At Courant number 1 (c2 = 1, k = 0) the leapfrog is exact for the wave
  equation and its response to a unit impulse is the discrete d'Alembert
  solution: m levels after the impulse level it is 1 on the nodes
  j-m, j-m+2, ..., j+m and 0 elsewhere (integers, so exact in floating
  point).  Superposition of two impulses is checked against the sum.
* One and two steps from rest at general lambda: the impulse itself, then
  k a at the node and c2 a at its neighbours, written out by hand.
* RSWR carries the sources through predict and update: with sources next
  to output nodes, in overlaps and on input ends its result equals the
  single-domain solve to the rounding of the ghost (FP64), the predicted
  fluxes change with the sources, and a prediction that leaves them out
  breaks the result (so the equality is not vacuous).
"""
import numpy as np
import pytest

import oracle
import workloads

DT = [np.float64, np.float32]


def impulse_pattern(M, j, n_imp, n_levels):
    """Levels 1..n_levels of the Courant-1 response to a unit impulse added
    by the step from level n_imp to n_imp + 1 at node j (no boundary hit)."""
    out = np.zeros((n_levels, M))
    for L in range(n_imp + 1, n_levels + 1):
        m = L - n_imp - 1
        out[L - 1, j - m:j + m + 1:2] = 1.0
    return out


@pytest.mark.parametrize("dtype", DT)
def test_courant_one_impulse_is_discrete_dalembert(dtype):
    M, j, n_imp, n = 301, 140, 5, 100
    amp = np.zeros((1, n + 1))
    amp[0, n_imp] = 1.0
    fa = np.zeros(n + 1, dtype)
    _, tr = oracle.single(M, 1.0, 1.0 / (M - 1), fa, fa, n, rec=np.arange(M),
                          src=([j], amp.astype(dtype)))
    want = impulse_pattern(M, j, n_imp, n)
    assert np.array_equal(tr.T, want.astype(dtype))


@pytest.mark.parametrize("dtype", DT)
def test_courant_one_superposition(dtype):
    M, n = 401, 120
    amp = np.zeros((2, n + 1))
    amp[0, 3] = 1.0
    amp[1, 20] = 2.0
    fa = np.zeros(n + 1, dtype)
    _, tr = oracle.single(M, 1.0, 1.0 / (M - 1), fa, fa, n, rec=np.arange(M),
                          src=([150, 190], amp.astype(dtype)))
    want = impulse_pattern(M, 150, 3, n) + 2 * impulse_pattern(M, 190, 20, n)
    assert np.array_equal(tr.T, want.astype(dtype))


@pytest.mark.parametrize("dtype", DT)
def test_first_two_steps_by_hand(dtype):
    M, j, lam = 51, 20, 0.9
    a = dtype(0.37)
    amp = np.zeros((1, 3), dtype)
    amp[0, 0] = a
    fa = np.zeros(3, dtype)
    _, tr = oracle.single(M, lam, 1.0 / (M - 1), fa, fa, 2, rec=[j - 1, j, j + 1],
                          src=([j], amp))
    c2 = dtype(lam * lam)
    k = dtype(2.0 - 2.0 * lam * lam)
    assert tr[1, 0] == a and tr[0, 0] == 0 and tr[2, 0] == 0
    assert tr[1, 1] == dtype(k * a)
    assert tr[0, 1] == dtype(c2 * a) and tr[2, 1] == dtype(c2 * a)


def test_dirichlet_nodes_take_no_source():
    M, n = 41, 10
    amp = np.ones((2, n + 1))
    fa = np.zeros(n + 1)
    st, _ = oracle.single(M, 0.9, 1.0 / (M - 1), fa, fa, n, src=([0, M - 1], amp))
    assert not st.any()


LAYOUTS = [
    # M, N, P, sources placed relative to the layout
    (1001, 2, 20),
    (2001, 3, 40),
    (3001, 10, 64),
]


def placed_sources(lay, g, n_steps):
    """Sources on every output node and next to it, on input ends, inside
    overlaps, on node 1 and M-2, a repeated node, and a few at random."""
    M = lay.M
    nodes = [1, M - 2]
    for i in range(lay.N - 1):
        o_l, o_r = int(lay.lo[i + 1]), int(lay.hi[i])  # output nodes / input ends
        nodes += [o_l, o_l + 1, o_l - 3, o_r, o_r - 1, o_r + 2, (o_l + o_r) // 2]
    nodes += list(g.integers(1, M - 1, 6))
    nodes.append(nodes[2])
    nodes = np.array(nodes, np.int64)
    amp = g.standard_normal((len(nodes), n_steps + 1)) * 0.05
    return nodes, amp


def rel_l2(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)


def source_problem(case, n_steps=150):
    M, N, P = LAYOUTS[case]
    lay = oracle.layout(M, N, P)
    g = np.random.default_rng(100 + case)
    nodes, amp = placed_sources(lay, g, n_steps)
    st0 = workloads.smooth_state(M, g)
    t = np.arange(n_steps + 1) / n_steps
    fa, fb = np.sin(7 * t), np.cos(5 * t)
    S = min(lay.span_cone, oracle.span_paper(P, 0.9))
    return lay, nodes, amp, st0, fa, fb, S


@pytest.mark.parametrize("case", range(len(LAYOUTS)))
def test_rswr_with_sources_equals_single_domain(case):
    """FP64: RSWR reaches the single-domain solution with sources (to the
    rounding of the ghost, q r != 1 in floating point)."""
    lay, nodes, amp, st0, fa, fb, S = source_problem(case)
    n_steps, lam, dx = amp.shape[1] - 1, 0.9, 1.0 / (lay.M - 1)
    ref, tr_ref = oracle.single(lay.M, lam, dx, fa, fb, n_steps, state=st0, rec=nodes,
                                src=(nodes, amp))
    got, tr, _ = oracle.rswr(lay, lam, dx, fa, fb, n_steps, span=S, state=st0,
                             rec=nodes, src=(nodes, amp))
    assert rel_l2(got, ref) <= 1e-12
    assert rel_l2(tr, tr_ref) <= 1e-12
    # the sources do reach the predicted output fluxes ...
    f0 = oracle.predict(lay, lam, dx, fa, fb, 0, S, st0)
    f1 = oracle.predict(lay, lam, dx, fa, fb, 0, S, st0, src=(nodes, amp))
    assert not np.array_equal(f0, f1)
    # ... and a prediction without them breaks the result
    st = st0.copy()
    for n0 in range(0, n_steps, S):
        Sk = min(S, n_steps - n0)
        fl = oracle.predict(lay, lam, dx, fa, fb, n0, Sk, st)
        st, _ = oracle.update(lay, lam, dx, fa, fb, n0, Sk, st, fl, src=(nodes, amp))
    assert rel_l2(st, ref) > 1e-6


@pytest.mark.parametrize("case", range(len(LAYOUTS)))
def test_rswr_with_sources_fp32_as_accurate_as_single(case):
    lay, nodes, amp, st0, fa, fb, S = source_problem(case)
    n_steps, lam, dx = amp.shape[1] - 1, 0.9, 1.0 / (lay.M - 1)
    ref, _ = oracle.single(lay.M, lam, dx, fa, fb, n_steps, state=st0, src=(nodes, amp))
    f32 = np.float32
    src32 = (nodes, amp.astype(f32))
    s32, _ = oracle.single(lay.M, lam, dx, fa.astype(f32), fb.astype(f32), n_steps,
                           state=st0.astype(f32), src=src32)
    r32, _, _ = oracle.rswr(lay, lam, dx, fa.astype(f32), fb.astype(f32), n_steps,
                            span=S, state=st0.astype(f32), src=src32)
    assert rel_l2(r32, ref) <= 2.0 * rel_l2(s32, ref) + 1e-7


def test_pulse_source_recipe():
    g = workloads.rng(9)
    nodes, amp = workloads.pulse_sources(10001, 10, 2000, g)
    assert nodes.shape == (10,) and amp.shape == (10, 2001)
    assert nodes.min() >= 1 and nodes.max() <= 9999 and np.all(np.diff(nodes) > 0)
    assert 0.01 < np.abs(amp).max() < 1.0
