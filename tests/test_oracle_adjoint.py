"""Pins of the oracle's reverse-mode gradient of the receiver misfit
J = sum_r sum_n (U^n[j_r] - d_r^n)^2 with respect to the boundary source
samples f_A[n] and the leapfrog number lam = a dt / dx.

The traces are linear in (f_A, f_B) from rest, so the gradient is checked
against a brute-force Jacobian built from unit-impulse forward solves, the
dot-product identity <A df, w> = <df, A^T w>, causality zeros, and central
finite differences in lam.
"""
import numpy as np
import pytest

import oracle


def forward_traces(M, lam, dx, fa, fb, n_steps, rec):
    _, tr = oracle.single(M, lam, dx, fa, fb, n_steps, rec=rec)
    return tr


def misfit(M, lam, dx, fa, fb, n_steps, rec, d):
    tr = forward_traces(M, lam, dx, fa, fb, n_steps, rec)
    return float(np.sum((tr - d) ** 2)), tr


@pytest.fixture(scope="module")
def tiny():
    M, n_steps = 21, 60
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(3)
    fa = np.concatenate([[0.0], g.standard_normal(n_steps)])
    fb = np.concatenate([[0.0], 0.3 * g.standard_normal(n_steps)])
    rec = np.array([3, 10, 17], np.int64)
    d = g.standard_normal((len(rec), n_steps))
    return M, n_steps, dx, fa, fb, rec, d


def test_gradient_matches_bruteforce_jacobian(tiny):
    M, n_steps, dx, fa, fb, rec, d = tiny
    lam = 0.9
    J, tr = misfit(M, lam, dx, fa, fb, n_steps, rec, d)
    resid = 2.0 * (tr - d)
    ga, gb, _ = oracle.adjoint(M, lam, dx, fa, fb, n_steps, rec, resid, ck=5)
    z = np.zeros(n_steps + 1)
    for which, grad in (("a", ga), ("b", gb)):
        bf = np.zeros(n_steps + 1)
        for n in range(1, n_steps + 1):
            e = np.zeros(n_steps + 1)
            e[n] = 1.0
            col = forward_traces(M, lam, dx, e if which == "a" else z,
                                 z if which == "a" else e, n_steps, rec)
            bf[n] = np.sum(col * resid)
        assert grad[0] == 0.0
        assert np.abs(grad - bf).max() <= 1e-12 * np.abs(bf).max(), which


def test_dot_product_identity():
    M, n_steps = 201, 400
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(5)
    rec = np.sort(g.choice(np.arange(1, M - 1), 7, replace=False))
    w = g.standard_normal((len(rec), n_steps))
    df = np.concatenate([[0.0], g.standard_normal(n_steps)])
    z = np.zeros(n_steps + 1)
    Adf = forward_traces(M, 0.9, dx, df, z, n_steps, rec)
    ga, _, _ = oracle.adjoint(M, 0.9, dx, z, z, n_steps, rec, w)
    lhs = np.sum(Adf * w)
    rhs = np.sum(df * ga)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(Adf ** 2) * np.sum(w ** 2))


def test_causality_zeros():
    M, n_steps = 301, 500
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(8)
    rec = np.array([40, 120, 250], np.int64)
    w = g.standard_normal((3, n_steps))
    z = np.zeros(n_steps + 1)
    ga, _, _ = oracle.adjoint(M, 0.9, dx, z, z, n_steps, rec, w)
    cut = n_steps - rec.min()
    assert np.all(ga[cut + 1:] == 0.0)
    assert np.all(ga[1:cut + 1] != 0.0)


def test_lambda_gradient_central_difference():
    M, n_steps = 161, 700
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(9)
    t = np.arange(n_steps + 1) * 0.9 * dx
    fa = np.exp(-((t - 0.08) / 0.02) ** 2)
    fb = np.zeros_like(fa)
    rec = np.array([20, 77, 140], np.int64)
    d = forward_traces(M, 0.99, dx, fa, fb, n_steps, rec)  # "other speed" data
    lam = 0.9
    J0, tr = misfit(M, lam, dx, fa, fb, n_steps, rec, d)
    _, _, glam = oracle.adjoint(M, lam, dx, fa, fb, n_steps, rec, 2.0 * (tr - d))
    h = 1e-6
    Jp, _ = misfit(M, lam + h, dx, fa, fb, n_steps, rec, d)
    Jm, _ = misfit(M, lam - h, dx, fa, fb, n_steps, rec, d)
    fd = (Jp - Jm) / (2 * h)
    assert abs(glam) > 1e-3
    assert abs(fd - glam) <= 1e-6 * abs(glam)


def test_checkpoint_interval_does_not_change_result():
    M, n_steps = 101, 230
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(2)
    fa = np.concatenate([[0.0], g.standard_normal(n_steps)])
    fb = np.zeros(n_steps + 1)
    rec = np.array([5, 50], np.int64)
    w = g.standard_normal((2, n_steps))
    outs = [oracle.adjoint(M, 0.9, dx, fa, fb, n_steps, rec, w, ck=ck)
            for ck in (1, 7, 64, 1000)]
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[2] == outs[0][2]


def _levels(M, lam, dx, fa, fb, n_steps):
    """U^{-1} .. U^{n_steps} of the single-domain solve from rest, one
    oracle step at a time."""
    lev = [np.zeros(M), np.zeros(M)]
    st = np.zeros((2, M))
    for n in range(n_steps):
        st, _ = oracle.single(M, lam, dx, fa, fb, 1, state=st, n0=n)
        lev.append(st[1].copy())
    return lev  # lev[n + 1] = U^n


def test_lambda_terms_against_bruteforce_sensitivities(tiny):
    """W^n_j, the sensitivity of sum_r,t w[r,t] trace[r,t] to a unit change of
    U^n_j, taken by re-running the forward solve from the perturbed state
    (traces are affine in the state); then dJ/dlam = 2 lam sum W Lap(U^{n-1})
    and the magnitude sum 2 |lam| sum |W Lap(U^{n-1})| over interior nodes
    against the oracle's reverse mode."""
    M, n_steps, dx, fa, fb, rec, w = tiny
    lam = 0.9
    lev = _levels(M, lam, dx, fa, fb, n_steps)
    tot = tot_abs = 0.0
    for n in range(1, n_steps + 1):
        lap = np.zeros(M)
        u = lev[n]  # U^{n-1}
        lap[1:-1] = (u[:-2] + u[2:]) - 2.0 * u[1:-1]
        for j in range(1, M - 1):
            st = np.stack([lev[n], lev[n + 1]])  # U^{n-1}, U^n
            W = float(np.sum(w[:, n - 1] * (rec == j)))
            if n < n_steps:
                base, tr0 = oracle.single(M, lam, dx, fa, fb, n_steps - n, state=st, n0=n,
                                          rec=rec)
                st[1, j] += 1.0
                _, tr1 = oracle.single(M, lam, dx, fa, fb, n_steps - n, state=st, n0=n,
                                       rec=rec)
                W += float(np.sum(w[:, n:] * (tr1 - tr0)))
            tot += W * lap[j]
            tot_abs += abs(W * lap[j])
    _, _, gl, sa = oracle.adjoint(M, lam, dx, fa, fb, n_steps, rec, w, terms=True)
    assert tot != 0.0 and tot_abs > abs(tot)
    assert abs(gl - 2 * lam * tot) <= 1e-12 * 2 * lam * tot_abs
    assert abs(sa - 2 * lam * tot_abs) <= 1e-12 * sa


def test_float32_build_agrees_with_float64():
    """The float build of the reverse mode (same operations, W and U in
    float) against the double build: dJ/df within float rounding, dJ/dlam
    within float rounding of its magnitude sum; causality zeros exact."""
    M, n_steps = 301, 500
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(12)
    t = np.arange(n_steps + 1) * 0.9 * dx
    fa = np.sin(2 * np.pi * 6 * t) * np.exp(-3 * t)
    fa[0] = 0.0
    fb = np.zeros_like(fa)
    rec = np.array([30, 120, 250], np.int64)
    w = g.standard_normal((3, n_steps))
    ga64, _, gl64, sa64 = oracle.adjoint(M, 0.9, dx, fa, fb, n_steps, rec, w, terms=True)
    ga32, gb32, gl32, sa32 = oracle.adjoint(M, 0.9, dx, fa.astype(np.float32),
                                            fb.astype(np.float32), n_steps, rec,
                                            w.astype(np.float32), dtype=np.float32,
                                            terms=True)
    assert ga32.dtype == np.float32
    assert np.linalg.norm(ga32 - ga64) <= 1e-5 * np.linalg.norm(ga64)
    assert abs(gl32 - gl64) <= 1e-4 * sa64
    assert abs(sa32 - sa64) <= 1e-4 * sa64
    cut = n_steps - rec.min()
    assert np.all(ga32[cut + 1:] == 0.0)


def test_float32_dot_product_identity():
    M, n_steps = 201, 400
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(6)
    rec = np.sort(g.choice(np.arange(1, M - 1), 5, replace=False))
    w = g.standard_normal((len(rec), n_steps)).astype(np.float32)
    df = np.concatenate([[0.0], g.standard_normal(n_steps)]).astype(np.float32)
    z = np.zeros(n_steps + 1, np.float32)
    _, Adf = oracle.single(M, 0.9, dx, df, z, n_steps, rec=rec)
    ga, _, _ = oracle.adjoint(M, 0.9, dx, z, z, n_steps, rec, w, dtype=np.float32)
    lhs = np.sum(Adf.astype(np.float64) * w)
    rhs = np.sum(df.astype(np.float64) * ga)
    assert abs(lhs - rhs) <= 1e-5 * np.sqrt(np.sum(Adf.astype(np.float64) ** 2) *
                                            np.sum(w.astype(np.float64) ** 2))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_truncated_domain_gives_the_same_gradient(dtype):
    """From rest, driven at node 0 only, U^n_j = 0 exactly for j > n, and a
    change at node c reaches (j, n) of the reverse sweep only after
    (c - j_r) + (c - j) levels; with c = n_steps + 2 and receivers below
    n_steps, cutting the domain at node c changes no value the gradient
    reads.  So the reverse mode on M_s = n_steps + 3 nodes gives dJ/df_A of
    the whole domain bit for bit, and dJ/dlam up to the order of its sums
    (the cut domain has fewer exactly-zero terms)."""
    M, n_steps = 4001, 1500
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(31)
    t = np.arange(n_steps + 1) * 0.9 * dx
    fa = (np.sin(2 * np.pi * 9 * t / t[-1]) * np.exp(-((t - 0.3 * t[-1]) / (0.2 * t[-1])) ** 2)
          ).astype(dtype)
    fa[0] = 0
    fb = np.zeros_like(fa)
    rec = np.sort(g.choice(np.arange(1, int(0.8 * 0.9 * n_steps)), 6, replace=False))
    w = g.standard_normal((6, n_steps)).astype(dtype)
    full = oracle.adjoint(M, 0.9, dx, fa, fb, n_steps, rec, w, dtype=dtype, terms=True)
    cut = oracle.adjoint(n_steps + 3, 0.9, dx, fa, fb, n_steps, rec, w, dtype=dtype, terms=True)
    assert np.array_equal(full[0], cut[0])
    assert np.abs(full[0]).max() > 0
    assert abs(full[2] - cut[2]) <= 1e-14 * full[3]
    assert abs(full[3] - cut[3]) <= 1e-14 * full[3]
