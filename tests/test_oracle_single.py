"""Pins of the oracle's single-domain solver (the "true solution" of Sec. 2.1).

Each test ties the oracle to something other than itself: d'Alembert's image
sum (exact for the leapfrog at Courant number 1), second-order convergence to
the continuous solution, the discrete energy of the leapfrog, causality,
mirror symmetry and linearity.
"""
import numpy as np
import pytest

import oracle


def smooth_pulse(t, width, power=6):
    """sin^power(pi t / width) on [0, width], zero elsewhere."""
    out = np.where((t > 0) & (t < width), np.sin(np.pi * t / width) ** power, 0.0)
    return out


def image_sum_nodes(g, M, n_steps):
    """d'Alembert on [0, L] with u(0,t) = G(t), u(L,t) = 0, zero initial data:
    u(x,t) = sum_k G(t - (2kL + x)/a) - G(t - (2(k+1)L - x)/a).  At Courant
    number 1 every argument is a whole number of time steps."""
    L = M - 1
    U = np.zeros((n_steps + 1, M))
    j = np.arange(M)
    for n in range(n_steps + 1):
        k = 0
        while True:
            m1 = n - 2 * k * L - j
            m2 = n - 2 * (k + 1) * L + j
            if m1.max() < 1 and m2.max() < 1:
                break
            U[n] += np.where(m1 >= 1, g[np.clip(m1, 0, None)], 0.0)
            U[n] -= np.where(m2 >= 1, g[np.clip(m2, 0, None)], 0.0)
            k += 1
    return U


def all_levels(M, lam, dx, fa, fb, n_steps, state=None):
    rec = np.arange(M)
    st, tr = oracle.single(M, lam, dx, fa, fb, n_steps, state=state, rec=rec)
    return st, tr.T  # tr.T[s] = level s+1


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 2e-5)])
def test_courant_one_is_dalembert(dtype, tol):
    M, n_steps = 201, 900  # several reflections off both ends
    dx = 1.0 / (M - 1)
    dt = dx  # a = 1, C = 1
    t = np.arange(n_steps + 1) * dt
    g = smooth_pulse(t, 60 * dt)
    fa, fb = g.astype(dtype), np.zeros(n_steps + 1, dtype)
    _, lev = all_levels(M, 1.0, dx, fa, fb, n_steps)
    ref = image_sum_nodes(g, M, n_steps)[1:]
    err = np.abs(lev.astype(np.float64) - ref).max()
    assert err <= tol * np.abs(ref).max(), err


def test_second_order_convergence():
    """At Courant 0.9 the error against the continuous image sum falls by
    about 4 each time dx is halved (the leapfrog is second order)."""
    T_w, a = 0.3, 1.0
    errs = []
    for lvl in range(4):
        M = 100 * 2 ** lvl + 1
        dx = 1.0 / (M - 1)
        dt = 0.9 * dx / a
        n_steps = 500 * 2 ** lvl
        t = np.arange(n_steps + 1) * dt
        fa = smooth_pulse(t, T_w)
        st, _ = oracle.single(M, 0.9, dx, fa, np.zeros_like(fa), n_steps)
        T = n_steps * dt
        x = np.arange(M) * dx
        u = np.zeros(M)
        for k in range(4):
            u += smooth_pulse(np.array(T - (2 * k + x) / a), T_w)
            u -= smooth_pulse(np.array(T - (2 * (k + 1) - x) / a), T_w)
        errs.append(np.abs(st[1] - u).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 3.5 < r < 4.5, (errs, ratios)


def test_discrete_energy_is_conserved():
    """E^{n+1/2} = sum ((U^{n+1}-U^n)/dt)^2
                 + a^2 sum (D+U^{n+1})(D+U^n)/dx^2 is constant for the leapfrog
    with homogeneous Dirichlet ends."""
    M, n_steps, a = 257, 1500, 1.0
    dx = 1.0 / (M - 1)
    lam = 0.9
    dt = lam * dx / a
    x = np.linspace(0, 1, M)
    st = np.zeros((2, M))
    for m, amp in ((1, 1.0), (3, 0.5), (7, 0.25), (20, 0.1)):
        st[1] += amp * np.sin(np.pi * m * x)
        st[0] += amp * np.cos(0.37 * m * dt) * np.sin(np.pi * m * x)
    st[:, 0] = st[:, -1] = 0.0
    z = np.zeros(n_steps + 1)
    _, lev = all_levels(M, lam, dx, z, z, n_steps, state=st)
    U = np.vstack([st, lev])  # U[0] = level -1, U[1] = level 0, ...
    E = []
    for n in range(1, n_steps + 1):
        kin = np.sum(((U[n + 1] - U[n]) / dt) ** 2)
        pot = a * a * np.sum(np.diff(U[n + 1]) * np.diff(U[n])) / dx ** 2
        E.append(kin + pot)
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-12 * E[0]


def test_energy_detects_wrong_speed():
    """The energy test is sensitive: with a^2 off by 1% it drifts."""
    M, n_steps, a = 129, 400, 1.0
    dx = 1.0 / (M - 1)
    lam = 0.9
    dt = lam * dx / a
    x = np.linspace(0, 1, M)
    st = np.zeros((2, M))
    st[1] = np.sin(np.pi * 5 * x)
    st[0] = st[1] * 0.99
    st[:, 0] = st[:, -1] = 0
    z = np.zeros(n_steps + 1)
    _, lev = all_levels(M, lam, dx, z, z, n_steps, state=st)
    U = np.vstack([st, lev])
    E = [np.sum(((U[n + 1] - U[n]) / dt) ** 2)
         + 1.01 * a * a * np.sum(np.diff(U[n + 1]) * np.diff(U[n])) / dx ** 2
         for n in range(1, n_steps + 1)]
    assert np.ptp(E) > 1e-4 * abs(E[0])


def test_causality():
    """Driven from the left at rest (level 0 belongs to the initial condition,
    so the boundary first moves at level 1): U^n_j is exactly zero for
    j >= n and the front node j = n-1 is not."""
    M, n_steps = 300, 250
    dx = 1.0 / (M - 1)
    t = np.arange(n_steps + 1) * 0.9 * dx
    fa = 1.0 + t  # non-zero from level 1 on
    _, lev = all_levels(M, 0.9, dx, fa, np.zeros_like(fa), n_steps)
    for n in range(1, n_steps + 1):
        assert np.all(lev[n - 1][n:] == 0.0)
        assert lev[n - 1][n - 1] != 0.0


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_mirror_symmetry_bitwise(dtype):
    M, n_steps = 401, 1200
    dx = 1.0 / (M - 1)
    t = np.arange(n_steps + 1) * 0.9 * dx
    g = np.exp(-((t - 0.1) / 0.02) ** 2).astype(dtype)
    z = np.zeros_like(g)
    _, left = all_levels(M, 0.9, dx, g, z, n_steps)
    _, right = all_levels(M, 0.9, dx, z, g, n_steps)
    assert np.array_equal(left, right[:, ::-1])


def test_linearity():
    M, n_steps = 301, 600
    dx = 1.0 / (M - 1)
    t = np.arange(n_steps + 1) * 0.9 * dx
    g = np.exp(-((t - 0.1) / 0.02) ** 2)
    h = np.sin(40 * t) * t
    z = np.zeros_like(g)
    _, a1 = all_levels(M, 0.9, dx, g, z, n_steps)
    _, a2 = all_levels(M, 0.9, dx, 2.0 * g, z, n_steps)
    assert np.array_equal(2.0 * a1, a2)  # scaling by 2 is exact
    _, b1 = all_levels(M, 0.9, dx, z, h, n_steps)
    _, ab = all_levels(M, 0.9, dx, g, h, n_steps)
    assert np.abs(ab - (a1 + b1)).max() <= 1e-13 * np.abs(ab).max()


def test_point_values_match_full_solve():
    """The light-cone evaluator used for large cases equals the full solve."""
    M, n_steps = 2000, 300
    dx = 1.0 / (M - 1)
    g = np.random.default_rng(1)
    st0 = g.standard_normal((2, M))
    t = np.arange(n_steps + 1) * 0.9 * dx
    fa = np.sin(30 * t)
    fb = np.cos(20 * t)
    full, _ = oracle.single(M, 0.9, dx, fa, fb, n_steps, state=st0)
    nodes = np.array([0, 5, 700, 701, 1500, M - 1])
    pv = oracle.point_values(M, 0.9, dx, fa, fb, n_steps, st0, nodes)
    assert np.array_equal(pv, full[:, nodes])
