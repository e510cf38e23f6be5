"""Seeded synthetic inputs for the RSWR hot path.

This module holds problem data only -- boundary sources sampled on the time
grid, initial states, receiver positions and the batched-instance recipe -- and
none of the method's arithmetic.  Both the GPU path and the CPU oracle consume
the arrays it returns, so neither side has to reproduce the other's random
numbers.  Every generator uses numpy's PCG64 with seed 220310477 + config.

The paper (arXiv 2203.10477, Sec. 4) runs its experiments on unspecified
pulse sources without data or parameters; these recipes stand in for them.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 220310477


def rng(tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(tag)))


def time_grid(M: int, n_steps: int, courant: float, a_ref: float,
              x_a: float = 0.0, x_b: float = 1.0) -> np.ndarray:
    """Sampling times t_n = n dt, n = 0..n_steps, dt = courant dx / a_ref."""
    dx = (x_b - x_a) / (M - 1)
    dt = courant * dx / a_ref
    return np.arange(n_steps + 1, dtype=np.float64) * dt


def gaussian(t, tc, w):
    return np.exp(-((t - tc) / w) ** 2)


def ricker(t, f, t0, amp):
    arg = (np.pi * f * (t - t0)) ** 2
    return amp * (1.0 - 2.0 * arg) * np.exp(-arg)


def smooth_state(M: int, g: np.random.Generator, n_modes: int = 6,
                 shift: float = 1e-3) -> np.ndarray:
    """A smooth non-zero two-level state (rows: level n0-1, level n0)."""
    x = np.linspace(0.0, 1.0, M)
    st = np.zeros((2, M))
    for _ in range(n_modes):
        amp = g.uniform(0.2, 1.0)
        m = g.integers(1, 40)
        ph = g.uniform(0, 2 * np.pi)
        st[1] += amp * np.sin(2 * np.pi * m * x + ph)
        st[0] += amp * np.sin(2 * np.pi * m * (x + shift) + ph)
    return st


@dataclass
class Problem:
    """One RSWR problem instance (Sec. 2.1 Eqs. (1)-(3), Sec. 2.2, Sec. 3)."""
    name: str
    M: int
    N: int
    P: int
    n_steps: int
    fa: np.ndarray              # f_A at levels 0..n_steps (level 0 unused)
    fb: np.ndarray              # f_B at levels 0..n_steps
    a: float = 1.0
    a_ref: float = 1.0          # speed that fixes dt
    courant: float = 0.9
    courant_frac: tuple = (9, 10)
    x_a: float = 0.0
    x_b: float = 1.0
    state: Optional[np.ndarray] = None   # (2, M) start state; None = at rest
    rec: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    dtype: type = np.float64

    @property
    def dx(self):
        return (self.x_b - self.x_a) / (self.M - 1)

    @property
    def lam(self):
        return self.courant * (self.a / self.a_ref)

    def state0(self):
        if self.state is None:
            return np.zeros((2, self.M), self.dtype)
        return np.ascontiguousarray(self.state, self.dtype)

    def sources(self):
        return (np.ascontiguousarray(self.fa, self.dtype),
                np.ascontiguousarray(self.fb, self.dtype))


def config1(dtype=np.float64) -> Problem:
    """N=2 parity case: 1001 nodes on [0,1], overlap 20 intervals, Gaussian
    pulse g(t) = exp(-((t-0.1)/0.02)^2) on the left, u = 0 on the right,
    Courant 0.9, 2000 steps."""
    M, n = 1001, 2000
    t = time_grid(M, n, 0.9, 1.0)
    return Problem("plain-1001-N2-P20", M=M, N=2, P=20, n_steps=n,
                   fa=gaussian(t, 0.1, 0.02), fb=np.zeros(n + 1), dtype=dtype)


def ricker_source(M, n_steps, g, courant=0.9, a_ref=1.0, t0_range=None):
    """Ricker wavelet whose peak frequency is 40 over the time the run lasts
    (the reachable crossing time n_steps dt), centred 1.5 periods in."""
    t = time_grid(M, n_steps, courant, a_ref)
    T = t[-1]
    f = 40.0 / T
    amp = g.uniform(0.5, 2.0)
    t0 = 1.5 / f if t0_range is None else g.uniform(*t0_range) / f
    return ricker(t, f, t0, amp)


def pulse_sources(M, N, n_steps, g, courant=0.9, a_ref=1.0, count=None):
    """Interior pulse sources standing in for the "N pulse sources" of the
    paper's experiments (Sec. 4): `count` (default N) Ricker pulses, one in
    each of `count` equal stretches of the interior, at a uniformly drawn
    node; peak frequency 40 over the run, delay 1.2..3 periods, amplitude
    A in [0.5, 2].  Returns (nodes[count] int64, amp[count, n_steps + 1])
    with amp[q, n] = A pi f dt ricker(t_n): the value the step from level n
    to n+1 adds at nodes[q] (of the order of dt^2 times a point source of
    strength A f / dt, which radiates a pulse of order A)."""
    count = N if count is None else count
    t = time_grid(M, n_steps, courant, a_ref)
    dt = t[1] - t[0]
    f = 40.0 / t[-1]
    edges = np.linspace(1, M - 2, count + 1)
    nodes = np.empty(count, np.int64)
    amp = np.empty((count, n_steps + 1))
    for q in range(count):
        lo, hi = int(np.ceil(edges[q])), int(np.floor(edges[q + 1]))
        nodes[q] = g.integers(lo, max(hi, lo) + 1)
        A = g.uniform(0.5, 2.0)
        t0 = g.uniform(1.2, 3.0) / f
        amp[q] = np.pi * f * dt * ricker(t, f, t0, A)
    return nodes, amp


def config2(dtype=np.float64, M=2 ** 20, N=64, P=64, n_steps=10 ** 4,
            smooth=False) -> Problem:
    """Plain throughput case: 2^20 nodes, 64 windows, overlap 64, 10^4 steps,
    Ricker source with amplitude in [0.5, 2]."""
    g = rng(2)
    fa = ricker_source(M, n_steps, g)
    st = smooth_state(M, g) if smooth else None
    return Problem(f"plain-{M}-N{N}-P{P}", M=M, N=N, P=P, n_steps=n_steps, fa=fa,
                   fb=np.zeros(n_steps + 1), state=st, dtype=dtype)


def receivers(g, n_rec, hi_node):
    return np.sort(g.choice(np.arange(1, hi_node + 1), size=n_rec,
                            replace=False)).astype(np.int64)


def config4(dtype=np.float64, M=2 ** 18, N=128, P=64, n_steps=8192,
            n_rec=16) -> Problem:
    """Adjoint case: 2^18 nodes, 128 windows, overlap 64, 8192 steps, 16
    receivers on nodes the wave reaches (1 .. floor(0.8 C n_steps))."""
    g = rng(4)
    fa = ricker_source(M, n_steps, g)
    hi_node = min(M - 2, int(0.8 * 0.9 * n_steps))
    rec = receivers(g, n_rec, hi_node)
    return Problem(f"adjoint-{M}-N{N}-P{P}", M=M, N=N, P=P, n_steps=n_steps, fa=fa,
                   fb=np.zeros(n_steps + 1), rec=rec, dtype=dtype)


def config5(dtype=np.float32, M=2 ** 24, N=4096, P=64, n_steps=2 * 10 ** 4,
            smooth=False) -> Problem:
    """Large case: 2^24 nodes, 4096 windows, overlap 64, 2*10^4 steps."""
    g = rng(5)
    fa = ricker_source(M, n_steps, g)
    st = smooth_state(M, g) if smooth else None
    return Problem(f"plain-{M}-N{N}-P{P}", M=M, N=N, P=P, n_steps=n_steps, fa=fa,
                   fb=np.zeros(n_steps + 1), state=st, dtype=dtype)


def adjoint_batch_sources(M, n_steps, count, tag=55):
    """`count` random Ricker sources (amplitude in [0.5,2], centre 1.2..2.0
    periods) for a batch of adjoint solves on one shape."""
    g = rng(tag)
    return np.stack([ricker_source(M, n_steps, g, t0_range=(1.2, 2.0))
                     for _ in range(count)])


def config3(count=512, n_steps=4096, log2_range=(12, 18), tag=3,
            dtype=np.float32):
    """Batched case: instances with M = round(2^U[12,18]), a ~ U[0.5,2],
    N ~ U{4..256}, P ~ 2 U{16..64}; N is clamped to floor((M-1)/P) so every
    core is at least P wide; Gaussian pulse with width w ~ U[0.01,0.05] T and
    centre ~ U[3w, 0.5T], T = n_steps dt.  Returns (problems, n_clamped)."""
    g = rng(tag)
    probs, clamped = [], 0
    for b in range(count):
        M = int(round(2.0 ** g.uniform(*log2_range)))
        a = float(g.uniform(0.5, 2.0))
        N = int(g.integers(4, 257))
        P = 2 * int(g.integers(16, 65))
        nmax = (M - 1) // P
        if N > nmax:
            N = max(1, nmax)
            clamped += 1
        t = time_grid(M, n_steps, 0.9, a)
        T = t[-1]
        w = g.uniform(0.01, 0.05) * T
        tc = g.uniform(3 * w, 0.5 * T)
        probs.append(Problem(f"batch-{b}", M=M, N=N, P=P, n_steps=n_steps,
                             fa=gaussian(t, tc, w), fb=np.zeros(n_steps + 1), a=a,
                             a_ref=a, dtype=dtype))
    return probs, clamped
