"""CPU oracle of the RSWR hot path (Wei & Zhao, arXiv 2203.10477).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use it; the GPU product path never imports it.  It shares
no code with the GPU library: the arithmetic lives in plain C
(rswr_oracle_real.c, rswr_layout.c) and this module only marshals numpy arrays.

State arrays are numpy arrays of shape (2, M): row 0 is level n0-1, row 1 level
n0.  Source arrays f_a, f_b are indexed by absolute level.  Flux arrays have
shape (N-1, 2, ld): [i, 0, s] is window i's output flux at lo_{i+1}, [i, 1, s]
window i+1's output flux at hi_i, both at level n0+s.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FIXED, QUIET, PAPER = 0, 1, 2

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    lib.oracle_layout.argtypes = [i64, i32, i32, vp, vp, vp, vp]
    lib.oracle_layout.restype = ctypes.c_int
    lib.oracle_check_layout.argtypes = [i64, i32, vp, vp, vp, vp]
    lib.oracle_check_layout.restype = ctypes.c_int
    lib.oracle_span_cone.argtypes = [i32, vp, vp]
    lib.oracle_span_cone.restype = i32
    lib.oracle_threads.argtypes = [ctypes.c_int]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_span_paper.argtypes = [i32, dbl, i32, i32]
    lib.oracle_span_paper.restype = i32
    for suf in ("_f64", "_f32"):
        f = getattr(lib, "oracle_single" + suf)
        f.argtypes = [i64, dbl, dbl, vp, vp, i64, i64, vp, i32, vp, vp, i64, i32, vp, vp,
                      i64]
        f.restype = None
        f = getattr(lib, "oracle_predict" + suf)
        f.argtypes = [i64, i32, vp, vp, dbl, dbl, vp, vp, i64, i32, vp, vp, i32, vp, i32,
                      vp, vp, i64]
        f.restype = None
        f = getattr(lib, "oracle_update" + suf)
        f.argtypes = [i64, i32, vp, vp, vp, vp, dbl, dbl, vp, vp, i64, i32, vp, vp,
                      i32, vp, i32, vp, i32, vp, vp, i64, i64, i32, vp, vp, i64]
        f.restype = None
        f = getattr(lib, "oracle_rswr" + suf)
        f.argtypes = [i64, i32, vp, vp, vp, vp, dbl, dbl, vp, vp, i64, i64, vp, i32,
                      i32, i32, i32, dbl, i32, vp, vp, i64, vp, i32, i32, vp, vp, i64]
        f.restype = ctypes.c_int
    for suf in ("_f64", "_f32"):
        f = getattr(lib, "oracle_rswr_many" + suf)
        f.argtypes = [i32] + [vp] * 13
        f.restype = None
        f = getattr(lib, "oracle_adjoint" + suf)
        f.argtypes = [i64, dbl, dbl, vp, vp, i64, i32, vp, vp, i64, i32, vp, vp, vp, vp]
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _suffix(dtype):
    dtype = np.dtype(dtype)
    if dtype == np.float64:
        return "_f64"
    if dtype == np.float32:
        return "_f32"
    raise TypeError(f"oracle supports float64 and float32, not {dtype}")


def _c(a, dtype=None):
    return np.ascontiguousarray(a, dtype=dtype)


def _src(src, dtype):
    """Interior point sources: None, or (nodes[n_src], amp[n_src, ld]) where
    amp[q, n] is added to node nodes[q] by the step from level n to n+1.
    Returns (arrays kept alive, n_src, node pointer, amp pointer, ld)."""
    if src is None:
        return None, 0, None, None, 0
    nodes = _c(np.asarray(src[0], np.int64).reshape(-1))
    amp = _c(np.asarray(src[1]).reshape(len(nodes), -1), dtype)
    return (nodes, amp), len(nodes), _ptr(nodes), _ptr(amp), amp.shape[1]


def threads(n=0):
    """Set the threads of the oracle's parallel loops (n >= 1); returns the
    number in force."""
    return int(_load().oracle_threads(int(n)))


class Layout:
    """Windows [lo_i, hi_i] and owned ranges [own_lo_i, own_hi_i] (Sec. 2.2, 3)."""

    def __init__(self, M, lo, hi, own_lo, own_hi):
        self.M = int(M)
        self.lo, self.hi = lo, hi
        self.own_lo, self.own_hi = own_lo, own_hi
        self.N = len(lo)

    @property
    def span_cone(self):
        return int(_load().oracle_span_cone(self.N, _ptr(self.lo), _ptr(self.hi)))


def layout(M, N, P):
    """Uniform layout: cores round(i(M-1)/N), half-overlap P/2 on each side."""
    lib = _load()
    lo, hi, ol, oh = (np.zeros(N, np.int64) for _ in range(4))
    rc = lib.oracle_layout(M, N, P, _ptr(lo), _ptr(hi), _ptr(ol), _ptr(oh))
    if rc != 0:
        raise ValueError(f"invalid layout M={M} N={N} P={P} (code {rc})")
    return Layout(M, lo, hi, ol, oh)


def explicit_layout(M, lo, hi):
    lib = _load()
    lo, hi = _c(lo, np.int64), _c(hi, np.int64)
    N = len(lo)
    ol, oh = np.zeros(N, np.int64), np.zeros(N, np.int64)
    rc = lib.oracle_check_layout(M, N, _ptr(lo), _ptr(hi), _ptr(ol), _ptr(oh))
    if rc != 0:
        raise ValueError(f"invalid explicit layout (code {rc})")
    return Layout(M, lo, hi, ol, oh)


def span_paper(P, lam, frac=None):
    """Largest S with 2 S lam < P (Eq. (10) in steps); frac=(num, den) is exact."""
    num, den = frac if frac is not None else (0, 0)
    return int(_load().oracle_span_paper(P, float(lam), num, den))


def single(M, lam, dx, fa, fb, n_steps, state=None, n0=0, rec=(), src=None):
    """Single-domain leapfrog; returns (state, traces[n_rec, n_steps]).
    src: interior point sources, see _src."""
    fa = _c(fa)
    dtype = fa.dtype
    fb = _c(fb, dtype)
    st = np.zeros((2, M), dtype) if state is None else _c(state, dtype).copy()
    rec = _c(np.asarray(rec, np.int64).reshape(-1))
    tr = np.zeros((len(rec), max(n_steps, 1)), dtype)
    assert fa.shape[0] >= n0 + n_steps + 1 and fb.shape[0] >= n0 + n_steps + 1
    keep, ns, sn, sa, sld = _src(src, dtype)
    assert ns == 0 or sld >= n0 + n_steps
    getattr(_load(), "oracle_single" + _suffix(dtype))(
        M, lam, dx, _ptr(fa), _ptr(fb), n0, n_steps, _ptr(st), len(rec), _ptr(rec),
        _ptr(tr), tr.shape[1], ns, sn, sa, sld)
    return st, tr[:, :n_steps]


def predict(lay, lam, dx, fa, fb, n0, shat, state, ld=None, hist=False, src=None):
    """Literal prediction of every window; returns flux (N-1, 2, ld) [, hist]."""
    fa = _c(fa)
    dtype = fa.dtype
    fb = _c(fb, dtype)
    state = _c(state, dtype)
    N = lay.N
    ld = shat if ld is None else ld
    flux = np.zeros((max(N - 1, 1), 2, ld), dtype)
    h = None
    if hist:
        hld = max([int(lay.hi[i] - lay.lo[i + 1] + 1) for i in range(N - 1)] + [1])
        h = np.zeros((max(N - 1, 1), 2, shat + 1, hld), dtype)
    keep, ns, sn, sa, sld = _src(src, dtype)
    assert ns == 0 or sld >= n0 + shat
    getattr(_load(), "oracle_predict" + _suffix(dtype))(
        lay.M, N, _ptr(lay.lo), _ptr(lay.hi), lam, dx, _ptr(fa), _ptr(fb), n0, shat,
        _ptr(state), _ptr(flux), ld, _ptr(h), ns, sn, sa, sld)
    return (flux, h) if hist else flux


def update(lay, lam, dx, fa, fb, n0, S, state, flux, windows=None, rec=(),
           traces=None, trace_level0=0, out=None, src=None):
    """Literal update + gluing; returns (state_out, traces)."""
    fa = _c(fa)
    dtype = fa.dtype
    fb = _c(fb, dtype)
    state = _c(state, dtype)
    flux = _c(flux, dtype)
    ld = flux.shape[2]
    out = np.zeros_like(state) if out is None else out
    rec = _c(np.asarray(rec, np.int64).reshape(-1))
    if traces is None:
        traces = np.zeros((len(rec), max(n0 + S - trace_level0, 1)), dtype)
    sel = None if windows is None else _c(windows, np.int32)
    keep, ns, sn, sa, sld = _src(src, dtype)
    assert ns == 0 or sld >= n0 + S
    getattr(_load(), "oracle_update" + _suffix(dtype))(
        lay.M, lay.N, _ptr(lay.lo), _ptr(lay.hi), _ptr(lay.own_lo), _ptr(lay.own_hi),
        lam, dx, _ptr(fa), _ptr(fb), n0, S, _ptr(state), _ptr(flux), ld, _ptr(out),
        0 if sel is None else len(sel), _ptr(sel), len(rec), _ptr(rec), _ptr(traces),
        traces.shape[1], trace_level0, ns, sn, sa, sld)
    return out, traces


def rswr(lay, lam, dx, fa, fb, n_steps, mode=FIXED, span=None, beta=0.1,
         state=None, n0=0, rec=(), tau_hat=0, src=None):
    """The whole span loop; returns (state, traces[n_rec, n_steps], spans).

    tau_hat is the first predictive span of the adaptive modes (Sec. 2.3);
    0 means the light-cone limit span_cone."""
    fa = _c(fa)
    dtype = fa.dtype
    fb = _c(fb, dtype)
    M = lay.M
    st = np.zeros((2, M), dtype) if state is None else _c(state, dtype).copy()
    rec = _c(np.asarray(rec, np.int64).reshape(-1))
    tr = np.zeros((len(rec), max(n_steps, 1)), dtype)
    cone = lay.span_cone
    if mode == FIXED and span is None:
        raise ValueError("FIXED mode needs a span")
    cap = n_steps + 1
    spans = np.zeros(cap, np.int32)
    keep, ns, sn, sa, sld = _src(src, dtype)
    assert ns == 0 or sld >= n0 + n_steps
    k = getattr(_load(), "oracle_rswr" + _suffix(dtype))(
        M, lay.N, _ptr(lay.lo), _ptr(lay.hi), _ptr(lay.own_lo), _ptr(lay.own_hi), lam,
        dx, _ptr(fa), _ptr(fb), n0, n_steps, _ptr(st), mode,
        0 if span is None else int(span), min(cone, 2**31 - 1), int(tau_hat), beta,
        len(rec),
        _ptr(rec), _ptr(tr), tr.shape[1], _ptr(spans), cap, ns, sn, sa, sld)
    if k < 0:
        raise ValueError(f"oracle_rswr failed ({k})")
    return st, tr[:, :n_steps], spans[:k]


def rswr_many(lays, lams, dxs, fas, fbs, n_steps, spans, states=None):
    """FIXED-span RSWR of many independent problems from level 0 (no
    receivers or sources), the problems spread over the threads.  lays:
    Layout per problem; fas/fbs: sources (one dtype for all); states: start
    states (2, M) or None (at rest).  Returns the final states."""
    n = len(lays)
    # largest problems first, so the threads finish together
    order = sorted(range(n), key=lambda i: -lays[i].M * int(n_steps[i]))
    if order != list(range(n)):
        pick = lambda xs: [xs[i] for i in order]
        out = rswr_many(pick(lays), pick(lams), pick(dxs), pick(fas), pick(fbs),
                        pick(n_steps), pick(spans), None if states is None else pick(states))
        res = [None] * n
        for k, i in enumerate(order):
            res[i] = out[k]
        return res
    dtype = np.asarray(fas[0]).dtype
    suf = _suffix(dtype)
    keep = []

    def arr(xs, ctype):
        a = (ctype * max(n, 1))(*xs)
        keep.append(a)
        return ctypes.cast(a, ctypes.c_void_p)

    fa_c = [_c(a, dtype) for a in fas]
    fb_c = [_c(b, dtype) for b in fbs]
    st = [np.zeros((2, l.M), dtype) if states is None or states[i] is None
          else _c(states[i], dtype).copy() for i, l in enumerate(lays)]
    for q, f, g in zip(lays, fa_c, fb_c):
        assert f.shape[0] >= 1 and g.shape[0] == f.shape[0]
    for k, f in zip(n_steps, fa_c):
        assert f.shape[0] >= int(k) + 1
    vp = ctypes.c_void_p
    getattr(_load(), "oracle_rswr_many" + suf)(
        n, arr([l.M for l in lays], ctypes.c_int64), arr([l.N for l in lays], ctypes.c_int32),
        arr([l.lo.ctypes.data for l in lays], vp), arr([l.hi.ctypes.data for l in lays], vp),
        arr([l.own_lo.ctypes.data for l in lays], vp),
        arr([l.own_hi.ctypes.data for l in lays], vp),
        arr([float(x) for x in lams], ctypes.c_double),
        arr([float(x) for x in dxs], ctypes.c_double),
        arr([a.ctypes.data for a in fa_c], vp), arr([b.ctypes.data for b in fb_c], vp),
        arr([int(k) for k in n_steps], ctypes.c_int64),
        arr([int(s) for s in spans], ctypes.c_int32), arr([a.ctypes.data for a in st], vp))
    return st


def adjoint(M, lam, dx, fa, fb, n_steps, rec, grad_traces, ck=64, dtype=np.float64,
            terms=False):
    """Reverse mode of the single-domain solve from rest, in float64 or
    float32 (the precision of W, the forward field and the Laplacian; every
    dJ/dlam product and sum is taken in double).

    Returns (dJ/df_a[0..n_steps], dJ/df_b[0..n_steps], dJ/dlam), and with
    terms=True also 2|lam| sum |W Lap U|, the scale of dJ/dlam's rounding."""
    suf = _suffix(dtype)
    fa = _c(fa, dtype)
    fb = _c(fb, dtype)
    rec = _c(np.asarray(rec, np.int64).reshape(-1))
    gt = _c(grad_traces, dtype)
    ga = np.zeros(n_steps + 1, dtype)
    gb = np.zeros(n_steps + 1, dtype)
    gl = ctypes.c_double(0.0)
    sa = ctypes.c_double(0.0)
    rc = getattr(_load(), "oracle_adjoint" + suf)(
        M, lam, dx, _ptr(fa), _ptr(fb), n_steps, len(rec), _ptr(rec), _ptr(gt),
        gt.shape[1] if gt.ndim == 2 else n_steps, ck, _ptr(ga), _ptr(gb), ctypes.byref(gl),
        ctypes.byref(sa))
    if rc != 0:
        raise RuntimeError(f"oracle_adjoint{suf} failed ({rc})")
    return (ga, gb, gl.value, sa.value) if terms else (ga, gb, gl.value)


def point_values(M, lam, dx, fa, fb, n_steps, state, nodes, n0=0, src=None):
    """Values of the single-domain solution at `nodes` after n_steps.

    Each contiguous group of requested nodes is computed by oracle_single on
    the sub-range reachable within n_steps (a node moves its influence one
    node per level); the cut ends carry zero data, which cannot reach the
    requested nodes in time."""
    fa = _c(fa)
    dtype = fa.dtype
    fb = _c(fb, dtype)
    state = _c(state, dtype)
    nodes = np.asarray(nodes, np.int64)
    out = np.zeros((2, len(nodes)), dtype)
    order = np.argsort(nodes)
    groups, cur = [], [order[0]]
    for a, b in zip(order[:-1], order[1:]):
        if nodes[b] - nodes[a] <= 2 * n_steps + 2:
            cur.append(b)
        else:
            groups.append(cur)
            cur = [b]
    groups.append(cur)
    for g in groups:
        jmin, jmax = int(nodes[g].min()), int(nodes[g].max())
        A = max(0, jmin - n_steps - 1)
        B = min(M - 1, jmax + n_steps + 1)
        Ms = B - A + 1
        sfa = fa if A == 0 else np.zeros_like(fa)
        sfb = fb if B == M - 1 else np.zeros_like(fb)
        ssrc = None
        if src is not None:
            sn = np.asarray(src[0], np.int64)
            keep = (sn > A) & (sn < B)
            ssrc = (sn[keep] - A, np.asarray(src[1])[keep])
        st, _ = single(Ms, lam, dx, sfa, sfb, n_steps, state=state[:, A:B + 1].copy(),
                       n0=n0, src=ssrc)
        for idx in g:
            out[:, idx] = st[:, nodes[idx] - A]
    return out
