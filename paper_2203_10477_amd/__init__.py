"""RSWR hot path on AMD MI355X: Python binding of librswr.so.

Method: Wei & Zhao, "A Non-iterative Overlapping Schwarz Waveform Relaxation
Algorithm for Wave Equation" (arXiv 2203.10477).  The functions here carry the
names of the C-ABI in include/rswr.h (rswr_plan / rswr_predict / rswr_select /
rswr_update / rswr_solve) and only marshal arguments: PyTorch provides device
memory and the current stream, every step of the method runs in the HIP
kernels of librswr.so.  There is no fallback: without the built library (or
without a GPU for the compute calls) every call raises.
"""
import ctypes
import os
from fractions import Fraction

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "librswr.so")
_lib = None

F32, F64 = 0, 1
FIXED, QUIET = 0, 1
STATUS = {0: "RSWR_OK", 1: "RSWR_ERR_INVALID_ARG", 2: "RSWR_ERR_UNSTABLE",
          3: "RSWR_ERR_LAYOUT", 4: "RSWR_ERR_SPAN", 5: "RSWR_ERR_NOMEM",
          6: "RSWR_ERR_HIP", 8: "RSWR_ERR_UNSUPPORTED"}


class RSWRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("x_a", ctypes.c_double), ("x_b", ctypes.c_double),
                ("n_points", ctypes.c_int64), ("a", ctypes.c_double),
                ("a_ref", ctypes.c_double), ("courant", ctypes.c_double),
                ("courant_num", ctypes.c_int32), ("courant_den", ctypes.c_int32),
                ("n_sub", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("sub_lo", ctypes.c_void_p), ("sub_hi", ctypes.c_void_p),
                ("span", ctypes.c_int32), ("span_mode", ctypes.c_int32),
                ("beta", ctypes.c_double), ("dtype", ctypes.c_int32),
                ("tile_threads", ctypes.c_int32), ("tile_per_thread", ctypes.c_int32),
                ("no_fuse", ctypes.c_int32), ("n_src", ctypes.c_int32),
                ("src_node", ctypes.c_void_p), ("src_amp", ctypes.c_void_p),
                ("src_ld", ctypes.c_int64), ("one_launch", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_sub", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("span", ctypes.c_int32),
                ("span_cone", ctypes.c_int32), ("span_paper", ctypes.c_int32),
                ("flux_ld", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("tile_threads", ctypes.c_int32), ("tile_per_thread", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("fused", ctypes.c_int32),
                ("one_launch", ctypes.c_int32)]


def lib():
    """Load librswr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with "
                           "`python -m paper_2203_10477_amd.build`")
    L = ctypes.CDLL(LIBPATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.rswr_plan.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(vp)]
    L.rswr_plan_destroy.argtypes = [vp]
    L.rswr_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
    L.rswr_plan_layout.argtypes = [vp, vp, vp, vp, vp]
    L.rswr_plan_tiles.argtypes = [vp, vp]
    L.rswr_predict.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp]
    L.rswr_select.argtypes = [vp, vp, i32, vp, vp]
    L.rswr_update.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, vp, vp]
    L.rswr_solve_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.rswr_checkpoint_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    L.rswr_adjoint_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.rswr_adjoint_fused.argtypes = [vp, ctypes.POINTER(i32)]
    L.rswr_solve_adjoint.argtypes = [vp, vp, vp, vp, i64, vp, i32, vp, vp, vp, vp, vp, sz,
                                     vp]
    L.rswr_solve.argtypes = [vp, vp, vp, vp, i64, i64, vp, i32, vp, vp, sz, vp, vp]
    L.rswr_solve_noalloc.argtypes = [vp, vp, vp, vp, i64, i64, vp]
    L.rswr_adjoint_batch_workspace_size.argtypes = [vp, i64, i32, i32, i32, ctypes.POINTER(sz)]
    L.rswr_solve_adjoint_batch.argtypes = [vp, i32, vp, vp, i64, i64, vp, i32, vp, vp, vp,
                                           vp, i32, i32, vp, sz, vp]
    L.rswr_span.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp]
    L.rswr_batch_plan.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.rswr_batch_destroy.argtypes = [vp]
    L.rswr_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.rswr_batch_solve.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    for name in ("rswr_plan", "rswr_plan_destroy", "rswr_plan_info", "rswr_plan_layout",
                 "rswr_plan_tiles",
                 "rswr_predict", "rswr_select", "rswr_update", "rswr_span",
                 "rswr_solve_workspace_size", "rswr_solve", "rswr_solve_noalloc",
                 "rswr_checkpoint_size",
                 "rswr_adjoint_workspace_size", "rswr_adjoint_fused", "rswr_solve_adjoint",
                 "rswr_adjoint_batch_workspace_size", "rswr_solve_adjoint_batch",
                 "rswr_batch_plan",
                 "rswr_batch_destroy", "rswr_batch_workspace_size", "rswr_batch_solve"):
        getattr(L, name).restype = ctypes.c_int
    L.rswr_status_string.argtypes = [ctypes.c_int]
    L.rswr_status_string.restype = ctypes.c_char_p
    L.rswr_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status, what):
    if status != 0:
        raise RSWRError(status, f"{what}: {lib().rswr_last_error().decode()}")


def _torch_dtype(code):
    return torch.float64 if code == F64 else torch.float32


class Plan:
    """rswr_plan: decomposition, span rule and kernel tiles (host only).

    n_points, n_sub, overlap: M grid nodes, N windows, overlap P in grid
    intervals (Sec. 2.2 Eqs. (4)-(5), Sec. 3).  courant = a dt / dx with dt
    fixed by a_ref (default a); courant_frac = (num, den) makes the span rule
    of Eq. (10) exact in integers ("auto": the fraction with denominator up
    to 1000 whose double equals courant, if any; None: the rule in double).  windows = (lo, hi) gives explicit windows.
    tile = (threads, nodes per lane) picks a built kernel shape; fuse=False
    keeps predict and update as separate launches in rswr_solve.
    sources = (nodes, amp): interior point sources (the pulse sources of
    Sec. 4): nodes in 1..M-2 (host), amp a device tensor [n_src, ld] of the
    plan's dtype; the step from level n to n+1 adds amp[q, n] at nodes[q].
    The plan keeps a reference to amp.  one_launch=True asks rswr_solve
    (without receivers) to run the whole span loop as one launch where the
    plan allows it (info["one_launch"]); results are identical.
    """

    def __init__(self, n_points, n_sub, overlap, a=1.0, courant=0.9,
                 courant_frac="auto", x_a=0.0, x_b=1.0, a_ref=0.0, span=0,
                 span_mode=FIXED, beta=0.1, dtype=torch.float64, windows=None,
                 tile=None, fuse=True, sources=None, one_launch=False):
        L = lib()
        d = _Desc()
        d.x_a, d.x_b, d.n_points = float(x_a), float(x_b), int(n_points)
        d.a, d.a_ref, d.courant = float(a), float(a_ref), float(courant)
        if isinstance(courant_frac, str) and courant_frac == "auto":
            fr = Fraction(float(courant)).limit_denominator(1000)
            courant_frac = ((fr.numerator, fr.denominator)
                            if fr > 0 and float(fr) == float(courant) else None)
        num, den = courant_frac if courant_frac is not None else (0, 0)
        d.courant_num, d.courant_den = int(num), int(den)
        d.n_sub, d.overlap = int(n_sub), int(overlap)
        self._win = None
        if windows is not None:
            lo = np.ascontiguousarray(windows[0], np.int64)
            hi = np.ascontiguousarray(windows[1], np.int64)
            self._win = (lo, hi)
            d.sub_lo = lo.ctypes.data
            d.sub_hi = hi.ctypes.data
        d.span, d.span_mode, d.beta = int(span), int(span_mode), float(beta)
        d.dtype = F64 if dtype == torch.float64 else F32
        if tile is not None:
            d.tile_threads, d.tile_per_thread = int(tile[0]), int(tile[1])
        d.no_fuse = 0 if fuse else 1
        d.one_launch = 1 if one_launch else 0
        self._src = None
        if sources is not None:
            nodes = np.ascontiguousarray(np.asarray(sources[0], np.int64).reshape(-1))
            amp = sources[1]
            want = torch.float64 if d.dtype == F64 else torch.float32
            if not (isinstance(amp, torch.Tensor) and amp.is_cuda and amp.dtype == want
                    and amp.dim() == 2 and amp.shape[0] == len(nodes)
                    and amp.is_contiguous()):
                raise RSWRError(1, "sources: amp must be a contiguous device tensor "
                                "[n_src, ld] of the plan's dtype")
            self._src = (nodes, amp)
            d.n_src = len(nodes)
            d.src_node = nodes.ctypes.data
            d.src_amp = amp.data_ptr()
            d.src_ld = amp.shape[1]
        h = ctypes.c_void_p()
        _check(L.rswr_plan(ctypes.byref(d), ctypes.byref(h)), "rswr_plan")
        self._h = h
        info = _Info()
        _check(L.rswr_plan_info(h, ctypes.byref(info)), "rswr_plan_info")
        self.info = {f[0].rstrip("_"): getattr(info, f[0]) for f in _Info._fields_}
        self.dtype = _torch_dtype(info.dtype)
        self.M = int(info.n_points)
        self.N = int(info.n_sub)
        self.span = int(info.span)
        self.flux_ld = int(info.flux_ld)
        self.flux_numel = max(self.N - 1, 1) * 2 * self.flux_ld

    @property
    def handle(self):
        return self._h

    def layout(self):
        """(lo, hi, own_lo, own_hi) as int64 numpy arrays."""
        arrs = [np.zeros(self.N, np.int64) for _ in range(4)]
        _check(lib().rswr_plan_layout(self._h, *[a.ctypes.data for a in arrs]),
               "rswr_plan_layout")
        return tuple(arrs)

    def tiles(self):
        """Update work-groups: int64 [n_tiles, 8] = region first node, region
        last node, first and last stored node, window, left end, right end
        (0 zero data, 1 input ghost, 2 Dirichlet neighbour), general flag."""
        t = np.zeros((self.info["n_tiles"], 8), np.int64)
        _check(lib().rswr_plan_tiles(self._h, t.ctypes.data), "rswr_plan_tiles")
        return t

    def flux_buffer(self, device="cuda"):
        return torch.zeros((max(self.N - 1, 1), 2, self.flux_ld), dtype=self.dtype,
                           device=device)

    def workspace_bytes(self, n_rec=0):
        b = ctypes.c_size_t()
        _check(lib().rswr_solve_workspace_size(self._h, int(n_rec), ctypes.byref(b)),
               "rswr_solve_workspace_size")
        return int(b.value)

    def n_spans(self, n_steps):
        return -(-int(n_steps) // self.span)

    def checkpoint_buffer(self, n_steps, device="cuda"):
        """Flat buffer for rswr_solve's checkpoints: span-boundary states, then
        every span's predicted fluxes (rswr_checkpoint_size)."""
        b = ctypes.c_size_t()
        _check(lib().rswr_checkpoint_size(self._h, int(n_steps), ctypes.byref(b)),
               "rswr_checkpoint_size")
        elem = 8 if self.dtype == torch.float64 else 4
        return torch.zeros(b.value // elem, dtype=self.dtype, device=device)

    def checkpoint_states(self, buf, n_steps):
        """View [n_spans+1, 2, M] of the span-boundary states in `buf`."""
        K = self.n_spans(n_steps)
        return buf[:(K + 1) * 2 * self.M].view(K + 1, 2, self.M)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.rswr_plan_destroy(h)
            self._h = None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, min_numel, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {min_numel}")
    return ctypes.c_void_p(t.data_ptr())


def rswr_predict(plan, state, f_a, f_b, n0, span_hat, flux=None):
    """Predict (Sec. 2.3): output flux waveforms [N-1, 2, flux_ld]."""
    if flux is None:
        flux = plan.flux_buffer(state.device)
    _check(lib().rswr_predict(plan.handle, _dev(state, plan.dtype, 2 * plan.M, "state"),
                              _dev(f_a, plan.dtype, n0 + span_hat, "f_a"),
                              _dev(f_b, plan.dtype, n0 + span_hat, "f_b"), int(n0),
                              int(span_hat), _dev(flux, plan.dtype, plan.flux_numel, "flux"),
                              _stream()), "rswr_predict")
    return flux


def rswr_select(plan, flux, span_hat, span_dev=None):
    """Select (Sec. 2.4): the span for this step as a 1-element int32 tensor."""
    if span_dev is None:
        span_dev = torch.zeros(1, dtype=torch.int32, device=flux.device)
    _check(lib().rswr_select(plan.handle, _dev(flux, plan.dtype, plan.flux_numel, "flux"),
                             int(span_hat),
                             _dev(span_dev, torch.int32, 1, "span_dev"), _stream()),
           "rswr_select")
    return span_dev


def rswr_update(plan, state_in, f_a, f_b, n0, flux, span=None, span_dev=None, out=None):
    """Update + glue (Sec. 2.5): the next two-level state [2, M]."""
    if out is None:
        out = torch.empty_like(state_in)
    sd = None if span_dev is None else _dev(span_dev, torch.int32, 1, "span_dev")
    need = n0 + 1 if span is None else n0 + span + 1
    _check(lib().rswr_update(plan.handle, _dev(state_in, plan.dtype, 2 * plan.M, "state_in"),
                             _dev(f_a, plan.dtype, need, "f_a"),
                             _dev(f_b, plan.dtype, need, "f_b"), int(n0),
                             _dev(flux, plan.dtype, plan.flux_numel, "flux"), sd,
                             int(span or 0), _dev(out, plan.dtype, 2 * plan.M, "state_out"),
                             _stream()), "rswr_update")
    return out


def rswr_span(plan, state_in, f_a, f_b, n0, span=None, flux=None, out=None):
    """One whole span (Sec. 2.6 loop body: predict, update, glue) of the
    fixed span, from levels n0-1, n0 to n0+span-1, n0+span; one launch when
    plan.info["fused"].  `flux` ([N-1, 2, flux_ld]) is optional for fused
    plans (it then receives the input ends' predicted rows) and required for
    the others when N > 1.  Returns the new state [2, M]."""
    if out is None:
        out = torch.empty_like(state_in)
    span = plan.span if span is None else int(span)
    fl = None if flux is None else _dev(flux, plan.dtype, plan.flux_numel, "flux")
    _check(lib().rswr_span(plan.handle, _dev(state_in, plan.dtype, 2 * plan.M, "state_in"),
                           _dev(f_a, plan.dtype, n0 + span + 1, "f_a"),
                           _dev(f_b, plan.dtype, n0 + span + 1, "f_b"), int(n0), span, fl,
                           _dev(out, plan.dtype, 2 * plan.M, "state_out"), _stream()),
           "rswr_span")
    return out


def rswr_solve(plan, state, f_a, f_b, n_steps, n0=0, receivers=None, checkpoints=None,
               workspace=None, traces=None):
    """The span loop (Sec. 2.6).  `state` [2, M] is advanced in place.

    Returns the traces [n_rec, n_steps] (None without receivers)."""
    rec = (np.zeros(0, np.int64) if receivers is None
           else np.ascontiguousarray(np.asarray(receivers, np.int64).reshape(-1)))
    n_rec = len(rec)
    if n_rec and traces is None:
        traces = torch.zeros((n_rec, n_steps), dtype=plan.dtype, device=state.device)
    if workspace is None:
        workspace = torch.empty(plan.workspace_bytes(n_rec), dtype=torch.uint8,
                                device=state.device)
    ck = None
    if checkpoints is not None:
        b = ctypes.c_size_t()
        _check(lib().rswr_checkpoint_size(plan.handle, int(n_steps), ctypes.byref(b)),
               "rswr_checkpoint_size")
        elem = 8 if plan.dtype == torch.float64 else 4
        ck = _dev(checkpoints, plan.dtype, b.value // elem, "checkpoints")
    _check(lib().rswr_solve(plan.handle, _dev(state, plan.dtype, 2 * plan.M, "state"),
                            _dev(f_a, plan.dtype, n0 + n_steps + 1, "f_a"),
                            _dev(f_b, plan.dtype, n0 + n_steps + 1, "f_b"), int(n0),
                            int(n_steps), rec.ctypes.data if n_rec else None, n_rec,
                            _dev(traces, plan.dtype, n_rec * n_steps, "traces")
                            if n_rec else None,
                            _dev(workspace, torch.uint8, 1, "workspace"),
                            workspace.numel(), ck, _stream()), "rswr_solve")
    return traces


def rswr_solve_noalloc(plan, state, f_a, f_b, n_steps, n0=0):
    """rswr_solve without receivers or checkpoints, its workspace the
    library's own device array (no allocation; see include/rswr.h).  The
    plan must have run a compute call on this device before.  `state`
    [2, M] is advanced in place."""
    _check(lib().rswr_solve_noalloc(plan.handle, _dev(state, plan.dtype, 2 * plan.M, "state"),
                                    _dev(f_a, plan.dtype, n0 + n_steps + 1, "f_a"),
                                    _dev(f_b, plan.dtype, n0 + n_steps + 1, "f_b"), int(n0),
                                    int(n_steps), _stream()), "rswr_solve_noalloc")
    return state


def rswr_adjoint_fused(plan):
    """True if rswr_solve_adjoint of `plan` runs the fused adjoint span on the
    current device (see include/rswr.h)."""
    f = ctypes.c_int32()
    _check(lib().rswr_adjoint_fused(plan.handle, ctypes.byref(f)), "rswr_adjoint_fused")
    return bool(f.value)


def rswr_solve_adjoint(plan, checkpoints, f_a, f_b, n_steps, receivers, grad_traces,
                       workspace=None):
    """Reverse mode of an n_steps solve from level 0 (see include/rswr.h).

    Returns (dJ/df_a [n_steps+1], dJ/df_b [n_steps+1], dJ/dlam as a 0-d
    float64 tensor)."""
    rec = np.ascontiguousarray(np.asarray(receivers, np.int64).reshape(-1))
    n_rec = len(rec)
    dev_ = f_a.device
    if workspace is None:
        b = ctypes.c_size_t()
        _check(lib().rswr_adjoint_workspace_size(plan.handle, n_rec, ctypes.byref(b)),
               "rswr_adjoint_workspace_size")
        workspace = torch.empty(b.value, dtype=torch.uint8, device=dev_)
    ga = torch.empty(n_steps + 1, dtype=plan.dtype, device=dev_)
    gb = torch.empty(n_steps + 1, dtype=plan.dtype, device=dev_)
    gl = torch.empty((), dtype=torch.float64, device=dev_)
    b = ctypes.c_size_t()
    _check(lib().rswr_checkpoint_size(plan.handle, int(n_steps), ctypes.byref(b)),
           "rswr_checkpoint_size")
    elem = 8 if plan.dtype == torch.float64 else 4
    gtr = grad_traces.contiguous()
    _check(lib().rswr_solve_adjoint(
        plan.handle, _dev(checkpoints, plan.dtype, b.value // elem, "checkpoints"),
        _dev(f_a, plan.dtype, n_steps + 1, "f_a"), _dev(f_b, plan.dtype, n_steps + 1, "f_b"),
        int(n_steps), rec.ctypes.data if n_rec else None, n_rec,
        _dev(gtr, plan.dtype, n_rec * n_steps, "grad_traces") if n_rec else None,
        _dev(ga, plan.dtype, n_steps + 1, "grad_f_a"),
        _dev(gb, plan.dtype, n_steps + 1, "grad_f_b"),
        ctypes.c_void_p(gl.data_ptr()), _dev(workspace, torch.uint8, 1, "workspace"),
        workspace.numel(), _stream()), "rswr_solve_adjoint")
    return ga, gb, gl


def rswr_solve_adjoint_batch(plan, f_a, f_b, n_steps, receivers, grad_traces, group=None,
                             seg=0, workspace=None):
    """Reverse mode of a batch of same-shape solves from rest (include/rswr.h):
    f_a, f_b [n_prob, ld >= n_steps+1], grad_traces [n_prob, n_rec, n_steps].
    `group` problems share each launch (default: all); seg = spans per
    checkpoint segment (0: about the square root of the span count).
    Returns (dJ/df_a [n_prob, n_steps+1], dJ/df_b, dJ/dlam [n_prob] float64)."""
    rec = np.ascontiguousarray(np.asarray(receivers, np.int64).reshape(-1))
    n_rec = len(rec)
    n_prob, src_ld = int(f_a.shape[0]), int(f_a.shape[1])
    if tuple(f_b.shape) != (n_prob, src_ld):
        raise ValueError("f_b must have the shape of f_a")
    group = n_prob if group is None else int(group)
    dev_ = f_a.device
    if workspace is None:
        b = ctypes.c_size_t()
        _check(lib().rswr_adjoint_batch_workspace_size(plan.handle, int(n_steps), n_rec, group,
                                                       int(seg), ctypes.byref(b)),
               "rswr_adjoint_batch_workspace_size")
        workspace = torch.empty(b.value, dtype=torch.uint8, device=dev_)
    ga = torch.empty(n_prob, n_steps + 1, dtype=plan.dtype, device=dev_)
    gb = torch.empty_like(ga)
    gl = torch.empty(n_prob, dtype=torch.float64, device=dev_)
    gtr = grad_traces.contiguous()
    _check(lib().rswr_solve_adjoint_batch(
        plan.handle, n_prob, _dev(f_a, plan.dtype, n_prob * src_ld, "f_a"),
        _dev(f_b, plan.dtype, n_prob * src_ld, "f_b"), src_ld, int(n_steps),
        rec.ctypes.data if n_rec else None, n_rec,
        _dev(gtr, plan.dtype, n_prob * n_rec * n_steps, "grad_traces") if n_rec else None,
        _dev(ga, plan.dtype, ga.numel(), "grad_f_a"), _dev(gb, plan.dtype, gb.numel(), "grad_f_b"),
        ctypes.c_void_p(gl.data_ptr()), group, int(seg),
        _dev(workspace, torch.uint8, 1, "workspace"), workspace.numel(), _stream()),
        "rswr_solve_adjoint_batch")
    return ga, gb, gl


class ProblemSpec:
    """Everything but f_A and a that fixes an RSWR forward run for autograd."""

    def __init__(self, n_points, n_sub, overlap, n_steps, receivers, f_b=None,
                 courant=0.9, a_ref=1.0, dtype=torch.float64, x_a=0.0, x_b=1.0):
        if not a_ref > 0:
            raise ValueError("a_ref must be positive: it fixes dt while a varies")
        self.n_points, self.n_sub, self.overlap = n_points, n_sub, overlap
        self.n_steps, self.courant, self.a_ref = n_steps, courant, a_ref
        self.receivers = np.asarray(receivers, np.int64)
        self.f_b, self.dtype, self.x_a, self.x_b = f_b, dtype, x_a, x_b

    def plan(self, a):
        return Plan(self.n_points, self.n_sub, self.overlap, a=float(a),
                    courant=self.courant, a_ref=self.a_ref, courant_frac=None,
                    dtype=self.dtype, x_a=self.x_a, x_b=self.x_b)


class RSWRFunction(torch.autograd.Function):
    """traces = RSWRFunction.apply(f_a, a, spec): receiver traces of an RSWR
    solve from rest with boundary samples f_a [n_steps+1] and wave speed a (a
    0-d tensor; dt stays fixed by spec.a_ref).  backward runs
    rswr_solve_adjoint on the span checkpoints of the forward run and returns
    dJ/df_a and dJ/da."""

    @staticmethod
    def forward(ctx, f_a, a, spec):
        plan = spec.plan(a.item())
        n = spec.n_steps
        f_b = spec.f_b if spec.f_b is not None else torch.zeros_like(f_a)
        st = torch.zeros((2, spec.n_points), dtype=spec.dtype, device=f_a.device)
        ck = plan.checkpoint_buffer(n, f_a.device)
        tr = rswr_solve(plan, st, f_a.contiguous(), f_b, n, receivers=spec.receivers,
                        checkpoints=ck)
        ctx.plan, ctx.spec = plan, spec
        ctx.save_for_backward(f_a, f_b, ck, a)
        return tr

    @staticmethod
    def backward(ctx, grad_traces):
        f_a, f_b, ck, a = ctx.saved_tensors
        plan, spec = ctx.plan, ctx.spec
        ga, _, gl = rswr_solve_adjoint(plan, ck, f_a.contiguous(), f_b, spec.n_steps,
                                       spec.receivers, grad_traces.to(spec.dtype))
        # lam = courant * a / a_ref at fixed dt
        grad_a = (gl * (spec.courant / spec.a_ref)).to(a.dtype)
        return ga, grad_a, None


class Batch:
    """Many fused-span plans of one dtype solved together (rswr_batch_plan).
    The plans are kept alive by this object."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * max(len(self.plans), 1))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().rswr_batch_plan(arr, len(self.plans), ctypes.byref(h)), "rswr_batch_plan")
        self._h = h
        self.dtype = self.plans[0].dtype if self.plans else torch.float64

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().rswr_batch_workspace_size(self._h, ctypes.byref(b)),
               "rswr_batch_workspace_size")
        return b.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.rswr_batch_destroy(h)
            self._h = None


def rswr_batch_solve(batch, states, f_a, f_b, n_steps, workspace=None):
    """Advance problem i of `batch` by n_steps[i] levels from level 0 (states
    [2, M_i] in place), all problems in one recorded graph."""
    n = len(batch.plans)
    if not (len(states) == len(f_a) == len(f_b) == len(n_steps) == n):
        raise ValueError("one state, f_a, f_b and n_steps per problem")
    if workspace is None:
        workspace = torch.empty(batch.workspace_bytes(), dtype=torch.uint8,
                                device=states[0].device)
    ptr = lambda xs: (ctypes.c_void_p * n)(*[x.value for x in xs])
    st = [_dev(s, p.dtype, 2 * p.M, "state") for s, p in zip(states, batch.plans)]
    fa = [_dev(a, p.dtype, int(k) + 1, "f_a") for a, p, k in zip(f_a, batch.plans, n_steps)]
    fb = [_dev(b, p.dtype, int(k) + 1, "f_b") for b, p, k in zip(f_b, batch.plans, n_steps)]
    ns = np.ascontiguousarray(np.asarray(n_steps, np.int64))
    _check(lib().rswr_batch_solve(batch.handle, ptr(st), ptr(fa), ptr(fb), ns.ctypes.data,
                                  ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                  _stream()), "rswr_batch_solve")
    return states


# Short names of the same calls.
predict, select, update, solve = rswr_predict, rswr_select, rswr_update, rswr_solve
span = rswr_span
batch_solve = rswr_batch_solve
solve_adjoint = rswr_solve_adjoint
solve_adjoint_batch = rswr_solve_adjoint_batch
