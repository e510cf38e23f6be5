"""Autotuner of the span kernel's tile shape.

For one problem (grid size, windows, overlap, span, dtype) every kernel shape
built into librswr.so (rswr_kernel_shapes) that can hold the span is timed on
the device: one whole span over all windows (rswr_span: one fused launch, or
predict + update where the plan cannot fuse) from a smooth state, repeated,
with HIP events on the current stream.  The fastest shape wins; the result
can be kept in a JSON cache keyed by device name and problem.
"""
import ctypes
import json
import os

import numpy as np
import torch

from . import Plan, RSWRError, lib, rswr_span


def kernel_shapes():
    L = lib()
    L.rswr_kernel_shapes.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int32]
    L.rswr_kernel_shapes.restype = ctypes.c_int32
    n = L.rswr_kernel_shapes(None, None, None, 0)
    th, pt, ok = (np.zeros(n, np.int32) for _ in range(3))
    L.rswr_kernel_shapes(th.ctypes.data, pt.ctypes.data, ok.ctypes.data, n)
    return [(int(a), int(b), bool(c)) for a, b, c in zip(th, pt, ok)]


def _key(n_points, n_sub, overlap, span, dtype):
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{name}|{str(dtype)}|{n_points}|{n_sub}|{overlap}|{span}"


def time_span(plan, reps=10, warmup=3):
    """Average microseconds of one span (rswr_span) of `plan`."""
    M = plan.M
    dev = "cuda"
    x = torch.linspace(0, 1, M, dtype=torch.float64, device=dev)
    st = torch.stack([torch.sin(40 * x + 0.1), torch.sin(40 * x)]).to(plan.dtype).contiguous()
    n = plan.span + 1
    fa = torch.zeros(n + 1, dtype=plan.dtype, device=dev)
    fb = torch.zeros_like(fa)
    flux = None if plan.info["fused"] else plan.flux_buffer(dev)
    out = torch.empty_like(st)
    for _ in range(warmup):
        rswr_span(plan, st, fa, fb, 0, flux=flux, out=out)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        rswr_span(plan, st, fa, fb, 0, flux=flux, out=out)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def autotune(n_points, n_sub, overlap, dtype=torch.float32, span=0, reps=10,
             cache=None, **plan_kw):
    """Returns ((threads, per_thread), {shape: microseconds})."""
    key = _key(n_points, n_sub, overlap, span, dtype)
    if cache and os.path.exists(cache):
        table = json.load(open(cache))
        if key in table:
            ent = table[key]
            return tuple(ent["best"]), {tuple(map(int, k.split("x"))): v
                                        for k, v in ent["times_us"].items()}
    times = {}
    for th, pt, fp64_ok in kernel_shapes():
        if dtype == torch.float64 and not fp64_ok:
            continue
        try:
            plan = Plan(n_points, n_sub, overlap, span=span, dtype=dtype, tile=(th, pt),
                        **plan_kw)
        except RSWRError:
            continue  # shape cannot hold this span
        times[(th, pt)] = time_span(plan, reps=reps)
    if not times:
        raise RuntimeError("no built kernel shape fits this problem")
    best = min(times, key=times.get)
    if cache:
        table = json.load(open(cache)) if os.path.exists(cache) else {}
        table[key] = {"best": list(best),
                      "times_us": {f"{a}x{b}": v for (a, b), v in times.items()}}
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return best, times
