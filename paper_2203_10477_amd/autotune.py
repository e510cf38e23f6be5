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


def _plan_for(prob, dtype, tile, span=0):
    return Plan(prob.M, prob.N, prob.P, a=prob.a, a_ref=prob.a_ref, courant=prob.courant,
                courant_frac=prob.courant_frac, x_a=prob.x_a, x_b=prob.x_b, span=span,
                dtype=dtype, tile=tile)


def batch_span(prob, dtype):
    """Fixed span of a batched problem: the default rule (light-cone limit and
    Eq. (10)), capped at the fused kernel's 63 levels."""
    return min(_plan_for(prob, dtype, None).span, 63)


def size_class(prob):
    """Problems with windows of similar width share a tile shape."""
    core = (prob.M - 1) / max(prob.N, 1)
    return int(np.floor(np.log2(core + prob.P + 1)))


def _candidates(prob, dtype, span):
    """Shapes whose plan runs the fused span, with the nodes the tiles
    compute per span (threads * nodes per lane * tiles)."""
    out = {}
    for th, pt, fp64_ok in kernel_shapes():
        if dtype == torch.float64 and not fp64_ok:
            continue
        try:
            p = _plan_for(prob, dtype, (th, pt), span)
        except RSWRError:
            continue
        if p.info["fused"]:
            out[(th, pt)] = p.info["n_tiles"] * th * pt
    return out


def time_batch(plans, probs, n_steps, reps=3):
    """Microseconds of one rswr_batch_solve of `plans` (n_steps each: an int
    or one per problem)."""
    from . import Batch, rswr_batch_solve
    b = Batch(plans)
    dev = "cuda"
    ns = list(n_steps) if hasattr(n_steps, "__len__") else [int(n_steps)] * len(plans)
    st = [torch.zeros(2, p.M, dtype=p.dtype, device=dev) for p in plans]
    fa = [torch.as_tensor(q.fa[:n + 1], dtype=p.dtype, device=dev)
          for q, p, n in zip(probs, plans, ns)]
    fb = [torch.zeros(n + 1, dtype=p.dtype, device=dev) for p, n in zip(plans, ns)]
    ws = torch.empty(b.workspace_bytes(), dtype=torch.uint8, device=dev)
    rswr_batch_solve(b, st, fa, fb, ns, ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rswr_batch_solve(b, st, fa, fb, ns, ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def autotune_batch(probs, dtype=torch.float32, sample=16, spans_timed=4, slack=1.5,
                   measure=True, refine=True, sweeps=2, log=None):
    """Tile shape per size class for a batch of problems.

    Every problem gets the span batch_span().  Within a size class, the shapes
    that run the fused span for every problem of a sample, and whose computed
    nodes stay within `slack` times the least, are timed as one batched solve
    of the sample over `spans_timed` spans; the fastest wins (measure=False:
    the least computed nodes wins).  With `refine`, each class's shortlist is
    then tried again in the complete batched solve (classes run side by side
    there), class by class, keeping a change only if the whole solve gets
    faster; `sweeps` passes over the classes (a change of one class can make
    another class's alternative pay).  `log`, if given, receives one line
    per class timed and per refinement trial.  Returns (tiles per problem, spans per problem, {class: (shape,
    {shape: microseconds})})."""
    spans = [batch_span(p, dtype) for p in probs]
    classes = {}
    for i, p in enumerate(probs):
        classes.setdefault(size_class(p), []).append(i)
    tiles = [None] * len(probs)
    report, shortlists = {}, {}
    g = np.random.default_rng(0)

    def fix_unfused(tl):
        # a shape chosen for a sample may not fuse every problem of its class
        for i, p in enumerate(probs):
            if not _plan_for(p, dtype, tl[i], spans[i]).info["fused"]:
                cand = _candidates(p, dtype, spans[i])
                tl[i] = min(cand, key=cand.get)
    for c, idx in sorted(classes.items()):
        pick = idx if len(idx) <= sample else sorted(g.choice(idx, sample, replace=False))
        work = None
        for i in pick:
            cand = _candidates(probs[i], dtype, spans[i])
            work = cand if work is None else {k: work[k] + v for k, v in cand.items() if k in work}
        if not work:
            raise RuntimeError(f"no fused shape fits size class {c}")
        least = min(work.values())
        shortlist = sorted(k for k, v in work.items() if v <= slack * least)
        times = {}
        if measure and len(shortlist) > 1:
            n_steps = spans_timed * max(spans[i] for i in pick)
            for sh in shortlist:
                plans = [_plan_for(probs[i], dtype, sh, spans[i]) for i in pick]
                times[sh] = time_batch(plans, [probs[i] for i in pick], n_steps)
            best = min(times, key=times.get)
        else:
            best = min(shortlist, key=lambda k: work[k])
        report[c] = (best, times)
        shortlists[c] = shortlist
        if log:
            log(f"size class {c}: {best[0]}x{best[1]} of {len(shortlist)} shapes")
        for i in idx:
            tiles[i] = best
    fix_unfused(tiles)
    if measure and refine:
        n_steps = [p.n_steps for p in probs]

        def whole(tl):
            plans = [_plan_for(p, dtype, tl[i], spans[i]) for i, p in enumerate(probs)]
            return min(time_batch(plans, probs, n_steps, reps=2) for _ in range(2))

        cur = whole(tiles)
        order = sorted(classes, key=lambda c: -sum(probs[i].M for i in classes[c]))
        for c in [c for _ in range(sweeps) for c in order]:
            for sh in shortlists[c]:
                if sh == report[c][0]:
                    continue
                trial = list(tiles)
                for i in classes[c]:
                    trial[i] = sh
                fix_unfused(trial)
                tt = whole(trial)
                if log:
                    log(f"refine class {c}: {sh[0]}x{sh[1]} {tt:.3f} ms (best {cur:.3f} ms)")
                if tt < cur:
                    cur, tiles = tt, trial
                    report[c] = (sh, report[c][1])
    return tiles, spans, report


def batch_plans(probs, dtype=torch.float32, tiles=None, spans=None):
    """Plans of a batch: the given (or least-work) tile shapes and spans."""
    spans = spans or [batch_span(p, dtype) for p in probs]
    out = []
    for i, p in enumerate(probs):
        tile = tiles[i] if tiles else None
        if tile is None:
            cand = _candidates(p, dtype, spans[i])
            tile = min(cand, key=cand.get)
        out.append(_plan_for(p, dtype, tile, spans[i]))
    return out
