#!/usr/bin/env python3
"""Benchmark of the RSWR hot path on one MI355X.

One step = one whole RSWR solve (Wei & Zhao, arXiv 2203.10477, Sec. 2.6 redo
loop: predict -> select -> update per span) of the large plain workload:
2^24 nodes on [0,1], 4096 windows, overlap 64 grid intervals, Courant 0.9,
span 35 (the Waveform Time Span Theorem, Eq. (10)), 2*10^4 steps, FP32,
Ricker source on the left end, at rest.  Inputs (initial state, sources) are
resident in HBM before the timed region; each step restores the initial state
with a device copy and runs the recorded graph of all 572 spans.

Prints one JSON line: throughput in grid-point updates per second (GLUPS,
M * n_steps / time), the roofline of the dominant kernel (the fused span
kernel: its average duration inside the timed region, from HIP events around
each solve on the stream it runs on), and the CPU oracle timed on a bounded
sample of the same workload.  Beside it, in the same line: the batched form
(512 problems of uneven size in one recorded graph) and the adjoint form
(forward with span checkpoints plus the backward sweep, FP64), each against
the plain single-problem solve.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/sec (GLUPS) + % HBM roofline, plain vs batched vs adjoint"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# HBM traffic of one span kernel launch on this workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE; see profiles/), and the VALU wave
# instructions of a full 35-step span (SQ_INSTS_VALU), valid only for the
# kernel sources with this SHA-256 prefix.
TRAFFIC = {"kernel_sha": "453a503eb47ed17f", "tile": [64, 33], "bytes": 270410823,
           "valu_insts": 32596057}


def kernel_sha():
    """Hash of the span kernel's sources (the fused kernel and its helpers)."""
    h = hashlib.sha256()
    for name in ("rswr_fused_plain.hip", "rswr_fused_kernel.h", "rswr_fused.h",
                 "rswr_device.h", "rswr_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2203_10477_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def span_bytes(plan, elem):
    """Algorithmic HBM bytes of one span: every window reads its two levels
    and the owned ranges of two levels are written.  Where the plan cannot
    fuse, the predicted fluxes also make a round trip through memory (S
    samples per input end, written once and read once)."""
    lo, hi, _, _ = plan.layout()
    sum_n = int((hi - lo + 1).sum())
    N, M, S = plan.N, plan.M, plan.span
    flux = 0 if plan.info["fused"] else 2 * 2 * (N - 1) * S
    return elem * (2 * sum_n + 2 * M + flux)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, target_s):
    """The CPU oracle on bounded samples of the same workload: its literal
    RSWR (whole-window predict + update, FP32) on all host threads and on
    one, and its plain single-domain leapfrog (one thread: the lower bound of
    any CPU solve).  Each leg runs spans from the state after one warm-up
    span, for about target_s seconds."""
    import oracle
    lay = oracle.layout(prob.M, prob.N, prob.P)
    S = min(lay.span_cone, oracle.span_paper(prob.P, prob.lam, prob.courant_frac))
    fa, fb = prob.sources()
    all_threads = oracle.threads()
    st, _, _ = oracle.rswr(lay, prob.lam, prob.dx, fa, fb, S, span=S, state=prob.state0())

    def leg(run, first_guess):
        t0 = time.perf_counter()
        run(first_guess)
        one = (time.perf_counter() - t0) / first_guess
        spans = max(1, min(500, int(target_s / max(one, 1e-4))))
        t0 = time.perf_counter()
        run(spans)
        dt = time.perf_counter() - t0
        return prob.M * spans * S / dt / 1e9, spans, dt

    rswr_run = lambda k: oracle.rswr(lay, prob.lam, prob.dx, fa, fb, k * S, span=S, state=st,
                                     n0=S)
    single_run = lambda k: oracle.single(prob.M, prob.lam, prob.dx, fa, fb, k * S, state=st,
                                         n0=S)
    all_v, all_spans, all_dt = leg(rswr_run, 1)
    oracle.threads(1)
    try:
        one_v, one_spans, one_dt = leg(rswr_run, 1)
        sd_v, sd_spans, sd_dt = leg(single_run, 1)
    finally:
        oracle.threads(all_threads)
    return {"value": round(all_v, 3), "unit": "GLUPS", "cores": all_threads, "kind": "oracle",
            "sample": f"literal RSWR (whole-window predict + update, FP32) on all {prob.N} "
                      f"windows of the same {prob.M}-node workload, {all_spans} spans of {S} "
                      f"steps after one warm-up span, {all_threads} threads, {all_dt:.1f} s",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "legs": {"rswr_all_threads": {"glups": round(all_v, 3), "threads": all_threads,
                                          "spans": all_spans, "s": round(all_dt, 1)},
                     "rswr_one_thread": {"glups": round(one_v, 3), "threads": 1,
                                         "spans": one_spans, "s": round(one_dt, 1)},
                     "single_domain_one_thread": {"glups": round(sd_v, 3), "threads": 1,
                                                  "spans": sd_spans, "s": round(sd_dt, 1)}}}


def timed(fn, reps):
    """Average milliseconds of fn() over reps runs after one warm-up, with
    HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batched_section(reps):
    """The batched form: 512 problems (2^12..2^18 nodes, 4 to 256 windows,
    overlap 32-128, a in [0.5, 2], 4096 steps, Gaussian pulses), FP32, one
    recorded graph per solve, tile shapes autotuned per size class."""
    import torch
    import paper_2203_10477_amd as rs
    import workloads
    from paper_2203_10477_amd.autotune import autotune_batch, batch_plans
    probs, clamped = workloads.config3()
    t0 = time.perf_counter()
    trials = []

    def log(line):
        if line.startswith("refine"):
            trials.append(line)
        else:
            print("[batched autotune]", line, file=sys.stderr, flush=True)
    tiles, spans, report = autotune_batch(probs, log=log)
    tune_s = time.perf_counter() - t0
    print(f"[batched autotune] {len(trials)} refinement trials in {tune_s:.0f} s",
          file=sys.stderr, flush=True)
    plans = batch_plans(probs, torch.float32, tiles=tiles, spans=spans)
    b = rs.Batch(plans)
    # all states in one buffer, so one fill restores the start (at rest)
    flat = torch.zeros(sum(2 * p.M for p in plans), dtype=torch.float32, device="cuda")
    st, off = [], 0
    for p in plans:
        st.append(flat[off:off + 2 * p.M].view(2, p.M))
        off += 2 * p.M
    fa = [torch.as_tensor(q.fa, dtype=torch.float32, device="cuda") for q in probs]
    fb = [torch.as_tensor(q.fb, dtype=torch.float32, device="cuda") for q in probs]
    ns = [q.n_steps for q in probs]
    ws = torch.empty(b.workspace_bytes(), dtype=torch.uint8, device="cuda")

    def run():
        flat.zero_()
        rs.rswr_batch_solve(b, st, fa, fb, ns, ws)

    zero_ms = timed(flat.zero_, reps)
    ms = timed(run, reps) - zero_ms
    upd = sum(q.M * q.n_steps for q in probs)
    # node-steps the tiles compute (every window recomputes its overlaps, and
    # a tile's cut ends are not stored) over the useful updates
    computed = sum(p.info["n_tiles"] * p.info["tile_threads"] * p.info["tile_per_thread"] *
                   q.n_steps for p, q in zip(plans, probs))
    nbytes = 0
    for p, q in zip(plans, probs):
        lo, hi, _, _ = p.layout()
        K = -(-q.n_steps // p.span)
        nbytes += 4 * K * (2 * int((hi - lo + 1).sum()) + 2 * p.M)
    return {"workload": "512 FP32 problems, 2^12..2^18 nodes (log-uniform), 4..256 windows, "
                        "overlap 32-128, a in [0.5,2], 4096 steps, Gaussian pulses",
            "value": round(upd / (ms * 1e-3) / 1e9, 2), "unit": "GLUPS", "ms": round(ms, 3),
            "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "computed_over_useful": round(computed / upd, 3),
            "algorithmic_bytes": nbytes, "nodes": sum(q.M for q in probs),
            "rounds": max(-(-q.n_steps // s) for q, s in zip(probs, spans)),
            "windows_clamped": clamped, "autotune_s": round(tune_s, 1),
            "shapes": {str(c): f"{v[0][0]}x{v[0][1]}" for c, v in report.items()}}


def plain_2p20_section(reps):
    """The 2^20-node case (64 windows, overlap 64, span 35, 10^4 steps,
    Ricker source) in FP64 and FP32: the whole solve, tile autotuned on one
    span, span by span in one recorded graph; beside it the same plan as
    one launch for the whole loop.  GLUPS and the fraction of the HBM
    roofline of the algorithmic bytes of the whole solve."""
    import numpy as np
    import torch
    import paper_2203_10477_amd as rs
    import workloads
    from paper_2203_10477_amd.autotune import autotune
    out = {}
    for name, npdt, dtype, elem in (("fp64", np.float64, torch.float64, 8),
                                    ("fp32", np.float32, torch.float32, 4)):
        prob = workloads.config2(npdt)
        tile, _ = autotune(prob.M, prob.N, prob.P, dtype=dtype, reps=5)
        fa = torch.as_tensor(prob.sources()[0], device="cuda")
        fb = torch.as_tensor(prob.sources()[1], device="cuda")
        st = torch.zeros(2, prob.M, dtype=dtype, device="cuda")
        zero_ms = timed(lambda: st.zero_(), reps)
        res = {}
        for form, one in (("span_by_span", False), ("one_launch", True)):
            plan = rs.Plan(prob.M, prob.N, prob.P, dtype=dtype, tile=tile, one_launch=one)
            ws = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device="cuda")
            ms = timed(lambda: (st.zero_(), rs.rswr_solve(plan, st, fa, fb, prob.n_steps,
                                                           workspace=ws)), reps) - zero_ms
            if not torch.isfinite(st).all():
                raise RuntimeError(f"non-finite state after the 2^20-node {name} {form} solve")
            K = -(-prob.n_steps // plan.span)
            nbytes = span_bytes(plan, elem) * K
            res[form] = {"glups": round(prob.M * prob.n_steps / (ms * 1e-3) / 1e9, 2),
                         "ms": round(ms, 3),
                         "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[name] = {"tile": list(tile), "span": plan.span, "spans": K,
                     "algorithmic_bytes_per_span": span_bytes(plan, elem), **res}
    prob = workloads.config2(np.float64)
    return {"workload": f"plain RSWR {prob.M} nodes, {prob.N} windows, overlap {prob.P}, "
                        f"{prob.n_steps} steps, Ricker", **out}


def spot_check_section(plan32, prob, fa, fb):
    """FP64 spot check of the large FP32 run on 1% of its spans: at span
    boundaries k = 0, 100, ..., the run's own FP32 state (the solve
    restarted at level k S gives the run's bits) is advanced one span in FP32
    and, from the same state and the same FP32 boundary samples, in FP64 on
    the GPU (the FP64 span kernel, bitwise equal to the oracle's FP64 span
    in the tests); the relative L2 difference of the two results."""
    import torch
    import paper_2203_10477_amd as rs
    S = plan32.span
    n = prob.n_steps
    K = -(-n // S)
    plan64 = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float64)
    fa64, fb64 = fa.double(), fb.double()
    st = torch.zeros(2, prob.M, dtype=torch.float32, device="cuda")
    lev, errs = 0, {}
    for k in range(0, K, 100):
        if k * S > lev:
            rs.rswr_solve(plan32, st, fa, fb, k * S - lev, n0=lev)
            lev = k * S
        one = min(S, n - lev)
        o32 = rs.rswr_span(plan32, st, fa, fb, lev, span=one)
        o64 = rs.rswr_span(plan64, st.double(), fa64, fb64, lev, span=one)
        d = (o32.double() - o64).norm() / o64.norm().clamp_min(1e-300)
        errs[k] = float(d.item())
    return {"spans_checked": list(errs), "max_rel_l2": max(errs.values()),
            "rel_l2": {str(k): v for k, v in errs.items()}, "bound": 1e-5,
            "ok": max(errs.values()) <= 1e-5}


def stream_copy_gbs(n_bytes=4 << 30, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of n_bytes, read +
    write bytes per second."""
    import torch
    a = torch.empty(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    ms = timed(lambda: b.copy_(a), reps)
    del a, b
    return round(2 * n_bytes / (ms * 1e-3) / 1e9, 1)


def adjoint_section(reps):
    """The adjoint form: 2^18 nodes, 128 windows, overlap 64, FP64, 8192 steps,
    16 receivers; the forward solve keeping span checkpoints, then the
    backward sweep giving dJ/df_A and dJ/da; against the plain FP64 solve of
    the same problem.  The tile shape is tuned on the form itself (forward
    with checkpoints + backward sweep, each shape timed once after a warm-up)."""
    import numpy as np
    import torch
    import paper_2203_10477_amd as rs
    import workloads
    from paper_2203_10477_amd.autotune import kernel_shapes
    prob = workloads.config4()
    fa_np, fb_np = prob.sources()
    fa = torch.as_tensor(fa_np, device="cuda")
    fb = torch.as_tensor(fb_np, device="cuda")
    st = torch.zeros(2, prob.M, dtype=torch.float64, device="cuda")
    n = prob.n_steps
    rec = prob.rec
    g = np.random.default_rng(7)
    gtr = torch.as_tensor(g.standard_normal((len(rec), n)), device="cuda")

    def setup(tile):
        plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float64, tile=tile)
        ws = torch.empty(plan.workspace_bytes(len(rec)), dtype=torch.uint8, device="cuda")
        return plan, ws

    ck = None
    tune = {}
    for th, pt, fp64_ok in kernel_shapes():
        if not fp64_ok or th * pt > 1024:
            continue
        try:
            plan, ws = setup((th, pt))
        except rs.RSWRError:
            continue
        ck = plan.checkpoint_buffer(n)

        def both():
            st.zero_()
            rs.rswr_solve(plan, st, fa, fb, n, receivers=rec, checkpoints=ck, workspace=ws)
            rs.rswr_solve_adjoint(plan, ck, fa, fb, n, rec, gtr)
        tune[(th, pt)] = timed(both, 1)
    tile = min(tune, key=tune.get)
    plan, ws = setup(tile)
    ck = plan.checkpoint_buffer(n)

    plain_ms = timed(lambda: (st.zero_(), rs.rswr_solve(plan, st, fa, fb, n, workspace=ws)),
                     reps)
    fwd_ms = timed(lambda: (st.zero_(), rs.rswr_solve(plan, st, fa, fb, n, receivers=rec,
                                                      checkpoints=ck, workspace=ws)), reps)
    adj_ms = timed(lambda: rs.rswr_solve_adjoint(plan, ck, fa, fb, n, rec, gtr), reps)
    zero_ms = timed(lambda: st.zero_(), reps)
    upd = prob.M * n / 1e9
    return {"workload": f"{prob.M} nodes, {prob.N} windows, overlap {prob.P}, span "
                        f"{plan.span}, {n} steps, FP64, {len(rec)} receivers",
            "plain_fp64_glups": round(upd / ((plain_ms - zero_ms) * 1e-3), 2),
            "forward_with_checkpoints_glups": round(upd / ((fwd_ms - zero_ms) * 1e-3), 2),
            "adjoint_sweep_glups": round(upd / (adj_ms * 1e-3), 2),
            "forward_plus_adjoint_glups": round(upd / ((fwd_ms - zero_ms + adj_ms) * 1e-3), 2),
            "ms": {"plain": round(plain_ms - zero_ms, 3), "forward": round(fwd_ms - zero_ms, 3),
                   "adjoint": round(adj_ms, 3)},
            "tile": list(tile),
            "tune_ms": {f"{a}x{b}": round(v, 2) for (a, b), v in tune.items()},
            "checkpoint_bytes": ck.numel() * 8}


def sources_section(reps, tile):
    """The pulse-source form: the large case (2^24 nodes, 4096 windows,
    overlap 64, 2*10^4 steps, FP32) with one Ricker pulse source in each of
    its 4096 windows, the setting of the paper's experiments (N pulse
    sources for N sub-domains); against the same solve without them."""
    import numpy as np
    import torch
    import paper_2203_10477_amd as rs
    import workloads
    prob = workloads.config5(np.float32)
    nodes, amp = workloads.pulse_sources(prob.M, prob.N, prob.n_steps, workloads.rng(6))
    amp_d = torch.as_tensor(amp.astype(np.float32), device="cuda")
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32, tile=tile,
                   sources=(nodes, amp_d))
    fa_np, fb_np = prob.sources()
    fa = torch.as_tensor(fa_np, device="cuda")
    fb = torch.as_tensor(fb_np, device="cuda")
    st = torch.zeros(2, prob.M, dtype=torch.float32, device="cuda")
    ws = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device="cuda")
    n = prob.n_steps
    ms = timed(lambda: (st.zero_(), rs.rswr_solve(plan, st, fa, fb, n, workspace=ws)), reps)
    zero_ms = timed(lambda: st.zero_(), reps)
    if not torch.isfinite(st).all():
        raise RuntimeError("non-finite state after the pulse-source solve")
    lo, hi = plan.info["tile_threads"], plan.info["tile_per_thread"]
    return {"workload": f"{prob.M} nodes, {prob.N} windows, overlap {prob.P}, span "
                        f"{plan.span}, {n} steps, FP32, {len(nodes)} pulse sources",
            "glups": round(prob.M * n / ((ms - zero_ms) * 1e-3) / 1e9, 2),
            "ms": round(ms - zero_ms, 3), "n_src": len(nodes), "tile": [lo, hi]}


def quiet_section(reps, tile=None):
    """The adaptive (QUIET) select of Sec. 2.6 on the large case (2^24 nodes,
    4096 windows, overlap 64, 2*10^4 steps, FP32, Ricker source at X_A):
    every span chosen on the device inside one recorded graph (predict ->
    select -> update per span, the two-launch kernels; spans from the light-
    cone limit up to its double while the overlaps are quiet).  Against the
    FIXED plan on the same two-launch kernels (span 35) and the FIXED fused
    solve (tile `tile`, else the plan's default)."""
    import math
    import numpy as np
    import torch
    import paper_2203_10477_amd as rs
    import workloads
    prob = workloads.config5(np.float32)
    fa_np, fb_np = prob.sources()
    fa = torch.as_tensor(fa_np, device="cuda")
    fb = torch.as_tensor(fb_np, device="cuda")
    n = prob.n_steps
    st = torch.zeros(2, prob.M, dtype=torch.float32, device="cuda")
    zero_ms = timed(lambda: st.zero_(), reps)
    out = {}
    plans = {"quiet": rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32,
                              span_mode=rs.QUIET),
             "fixed_two_launch": rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32,
                                         fuse=False),
             "fixed_fused": rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32,
                                    tile=tile)}
    for name, plan in plans.items():
        ws = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device="cuda")
        ms = timed(lambda: (st.zero_(), rs.rswr_solve(plan, st, fa, fb, n, workspace=ws)),
                   reps) - zero_ms
        if not torch.isfinite(st).all():
            raise RuntimeError(f"non-finite state after the {name} solve")
        out[name] = {"glups": round(prob.M * n / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 3),
                     "span": plan.span, "tile": [plan.info["tile_threads"],
                                                 plan.info["tile_per_thread"]]}
        del ws
    q = plans["quiet"]
    out["quiet"]["rounds_recorded"] = math.ceil(n / min(q.info["span_cone"], q.span))
    return {"workload": f"{prob.M} nodes, {prob.N} windows, overlap {prob.P}, "
                        f"{n} steps, FP32, Ricker at X_A", **out}


def adjoint_batch_section(tile, group=16):
    """The large case's adjoint batch: 64 adjoint solves of the 2^24-node,
    4096-window, overlap-64, 2*10^4-step FP32 problem, each driven by its own
    random Ricker source at X_A, 16 receivers on nodes the wave reaches, a
    random dJ/dtrace; checkpoints chunked (one state per segment of about
    sqrt(572) spans, each segment recomputed in the backward sweep), `group`
    problems per launch.  Timed once after one untimed call (which records
    the graph).  Rate: forward updates of the batch (64 M n_steps) per
    second of the whole call (forward pass, recomputation and backward
    sweep)."""
    import numpy as np
    import torch
    import paper_2203_10477_amd as rs
    import workloads
    prob = workloads.config5(np.float32)
    n, n_prob = prob.n_steps, 64
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=torch.float32, tile=tile)
    fa = torch.as_tensor(workloads.adjoint_batch_sources(prob.M, n, n_prob),
                         dtype=torch.float32, device="cuda")
    fb = torch.zeros_like(fa)
    g = workloads.rng(56)
    rec = workloads.receivers(g, 16, min(prob.M - 2, int(0.8 * 0.9 * n)))
    gtr = torch.as_tensor(g.standard_normal((n_prob, len(rec), n)), dtype=torch.float32,
                          device="cuda")
    ws_b = ctypes.c_size_t()
    rs._check(rs.lib().rswr_adjoint_batch_workspace_size(plan.handle, n, len(rec), group, 0,
                                                         ctypes.byref(ws_b)),
              "rswr_adjoint_batch_workspace_size")
    ws = torch.empty(ws_b.value, dtype=torch.uint8, device="cuda")
    run = lambda: rs.rswr_solve_adjoint_batch(plan, fa, fb, n, rec, gtr, group=group,
                                              workspace=ws)
    ms = timed(run, 1)
    ga, gb, gl = run()
    torch.cuda.synchronize()
    if not (torch.isfinite(ga).all() and torch.isfinite(gl).all()):
        raise RuntimeError("non-finite gradients in the adjoint batch")
    upd = n_prob * prob.M * n / 1e9
    K = -(-n // plan.span)
    return {"workload": f"{n_prob} adjoint solves of {prob.M} nodes, {prob.N} windows, "
                        f"overlap {prob.P}, span {plan.span}, {n} steps, FP32, "
                        f"{len(rec)} receivers, Ricker sources",
            "glups": round(upd / (ms * 1e-3), 2), "s": round(ms / 1e3, 3),
            "group": group, "seg_spans": int(np.ceil(np.sqrt(K))),
            "workspace_gb": round(ws_b.value / 1e9, 1),
            "tile": [plan.info["tile_threads"], plan.info["tile_per_thread"]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-reps", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, adjoint, pulse-source, adjoint-batch and "
                         "QUIET sections")
    ap.add_argument("--tile", default="", help="threads x nodes-per-lane, e.g. 320x13 "
                    "(default: autotuned)")
    ap.add_argument("--section", choices=("batched", "adjoint", "sources", "adjoint_batch",
                                          "quiet", "plain_2p20"),
                    default=None,
                    help="run one of the other forms alone and print its figures "
                         "(for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2203_10477_amd as rs
    import workloads

    from paper_2203_10477_amd.autotune import autotune

    if args.section:
        torch.cuda.set_device(0)
        reps = max(1, args.steps)
        if args.section == "batched":
            out = batched_section(reps)
        elif args.section == "adjoint":
            out = adjoint_section(reps)
        elif args.section == "adjoint_batch":
            tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
            out = adjoint_batch_section(tile)
        elif args.section == "quiet":
            tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
            out = quiet_section(reps, tile)
        elif args.section == "plain_2p20":
            out = plain_2p20_section(reps)
        else:
            tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
            out = sources_section(reps, tile)
        print(json.dumps({"section": args.section, **out}), flush=True)
        return

    dev = "cuda:0"
    torch.cuda.set_device(0)
    prob = workloads.config5(np.float32)
    dtype = torch.float32
    if args.tile:
        tile, tune = tuple(int(v) for v in args.tile.split("x")), {}
    else:
        tile, tune = autotune(prob.M, prob.N, prob.P, dtype=dtype, reps=5)
    plan = rs.Plan(prob.M, prob.N, prob.P, dtype=dtype, tile=tile)
    S = plan.span
    fa_np, fb_np = prob.sources()
    fa = torch.as_tensor(fa_np, device=dev)
    fb = torch.as_tensor(fb_np, device=dev)
    st0 = torch.as_tensor(prob.state0(), device=dev)
    st = st0.clone()
    ws = torch.empty(plan.workspace_bytes(0), dtype=torch.uint8, device=dev)

    # each step: restore the initial state, then the solve (one recorded
    # graph of all span launches); events around each solve give the span
    # kernel's average duration inside the timed region
    marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]

    def step(mark=None):
        st.copy_(st0)
        if mark:
            mark[0].record()
        rs.rswr_solve(plan, st, fa, fb, prob.n_steps, workspace=ws)
        if mark:
            mark[1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        step(marks[k])
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    ev_ms_step = ev0.elapsed_time(ev1) / args.steps
    solve_ms = sum(a.elapsed_time(b) for a, b in marks)
    glups = prob.M * prob.n_steps / (ms_step * 1e-3) / 1e9
    if not torch.isfinite(st).all():
        raise RuntimeError("non-finite state after the benchmark solve")

    # dominant kernel: the span kernel (one launch per span, all windows).
    # Its average duration in the timed region: solve time / launches.
    n_spans = -(-prob.n_steps // S)
    span_us = solve_ms * 1e3 / (args.steps * n_spans)
    fused = bool(plan.info["fused"])

    # The same kernel on a busy field: R spans from a smooth state that is
    # nonzero everywhere (the Ricker run is mostly at rest), timed the same
    # way; R even, so the recorded graph holds the span launches only.
    g = np.random.default_rng(1)
    sm0 = torch.as_tensor(workloads.smooth_state(prob.M, g, shift=prob.lam * prob.dx),
                          dtype=dtype, device=dev)
    R = max(2, args.kernel_reps - args.kernel_reps % 2)
    if R * S > prob.n_steps:
        raise ValueError("kernel-reps too large for the source length")
    sm = sm0.clone()
    rs.rswr_solve(plan, sm, fa, fb, R * S, workspace=ws)  # records the graph
    busy = []
    for _ in range(3):  # the median of three replays (busy data varies more)
        sm.copy_(sm0)
        torch.cuda.synchronize()
        ev0.record()
        rs.rswr_solve(plan, sm, fa, fb, R * S, workspace=ws)
        ev1.record()
        torch.cuda.synchronize()
        busy.append(ev0.elapsed_time(ev1) * 1e3 / R)
    busy_us = sorted(busy)[1]
    nbytes = span_bytes(plan, 4)
    achieved = nbytes / (span_us * 1e-6) / 1e9
    sha = kernel_sha()
    measured = (TRAFFIC["kernel_sha"] == sha and
                [plan.info["tile_threads"], plan.info["tile_per_thread"]] == TRAFFIC["tile"])
    traffic = TRAFFIC["bytes"] if measured else None
    # VALU wave instructions per wave and step (counter pass of the same
    # sources and tile; 8192 waves, 35 steps)
    valu_wave_step = (round(TRAFFIC["valu_insts"] / (plan.info["n_tiles"] * S), 1)
                      if measured else None)
    kname = ("k_fused (predict + update of one span, all windows, one launch)" if fused
             else "k_predict + k_update (one span, all windows)")

    line = {
        "metric": METRIC, "value": round(glups, 2), "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain RSWR {prob.M} nodes, {prob.N} windows, overlap "
                               f"{prob.P}, span {S}, {prob.n_steps} steps, FP32, Ricker",
                   "n_points": prob.M, "n_sub": prob.N, "overlap": prob.P, "span": S,
                   "n_steps": prob.n_steps, "n_spans": n_spans,
                   "tile": [plan.info["tile_threads"], plan.info["tile_per_thread"]],
                   "n_tiles": plan.info["n_tiles"],
                   "autotune_us": {f"{a}x{b}": round(v, 1) for (a, b), v in tune.items()}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kname,
                     "valu_insts": TRAFFIC["valu_insts"] if measured else None,
                     "valu_insts_per_wave_step": valu_wave_step,
                     "avg_us": round(span_us, 2), "algorithmic_bytes": nbytes,
                     "busy_field_avg_us": round(busy_us, 2),
                     "busy_field_frac": round(nbytes / (busy_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "step": {"event_ms_per_step": round(ev_ms_step, 4), "fused": fused,
                 "computed_over_useful": round(plan.info["n_tiles"] * plan.info["tile_threads"] *
                                               plan.info["tile_per_thread"] / prob.M, 3),
                 "hbm_frac_whole_step": round(nbytes * n_spans / (ms_step * 1e-3)
                                              / 1e9 / HBM_PEAK_GBS, 4)},
    }
    line["fp64_spot_check"] = spot_check_section(plan, prob, fa, fb)
    line["roofline"]["measured_copy_gbs"] = stream_copy_gbs()
    if not args.no_forms:
        line["plain_2p20"] = plain_2p20_section(max(1, args.steps))
        line["batched"] = batched_section(max(1, args.steps))
        line["batched"]["vs_plain"] = round(line["batched"]["value"] / glups, 4)
        # the same ratio per computed node-step
        line["batched"]["vs_plain_computed"] = round(
            line["batched"]["value"] * line["batched"]["computed_over_useful"] /
            (glups * line["step"]["computed_over_useful"]), 4)
        line["adjoint"] = adjoint_section(max(1, args.steps))
        line["sources"] = sources_section(max(1, args.steps), tile)
        line["sources"]["vs_plain"] = round(line["sources"]["glups"] / glups, 4)
        line["adjoint_batch"] = adjoint_batch_section(tile)
        line["adjoint_batch"]["vs_plain"] = round(line["adjoint_batch"]["glups"] / glups, 4)
        line["quiet"] = quiet_section(max(1, args.steps), tile)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
