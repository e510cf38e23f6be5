"""GPU parity of the batched solve: many problems (different grids, window
counts, overlaps, wave speeds, spans, lengths) advanced in one recorded graph
give bit-identical results to solving each alone, and to the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2203_10477_amd as rs
import workloads
from paper_2203_10477_amd.autotune import autotune_batch, batch_plans

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NP = {torch.float64: np.float64, torch.float32: np.float32}


def say(*a):
    print("[case]", *a, flush=True)


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def lay_of(plan):
    lo, hi, _, _ = plan.layout()
    return oracle.explicit_layout(plan.M, lo, hi)


def run_batch(plans, probs, n_steps, dtype):
    b = rs.Batch(plans)
    st = [torch.zeros(2, p.M, dtype=dtype, device=DEV) for p in plans]
    fa = [dev(q.fa[:n + 1], dtype) for q, n in zip(probs, n_steps)]
    fb = [dev(q.fb[:n + 1], dtype) for q, n in zip(probs, n_steps)]
    rs.rswr_batch_solve(b, st, fa, fb, n_steps)
    torch.cuda.synchronize()
    return [s.cpu().numpy() for s in st], (b, st, fa, fb)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_matches_single_solves_and_oracle(dtype):
    probs, _ = workloads.config3(count=24, n_steps=600, log2_range=(12, 14), tag=33)
    say("batch-24", dtype)
    plans = batch_plans(probs, dtype)
    pattern = [600, 599, 0, 37, 1, 311]
    n_steps = [pattern[i % len(pattern)] for i in range(len(probs))]
    got, (b, st, fa, fb) = run_batch(plans, probs, n_steps, dtype)
    for i, (p, q, n) in enumerate(zip(plans, probs, n_steps)):
        s1 = torch.zeros(2, p.M, dtype=dtype, device=DEV)
        rs.rswr_solve(p, s1, dev(q.fa[:n + 1], dtype), dev(q.fb[:n + 1], dtype), n)
        torch.cuda.synchronize()
        assert np.array_equal(got[i], s1.cpu().numpy()), (i, p.M, p.N, p.span, n)
    # against the oracle's literal RSWR on the smaller problems
    npdt = NP[dtype]
    small = sorted(range(len(probs)), key=lambda i: probs[i].M)[:4]
    for i in small:
        p, q, n = plans[i], probs[i], n_steps[i]
        ref, _, _ = oracle.rswr(lay_of(p), p.info["lambda"], p.info["dx"],
                                q.fa[:n + 1].astype(npdt), q.fb[:n + 1].astype(npdt), n,
                                span=p.span, state=np.zeros((2, p.M), npdt))
        assert np.array_equal(got[i], ref), i
    # a replay of the recorded graph from the same start gives the same states
    for s in st:
        s.zero_()
    rs.rswr_batch_solve(b, st, fa, fb, n_steps)
    torch.cuda.synchronize()
    for i, s in enumerate(st):
        assert np.array_equal(s.cpu().numpy(), got[i]), i


def test_batch_full_recipe_fp32_with_fp64_check():
    """All 512 problems of the batched workload (2^12..2^18 nodes, 4096 steps)
    in one graph: sampled problems bitwise against solving them alone; the
    two smallest within FP32 accuracy of the FP64 oracle (no worse than
    twice the FP32 single-domain solve's own error)."""
    probs, _ = workloads.config3()
    say("batch-512-fp32")
    tiles, spans, _ = autotune_batch(probs, measure=False)
    plans = batch_plans(probs, torch.float32, tiles=tiles, spans=spans)
    n_steps = [q.n_steps for q in probs]
    got, _ = run_batch(plans, probs, n_steps, torch.float32)
    g = np.random.default_rng(5)
    for i in sorted(g.choice(len(probs), 8, replace=False)):
        p, q = plans[i], probs[i]
        s1 = torch.zeros(2, p.M, dtype=torch.float32, device=DEV)
        rs.rswr_solve(p, s1, dev(q.fa, torch.float32), dev(q.fb, torch.float32), q.n_steps)
        torch.cuda.synchronize()
        assert np.array_equal(got[i], s1.cpu().numpy()), i
    for i in sorted(range(len(probs)), key=lambda i: probs[i].M)[:2]:
        p, q = plans[i], probs[i]
        lam, dx = p.info["lambda"], p.info["dx"]
        r64, _ = oracle.single(p.M, lam, dx, q.fa, q.fb, q.n_steps)
        s32, _ = oracle.single(p.M, lam, dx, q.fa.astype(np.float32), q.fb.astype(np.float32),
                               q.n_steps)
        scale = np.linalg.norm(r64)
        assert scale > 0
        e_single = np.linalg.norm(s32.astype(np.float64) - r64) / scale
        e_batch = np.linalg.norm(got[i].astype(np.float64) - r64) / scale
        assert e_batch <= 2 * e_single + 1e-7, (i, e_batch, e_single)
