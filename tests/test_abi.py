"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every function include/rswr.h declares, and rswr_plan (host only) builds the
decomposition of Sec. 2.2 / Sec. 3 and the span rule of Sec. 2.4 Eq. (10)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest
import torch

import oracle
import paper_2203_10477_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rswr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rswr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = rs.lib()
    names = declared_functions()
    assert "rswr_solve" in names and "rswr_predict" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = rs.lib()
    for code in range(9):
        assert L.rswr_status_string(code)


@pytest.mark.parametrize("M,N,P", [(1001, 2, 20), (4097, 8, 64), (2 ** 16, 64, 32),
                                   (301, 20, 20), (257, 1, 2)])
def test_plan_layout_matches_definition(M, N, P):
    plan = rs.Plan(M, N, P)
    lo, hi, olo, ohi = plan.layout()
    ref = oracle.layout(M, N, P)
    assert np.array_equal(lo, ref.lo) and np.array_equal(hi, ref.hi)
    assert np.array_equal(olo, ref.own_lo) and np.array_equal(ohi, ref.own_hi)
    if N > 1:
        assert plan.info["span_cone"] == ref.span_cone


def test_plan_span_table_golden():
    gold = json.load(open(os.path.join(GOLD, "span_table.json")))
    for P, S in gold["rows"]:
        M = 40 * P + 1
        plan = rs.Plan(M, 4, P)
        assert plan.info["span_paper"] == S
        assert plan.span == min(S, P)
        plan_d = rs.Plan(M, 4, P, courant_frac=None)  # double-precision rule
        assert plan_d.info["span_paper"] == S


def test_plan_golden_layout():
    gold = json.load(open(os.path.join(GOLD, "layout_1001_N2_P20.json")))
    plan = rs.Plan(gold["M"], gold["N"], gold["P"])
    lo, hi, olo, ohi = plan.layout()
    assert list(lo) == gold["lo"] and list(hi) == gold["hi"]
    assert list(olo) == gold["own_lo"] and list(ohi) == gold["own_hi"]
    assert plan.info["span_cone"] == gold["span_cone"] and plan.span == 11


def test_plan_errors():
    with pytest.raises(rs.RSWRError) as e:
        rs.Plan(1001, 2, 21)  # odd overlap
    assert e.value.status == 3
    with pytest.raises(rs.RSWRError) as e:
        rs.Plan(1001, 2, 20, courant=1.2)
    assert e.value.status == 2
    with pytest.raises(rs.RSWRError) as e:
        rs.Plan(1001, 2, 20, span=21)  # beyond the light cone
    assert e.value.status == 4
    with pytest.raises(rs.RSWRError) as e:
        rs.Plan(2, 1, 2)
    assert e.value.status == 1
    with pytest.raises(rs.RSWRError) as e:
        rs.Plan(1001, 2, 20, tile=(96, 3))
    assert e.value.status == 8
    with pytest.raises(rs.RSWRError) as e:
        rs.Plan(101, 60, 20)  # cores narrower than the end-core rule allows
    assert e.value.status == 3


def test_explicit_windows_and_cone():
    lo = [0, 90, 200, 260]
    hi = [110, 230, 290, 399]
    plan = rs.Plan(400, 4, 0, windows=(lo, hi))
    ref = oracle.explicit_layout(400, lo, hi)
    assert plan.info["span_cone"] == ref.span_cone == 20
    l2, h2, ol, oh = plan.layout()
    assert np.array_equal(ol, ref.own_lo) and np.array_equal(oh, ref.own_hi)
    with pytest.raises(rs.RSWRError):
        rs.Plan(400, 4, 0, windows=([0, 120, 100, 260], hi))


def test_quiet_plan_caps_span_at_twice_the_cone():
    plan = rs.Plan(1001, 2, 20, span_mode=rs.QUIET)
    assert plan.info["span"] == 40 and plan.flux_ld >= 40


def test_compute_calls_need_a_gpu_tensor():
    plan = rs.Plan(1001, 2, 20)
    st = torch.zeros(2, 1001, dtype=torch.float64)
    with pytest.raises(TypeError):
        rs.rswr_solve(plan, st, st[0], st[0], 10)


def _fused_by_rule(plan):
    """The fused-span rule from the plan's tiles: fixed span 1..63 and no
    window whose left input lies inside a region (those are the general
    tiles of windows other than the first)."""
    if plan.info["span"] < 1 or plan.span > 63:
        return False
    for _, _, _, _, w, _, _, gen in plan.tiles():
        if gen and w > 0:
            return False
    return True


@pytest.mark.parametrize("args,kw", [
    ((1001, 2, 20), {}),
    ((1 << 24, 4096, 64), {"dtype": torch.float32}),
    ((1 << 20, 64, 64), {}),
    ((301, 20, 20), {}),
    ((4097, 8, 64), {"tile": (128, 8)}),
    ((20001, 16, 64), {"tile": (256, 16)}),
    ((101, 2, 0), {"windows": ([0, 5], [30, 100])}),
    ((2001, 2, 0), {"windows": ([0, 5], [30, 2000])}),
    ((2001, 3, 0), {"windows": ([0, 400, 800], [700, 911, 2000]), "tile": (64, 8)}),
    ((40001, 4, 256), {"span": 40}),
    ((40001, 4, 256), {}),               # span 127 > 63: two launches
])
def test_fused_flag_follows_the_rule(args, kw):
    plan = rs.Plan(*args, **kw)
    assert plan.info["fused"] == int(_fused_by_rule(plan)), (args, kw)
    off = rs.Plan(*args, fuse=False, **kw)
    assert off.info["fused"] == 0


def test_fused_flag_cases():
    assert rs.Plan(1001, 2, 20).info["fused"] == 1
    assert rs.Plan(1 << 24, 4096, 64, dtype=torch.float32).info["fused"] == 1
    assert rs.Plan(1001, 2, 20, span_mode=rs.QUIET).info["fused"] == 0
    # a tile starts at the second window's input end, node 5: its frame
    # holds the Dirichlet node 0
    near = rs.Plan(2001, 2, 0, windows=([0, 5], [30, 2000]))
    assert near.span >= 5 and near.info["fused"] == 1
    assert (near.tiles()[:, 0] == 5).any()
    # an interior left input (a general tile of a narrow window) keeps two
    # launches
    gen = rs.Plan(301, 20, 20)
    assert any(g and w > 0 for *_, w, _, _, g in gen.tiles()) == (gen.info["fused"] == 0)


def test_batch_plan_rejections():
    """A batch takes fused plans of one dtype only (host-side checks)."""
    a = rs.Plan(1001, 2, 20)
    b = rs.Plan(1001, 2, 20, dtype=torch.float32)
    with pytest.raises(rs.RSWRError) as e:
        rs.Batch([a, b])
    assert e.value.status == 1
    two = rs.Plan(1001, 2, 20, fuse=False)
    with pytest.raises(rs.RSWRError) as e:
        rs.Batch([a, two])
    assert e.value.status == 8
    ok = rs.Batch([a, rs.Plan(4097, 8, 64)])
    # one second state buffer per problem plus tables
    assert ok.workspace_bytes() >= 2 * (1001 + 4097) * 8
    assert rs.Batch([]).workspace_bytes() >= 0


def test_batch_recipe_plans_all_fuse():
    """The batched workload's problems: span capped at 63, every plan fused,
    windows at least one overlap wide (cores clamped)."""
    import workloads
    from paper_2203_10477_amd.autotune import autotune_batch, batch_plans
    probs, clamped = workloads.config3()
    assert len(probs) == 512 and clamped > 0
    assert all((p.M - 1) // p.N >= p.P for p in probs)
    tiles, spans, report = autotune_batch(probs, measure=False)
    plans = batch_plans(probs, tiles=tiles, spans=spans)
    assert all(p.info["fused"] for p in plans)
    assert max(spans) == 63 and min(spans) >= 17
    assert len(report) >= 5


def raw_plan(M, N, P, nodes, ld=100, amp_ptr=0x1000, **kw):
    """rswr_plan through the raw C-ABI with interior sources; the sample
    pointer is only stored by the host code, never read here."""
    L = rs.lib()
    d = rs._Desc()
    d.x_a, d.x_b, d.n_points = 0.0, 1.0, M
    d.a, d.courant, d.courant_num, d.courant_den = 1.0, 0.9, 9, 10
    d.n_sub, d.overlap = N, P
    d.dtype = kw.get("dtype", 1)
    d.span_mode = kw.get("span_mode", 0)
    d.no_fuse = kw.get("no_fuse", 0)
    nodes = np.ascontiguousarray(nodes, np.int64)
    d.n_src = len(nodes)
    d.src_node = nodes.ctypes.data
    d.src_amp = amp_ptr
    d.src_ld = ld
    h = ctypes.c_void_p()
    st = L.rswr_plan(ctypes.byref(d), ctypes.byref(h))
    return st, h


def test_source_plan_rules():
    L = rs.lib()
    st, h = raw_plan(4097, 8, 64, [1, 600, 4095])
    assert st == 0
    L.rswr_plan_destroy(h)
    for bad in ([0], [4096], [-3], [5000]):
        st, _ = raw_plan(4097, 8, 64, bad)
        assert st == 1, bad  # RSWR_ERR_INVALID_ARG
    st, _ = raw_plan(4097, 8, 64, [100], amp_ptr=0)
    assert st == 1
    st, _ = raw_plan(4097, 8, 64, [100], ld=0)
    assert st == 1
    # sources need the fused span
    for kw in ({"no_fuse": 1}, {"span_mode": 1}):
        st, _ = raw_plan(4097, 8, 64, [100], **kw)
        assert rs.STATUS[st] == "RSWR_ERR_UNSUPPORTED", kw


def test_courant_fraction_must_match_courant():
    # Eq. (10): 2 S lam < P.  At C = 1 and P = 20 the rule gives S = 9; a
    # stale fraction of 9/10 would give 11.
    assert rs.Plan(1001, 2, 20, courant=1.0).info["span_paper"] == 9
    assert rs.Plan(1001, 2, 20, courant=0.9).info["span_paper"] == 11
    with pytest.raises(rs.RSWRError):
        rs.Plan(1001, 2, 20, courant=1.0, courant_frac=(9, 10))
    with pytest.raises(ValueError):
        rs.ProblemSpec(1001, 2, 20, 100, [3], a_ref=0.0)
