"""Host logic of the serving loop: range allocation and the seeded request trace (CPU)."""
import math

import numpy as np
import pytest

from paper_2006_06775_amd.serve import RangeAllocator, box_reserve, cube_edge, make_trace


def test_allocator_first_fit_alignment_and_coalescing():
    a = RangeAllocator(10 * 1024, align=1024)
    r1 = a.alloc(1500)
    r2 = a.alloc(1)
    r3 = a.alloc(3000)
    assert r1 == (0, 2048) and r2 == (2048, 1024) and r3 == (3072, 3072)
    assert a.alloc(5000) is None  # only 4096 left
    a.release(*r2)
    assert a.alloc(1024) == (2048, 1024)  # first fit reuses the hole
    a.release(2048, 1024)
    a.release(*r1)
    a.release(*r3)
    assert a.free == [(0, 10 * 1024)] and a.free_total() == 10 * 1024


def test_allocator_random_never_overlaps():
    rng = np.random.default_rng(0)
    a = RangeAllocator(1 << 20, align=1024)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            k = rng.integers(len(live))
            a.release(*live.pop(k))
        else:
            r = a.alloc(int(rng.integers(1, 60000)))
            if r is not None:
                assert r[0] % 1024 == 0 and r[0] + r[1] <= 1 << 20
                for s, l in live:
                    assert r[0] + r[1] <= s or s + l <= r[0]
                live.append(r)
        assert a.free_total() + sum(l for _, l in live) == 1 << 20


def test_trace_is_seeded_and_in_range():
    t1 = make_trace(512, seed=0, rate=50.0)
    t2 = make_trace(512, seed=0, rate=50.0)
    assert [(r.arrival, r.n, r.steps) for r in t1] == [(r.arrival, r.n, r.steps) for r in t2]
    ns = np.array([r.n for r in t1])
    st = np.array([r.steps for r in t1])
    assert ns.min() >= 1000 and ns.max() <= 2_000_000 and st.min() >= 10 and st.max() <= 100
    # log-uniform: the log of n is roughly uniform
    ln = np.log(ns)
    assert abs(ln.mean() - 0.5 * (math.log(1e3) + math.log(2e6))) < 0.4
    gaps = np.diff([r.arrival for r in t1])
    assert abs(gaps.mean() - 1 / 50.0) < 0.2 / 50.0
    assert t1[0].arrival == 0.0


def test_box_reserve_covers_the_cube():
    for n in (1000, 4096, 2_000_000):
        per = round(box_reserve(n, 15.0) ** (1 / 3))
        assert per * 15.0 >= cube_edge(n) + 3 * 15.0


def test_tune_pick_and_plan_lookup():
    from paper_2006_06775_amd import serve, tune
    table = {1000: {1.0: 3e-9, 1.2: 2e-9, 1.4: 2e-9}, 100_000: {1.0: 1e-9, 1.2: 1.5e-9, 1.4: 2e-9}}
    best = tune.pick(table)
    assert best == {1000: 1.2, 100_000: 1.0}  # ties go to the smaller factor
    plan = tune.BoxPlan(15.0, best, table)
    assert plan.box_for(900) == 15.0 * 1.2 and plan.box_for(5000) == 15.0 * 1.2
    assert plan.box_for(20_000) == 15.0 and plan.box_for(3_000_000) == 15.0
    assert serve.box_edge(plan, 900) == 18.0 and serve.box_edge(15.0, 900) == 15.0
    assert tune.fixed(1.0).box_for(123456) == 15.0
    # the work split: the default unless another is faster by more than 2 %
    assert tune.pick_cap({4096: 0.99e-9, 8192: 1.0e-9}) == 8192
    assert tune.pick_cap({4096: 0.97e-9, 8192: 1.0e-9}) == 4096
    assert tune.pick_cap({2048: 1.0e-9, 16384: 2e-9}) == 2048  # default not measured
    # one workgroup per tile (-1) competes like any other split
    assert tune.pick_cap({-1: 0.145e-9, 8192: 0.187e-9, 32768: 0.146e-9}) == -1
    assert tune.pick_cap({-1: 0.186e-9, 8192: 0.187e-9}) == 8192
    assert tune.pick_cap({-1: 0.1453e-9, 8192: 0.187e-9, 32768: 0.145e-9}) == -1  # near-tie: one per tile
    assert tune.pick_cap({-1: 0.16e-9, 8192: 0.187e-9, 32768: 0.145e-9}) == 32768
    assert -1 in tune.GRID_CAPS
    summary = tune.BoxPlan(15.0, {1000: 1.0}, grid_cap=-1, split_table={-1: 1e-10, 8192: 2e-10}).summary()
    assert summary["grid_cap"] == -1 and set(summary["split_ns_per_agent_update"]) == {"-1", "8192"}
