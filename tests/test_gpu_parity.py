"""GPU parity: the HIP search through the C ABI against the oracle, element by
element (match count, canonical state count, sorted match rows)."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import graphs as G
import oracle
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)   # any launch ends within a minute
    yield c
    c.close()


class Runner:
    def __init__(self, ctx):
        self.ctx = ctx
        self.tcache = {}

    def target(self, T):
        key = id(T)
        if key not in self.tcache:
            self.tcache[key] = (T, self.ctx.load_target(T))
        return self.tcache[key][1]

    def run(self, P, T, mode, labelled, rows=True, cap_rows=1 << 20, allow=(sge.OK,)):
        th = self.target(T)
        ph = self.ctx.load_pattern(P)
        try:
            self.ctx.set_mode(mode)
            self.ctx.set_labelled(labelled)
            if rows:
                res, r = self.ctx.enumerate(th, ph, P.n, cap_rows=cap_rows, allow=allow)
            else:
                res, r = self.ctx.count(th, ph, allow=allow), None
        finally:
            self.ctx.unload_pattern(ph)
        return res, r


@pytest.fixture(scope="module")
def run(ctx):
    return Runner(ctx)


def _sorted(rows):
    rows = np.asarray(rows, dtype=np.uint32)
    return rows[np.lexsort(rows.T[::-1])] if rows.shape[0] > 1 else rows


def check(run, P, T, mode, labelled, name=""):
    _note(f"case {name} k={P.n} n={T.n} mode={mode} labelled={labelled}")
    want = oracle.run(P, T, mode, labelled, rows=True)
    res, rows = run.run(P, T, mode, labelled)
    assert res.status == sge.OK
    assert res.matches == want["matches"], name
    assert res.states == want["states"], name
    if P.n:
        assert np.array_equal(_sorted(rows), _sorted(want["rows"])), name
    return res, want


@pytest.mark.parametrize("seed", range(40))
def test_tiny_random(run, seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(2, 12))
    k = int(g.integers(1, min(6, n) + 1))
    nlab = int(g.integers(1, 4))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.3, 1.0)), nlab)
    for mode in range(4):
        for labelled in (False, True):
            check(run, P, T, mode, labelled, f"tiny/{seed}")


@pytest.mark.parametrize("n,k", [(8, 3), (9, 5), (12, 4), (7, 7)])
def test_clique_closed_form(run, n, k):
    res, _ = run.run(G.complete(k), G.complete(n), 0, False, rows=False)
    assert res.matches == math.perm(n, k)
    assert res.states == sum(math.perm(n, d) for d in range(1, k + 1))


@pytest.mark.parametrize("name,g,aut", [
    ("K6", G.complete(6), 720), ("C9", G.cycle(9), 18), ("P7", G.path(7), 2), ("K1,5", G.star(5), 120),
    ("K3,4", G.complete_bipartite(3, 4), 144), ("Petersen", G.petersen(), 120), ("Q4", G.hypercube(4), 384),
    ("E5", G.edgeless(5), 120)])
def test_automorphisms(run, name, g, aut):
    for mode in range(4):
        res, _ = run.run(g, g, mode, False, rows=False)
        assert res.matches == aut, (name, mode)


def test_closed_forms_c2_target(run):
    T = synth.c2_target()
    import scipy.sparse as sp
    A = sp.csr_matrix((np.ones(T.m2), T.col, T.row_ptr), shape=(T.n, T.n))
    d = np.asarray(A.sum(1)).ravel().astype(np.int64)
    A2 = A @ A
    tr3 = int(round(A2.multiply(A).sum()))
    tr4 = int(round(A2.multiply(A2).sum()))
    m = int(d.sum()) // 2
    for P, want in [(G.complete(2), 2 * m), (G.path(3), int((d * (d - 1)).sum())),
                    (G.star(3), int((d * (d - 1) * (d - 2)).sum())), (G.complete(3), tr3),
                    (G.cycle(4), tr4 - 2 * int((d * d).sum()) + 2 * m)]:
        for mode in (0, 3):
            res, _ = run.run(P, T, mode, False, rows=False)
            assert res.matches == want


def test_c1_all(run):
    for j in range(synth.C1_COUNT):
        inst = synth.c1_instance(j)
        check(run, inst.pattern, inst.target, inst.mode, True, f"c1/{j}")
        run.tcache.clear()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_c1_rids_modes(run, mode):
    for j in range(0, synth.C1_COUNT, 5):
        inst = synth.c1_instance(j)
        check(run, inst.pattern, inst.target, mode, True, f"c1/{j}")
        run.tcache.clear()


def test_c2_all(run):
    for j in range(synth.C2_COUNT):
        inst = synth.c2_instance(j)
        res, want = check(run, inst.pattern, inst.target, inst.mode, True, f"c2/{j}")
        assert res.matches >= 1


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_c2_rids(run, mode):
    for j in range(0, synth.C2_COUNT, 7):
        inst = synth.c2_instance(j)
        check(run, inst.pattern, inst.target, mode, True, f"c2/{j}")


@pytest.mark.parametrize("lanes,chunk,donate", [(8, 0, True), (16, 1, True), (32, 3, True), (64, 0, True),
                                               (16, 0, False), (16, 1000000, True)])
def test_schedule_independence(run, ctx, lanes, chunk, donate):
    ctx.set_tuning(lanes, chunk, donate)
    try:
        for j in (2, 5, 11, 40):
            inst = synth.c2_instance(j)
            check(run, inst.pattern, inst.target, 0, True, f"c2/{j}/lanes{lanes}")
        inst = synth.c1_instance(3)
        check(run, inst.pattern, inst.target, 3, True, f"c1/3/lanes{lanes}")
    finally:
        ctx.set_tuning(0, 0, 1)


def test_launch_occupancy(run, ctx):
    # busy unit-time is positive and bounded by units x kernel time; steps take
    # a positive mean time
    inst = synth.c2_instance(5)
    res, _ = check(run, inst.pattern, inst.target, 0, True, "c2/5 occupancy")
    kernel_ms, work_ms, done_ms = ctx.last_launch_timing()
    busy, units = ctx.last_launch_occupancy()
    assert units >= 1 and busy > 0
    assert 0 < work_ms <= kernel_ms and 0 < done_ms <= kernel_ms
    assert busy <= units * kernel_ms * 1.001 + 1e-3, (busy, units, kernel_ms)
    assert res.steps >= 1


def test_empty_pattern(run):
    res, rows = run.run(G.edgeless(0), G.complete(4), 0, False)
    assert res.matches == 1 and res.states == 0


def test_pattern_larger_than_target(run):
    for mode in range(4):
        check(run, G.path(6), G.complete(5), mode, False, "k>n")


def test_state_cap(run, ctx):
    inst = synth.c2_instance(2)
    want = oracle.run(inst.pattern, inst.target, 0, True)
    for cap, expect in [(want["states"], sge.OK), (want["states"] - 1, sge.E_ABORTED), (100, sge.E_ABORTED)]:
        ctx.set_state_cap(cap)
        try:
            res, _ = run.run(inst.pattern, inst.target, 0, True, rows=False, allow=(sge.OK, sge.E_ABORTED))
        finally:
            ctx.set_state_cap(0)
        assert res.status == expect, (cap, res)
        if expect == sge.OK:
            assert res.states == want["states"]


def test_row_overflow(run):
    T = G.complete(6)
    P = G.path(3)
    res, rows = run.run(P, T, 0, False, cap_rows=7, allow=(sge.E_OVERFLOW,))
    assert res.status == sge.E_OVERFLOW and res.matches == 120
    full = {tuple(r) for r in oracle.run(P, T, 0, False, rows=True)["rows"].tolist()}
    assert rows.shape == (7, 3) and all(tuple(r) in full for r in rows.tolist())


def test_root_range_shards_sum(run, ctx):
    inst = synth.c2_instance(5)
    want = oracle.run(inst.pattern, inst.target, 0, True, rows=True)
    tot_m = tot_s = 0
    allrows = []
    edges = [0, 700, 1500, 2200, 3000]
    for lo, hi in zip(edges[:-1], edges[1:]):
        ctx.set_root_range(lo, hi)
        try:
            res, rows = run.run(inst.pattern, inst.target, 0, True)
        finally:
            ctx.set_root_range()
        tot_m += res.matches
        tot_s += res.states
        allrows.append(rows)
        shard = oracle.run(inst.pattern, inst.target, 0, True, root_range=(lo, hi))
        assert (res.matches, res.states) == (shard["matches"], shard["states"])
    assert tot_m == want["matches"]
    assert tot_s == want["states"]
    assert np.array_equal(_sorted(np.concatenate(allrows)), _sorted(want["rows"]))


# ---------------------------------------------------------------- single searches planned on the device
# (single searches are planned on the host unless the plan location says otherwise)

@pytest.fixture
def device_plan(ctx):
    ctx.set_plan_location(1)
    yield
    ctx.set_plan_location(-1)


@pytest.mark.parametrize("seed", range(0, 40, 3))
def test_tiny_random_device_plan(run, device_plan, seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(2, 12))
    k = int(g.integers(1, min(6, n) + 1))
    nlab = int(g.integers(1, 4))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.3, 1.0)), nlab)
    for mode in range(4):
        for labelled in (False, True):
            check(run, P, T, mode, labelled, f"tiny/{seed}/device-plan")


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_c2_device_plan(run, device_plan, mode):
    for j in range(0, synth.C2_COUNT, 9):
        inst = synth.c2_instance(j)
        check(run, inst.pattern, inst.target, mode, True, f"c2/{j}/device-plan")


def test_root_range_shards_device_plan(run, ctx, device_plan):
    inst = synth.c2_instance(5)
    for lo, hi in [(0, 700), (700, 1500), (2990, 3000)]:
        ctx.set_root_range(lo, hi)
        try:
            res, _ = run.run(inst.pattern, inst.target, 3, True)
        finally:
            ctx.set_root_range()
        shard = oracle.run(inst.pattern, inst.target, 3, True, root_range=(lo, hi))
        assert (res.matches, res.states) == (shard["matches"], shard["states"])
