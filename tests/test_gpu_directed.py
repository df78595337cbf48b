"""GPU parity on directed and edge-labelled graphs (the general problem of
Section 2.1): the CSR search through the C ABI against the oracle, element by
element (matches, canonical states, sorted rows), single and batched."""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import graphs as G
import oracle
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sorted(rows):
    rows = np.asarray(rows, dtype=np.uint32)
    return rows[np.lexsort(rows.T[::-1])] if rows.shape[0] > 1 else rows


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.close()


def check(ctx, P, T, mode, labelled, name=""):
    _note(f"directed case {name} k={P.n} n={T.n} mode={mode} labelled={labelled}")
    want = oracle.run(P, T, mode, labelled, rows=True)
    th = ctx.load_target(T)
    ph = ctx.load_pattern(P)
    try:
        ctx.set_mode(mode)
        ctx.set_labelled(labelled)
        res, rows = ctx.enumerate(th, ph, P.n, cap_rows=1 << 20)
    finally:
        ctx.unload_pattern(ph)
        ctx.unload_target(th)
    assert (res.matches, res.states) == (want["matches"], want["states"]), name
    if P.n:
        assert np.array_equal(_sorted(rows), _sorted(want["rows"])), name


@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_digraphs(ctx, seed):
    g = np.random.default_rng(21000 + seed)
    n = int(g.integers(2, 12))
    k = int(g.integers(1, min(6, n) + 1))
    T = G.random_digraph(g, n, float(g.uniform(0.15, 0.6)), int(g.integers(1, 3)), int(g.integers(1, 4)))
    P = G.random_digraph(g, k, float(g.uniform(0.2, 0.9)), int(g.integers(1, 3)), int(g.integers(1, 4)))
    for mode in range(4):
        for labelled in (False, True):
            check(ctx, P, T, mode, labelled, f"digraph/{seed}")


@pytest.mark.parametrize("seed", range(12))
def test_mixed_and_undirected_edge_labels(ctx, seed):
    g = np.random.default_rng(22000 + seed)
    Tu = G.random_undirected_elabelled(g, int(g.integers(3, 12)), 0.4, 2, 3)
    Pd = G.random_digraph(g, int(g.integers(2, 6)), 0.5, 2, 3)
    Pu = G.random_undirected_elabelled(g, int(g.integers(2, 6)), 0.6, 2, 3)
    Td = G.random_digraph(g, int(g.integers(3, 12)), 0.35, 2, 3)
    for mode in (0, 1, 3):
        for labelled in (False, True):
            check(ctx, Pd, Tu, mode, labelled, f"dir-on-undir/{seed}")
            check(ctx, Pu, Tu, mode, labelled, f"undir-elab/{seed}")
            check(ctx, Pu, Td, mode, labelled, f"undir-on-dir/{seed}")


@pytest.mark.parametrize("n,k", [(6, 3), (9, 4), (12, 5)])
def test_tournament_closed_forms(ctx, n, k):
    import math
    T = G.from_arcs(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    P = G.from_arcs(k, [(i, i + 1) for i in range(k - 1)])
    th, ph = ctx.load_target(T), ctx.load_pattern(P)
    try:
        for mode in range(4):
            ctx.set_mode(mode)
            ctx.set_labelled(False)
            assert ctx.count(th, ph).matches == math.comb(n, k)
    finally:
        ctx.unload_pattern(ph)
        ctx.unload_target(th)


def test_directed_workload_single_searches(ctx):
    for j in range(0, 100, 7):
        inst = synth.c2d_instance(j)
        if inst.labelled:
            check(ctx, inst.pattern, inst.target, inst.mode, inst.labelled, f"c2d/{j}")


def test_directed_workload_batch_vs_golden(ctx):
    with open(os.path.join(GOLDEN, "c2d.json")) as f:
        man = json.load(f)
    insts = [synth.c2d_instance(r["j"], r["attempt"]) for r in man["instances"]]
    th = ctx.load_target(insts[0].target)
    jobs = [(th, ctx.load_pattern(i.pattern), i.mode, i.labelled) for i in insts]
    _note("c2d batch x100")
    try:
        for where in (-1, 0):
            ctx.set_plan_location(where)
            st, res = ctx.batch_run(jobs)
            assert st == sge.OK
            assert res.matches.tolist() == [r["matches"] for r in man["instances"]]
            assert res.states.tolist() == [r["states"] for r in man["instances"]]
    finally:
        ctx.set_plan_location(-1)
        for _, p, _, _ in jobs:
            ctx.unload_pattern(p)
        ctx.unload_target(th)


def test_directed_root_shards(ctx):
    inst = synth.c2d_instance(3)           # unlabelled, directions only
    th, ph = ctx.load_target(inst.target), ctx.load_pattern(inst.pattern)
    try:
        ctx.set_mode(inst.mode)
        ctx.set_labelled(inst.labelled)
        for lo, hi in [(0, 1000), (1000, 2000), (2000, 3000)]:
            ctx.set_root_range(lo, hi)
            r = ctx.count(th, ph)
            w = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled, root_range=(lo, hi))
            assert (r.matches, r.states) == (w["matches"], w["states"])
    finally:
        ctx.set_root_range()
        ctx.unload_pattern(ph)
        ctx.unload_target(th)


def test_general_graphs_refuse_device_plan_and_dense(ctx):
    T = G.from_arcs(4, [(0, 1), (1, 2), (2, 3)])
    P = G.from_arcs(2, [(0, 1)])
    th, ph = ctx.load_target(T), ctx.load_pattern(P)
    try:
        with pytest.raises(sge.SgeError) as e:
            ctx.plan_device(th, ph, 2, 4, sge.RIDS, False)
        assert e.value.code == sge.E_INVAL
        ctx.set_plan_location(1)
        ctx.set_mode(0)
        ctx.set_labelled(False)
        with pytest.raises(sge.SgeError):
            ctx.count(th, ph)
        ctx.set_plan_location(-1)
        ctx.set_tuning(0, 0, 1, 1)        # force the dense kernel
        with pytest.raises(sge.SgeError):
            ctx.count(th, ph)
        ctx.set_tuning(0, 0, 1, -1)
        assert ctx.count(th, ph).matches == 3
    finally:
        ctx.set_plan_location(-1)
        ctx.set_tuning(0, 0, 1, -1)
        ctx.unload_pattern(ph)
        ctx.unload_target(th)
