"""GPU parity of the algorithmic-byte counter (the roofline numerator the
library reports per search) against the oracle's, for both kernel variants:
the CSR search against the oracle's sparse model, the dense-bitset search
against its dense model.  Also: switching the counter off changes no other
result, and the search kernel's HIP-event time agrees with the device clock."""
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

CSR, DENSE = 0, 1


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def manifest(cfg):
    with open(os.path.join(GOLDEN, f"{cfg}.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.set_tuning(0, 0, 1, -1)
    c.close()


def count(ctx, P, T, mode, labelled, kernel, root_range=None):
    th, ph = ctx.load_target(T), ctx.load_pattern(P)
    try:
        ctx.set_tuning(0, 0, 1, kernel)
        ctx.set_mode(mode)
        ctx.set_labelled(labelled)
        if root_range:
            ctx.set_root_range(*root_range)
        return ctx.count(th, ph)
    finally:
        ctx.set_root_range()
        ctx.set_tuning(0, 0, 1, -1)
        ctx.unload_pattern(ph)
        ctx.unload_target(th)


def want_bytes(w, kernel):
    return w["dense_bytes"] if kernel == DENSE else w["alg_bytes"]


@pytest.mark.parametrize("seed", range(24))
def test_tiny_random_both_kernels(ctx, seed):
    g = np.random.default_rng(500 + seed)
    n = int(g.integers(2, 14))
    k = int(g.integers(1, min(6, n) + 1))
    nlab = int(g.integers(1, 4))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.3, 1.0)), nlab)
    _note(f"bytes tiny/{seed} n={n} k={k}")
    for mode in range(4):
        for labelled in (False, True):
            w = oracle.run(P, T, mode, labelled)
            for kernel in (CSR, DENSE):
                r = count(ctx, P, T, mode, labelled, kernel)
                assert (r.matches, r.states) == (w["matches"], w["states"])
                assert r.alg_bytes == want_bytes(w, kernel), (seed, mode, labelled, kernel)


def test_root_ranges_both_kernels(ctx):
    inst = synth.c1_instance(11)
    for mode in (0, 3):
        for lo, hi in [(0, 50), (50, 120), (120, 1000), (300, 400)]:
            w = oracle.run(inst.pattern, inst.target, mode, True, root_range=(lo, hi))
            for kernel in (CSR, DENSE):
                _note(f"bytes c1/11 mode {mode} roots [{lo},{hi}) kernel {kernel}")
                r = count(ctx, inst.pattern, inst.target, mode, True, kernel, (lo, hi))
                assert r.states == w["states"]
                assert r.alg_bytes == want_bytes(w, kernel), (mode, lo, hi, kernel)


def test_multi_component_pattern(ctx):
    """Parentless positions after the first (a pattern of two components)."""
    T = synth.c1_instance(4).target
    P = G.from_edges(5, [(0, 1), (1, 2), (3, 4)], [0, 1, 2, 0, 3])
    for mode in range(4):
        w = oracle.run(P, T, mode, True)
        for kernel in (CSR, DENSE):
            r = count(ctx, P, T, mode, True, kernel)
            assert r.states == w["states"]
            assert r.alg_bytes == want_bytes(w, kernel), (mode, kernel)


def _batch(ctx, cfg, make, want_key, plan_where=-1):
    man = manifest(cfg)
    insts = [make(r["j"], r["attempt"]) for r in man["instances"]]
    tc, jobs = {}, []
    for i in insts:
        if id(i.target) not in tc:
            tc[id(i.target)] = ctx.load_target(i.target)
        jobs.append((tc[id(i.target)], ctx.load_pattern(i.pattern), i.mode, i.labelled))
    try:
        ctx.set_plan_location(plan_where)
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK
        assert res.states.tolist() == [r["states"] for r in man["instances"]]
        assert res.alg_bytes.tolist() == [r[want_key] for r in man["instances"]]
        return res
    finally:
        ctx.set_plan_location(-1)
        for t in tc.values():
            ctx.unload_target(t)
        for j in jobs:
            ctx.unload_pattern(j[1])


@pytest.mark.parametrize("where", [-1, 0])
def test_c2_batch_bytes(ctx, where):
    _note(f"bytes c2 batch, plan {where}")
    _batch(ctx, "c2", synth.c2_instance, "alg_bytes", where)


def test_c1_batch_bytes_dense(ctx):
    _note("bytes c1 batch (dense kernel)")
    ctx.set_tuning(0, 0, 1, DENSE)
    try:
        _batch(ctx, "c1", synth.c1_instance, "dense_bytes")
    finally:
        ctx.set_tuning(0, 0, 1, -1)


def test_c4_batch_bytes(ctx):
    _note("bytes c4 batch x4096")
    _batch(ctx, "c4", synth.c4_instance, "alg_bytes")


def test_c2d_batch_bytes(ctx):
    """Directed, edge-labelled graphs (arcs in both directions, arc labels)."""
    _note("bytes c2d batch")
    _batch(ctx, "c2d", synth.c2d_instance, "alg_bytes")


def test_counting_off_changes_nothing_else(ctx):
    man = manifest("c2")
    insts = [synth.c2_instance(r["j"], r["attempt"]) for r in man["instances"][:30]]
    th = ctx.load_target(insts[0].target)
    jobs = [(th, ctx.load_pattern(i.pattern), i.mode, i.labelled) for i in insts]
    try:
        ctx.set_count_bytes(False)
        st, off = ctx.batch_run(jobs)
        ctx.set_count_bytes(True)
        st2, on = ctx.batch_run(jobs)
        assert st == st2 == sge.OK
        assert off.alg_bytes.tolist() == [0] * len(jobs)
        assert off.states.tolist() == on.states.tolist() == [r["states"] for r in man["instances"][:30]]
        assert off.matches.tolist() == on.matches.tolist()
        assert on.alg_bytes.tolist() == [r["alg_bytes"] for r in man["instances"][:30]]
    finally:
        ctx.set_count_bytes(True)
        for j in jobs:
            ctx.unload_pattern(j[1])
        ctx.unload_target(th)


def test_kernel_event_time(ctx):
    """The HIP events around the search kernel (event nodes of the batch
    graph, plain records for a single search) bracket the kernel: their time
    is at least the device clock's first-block-to-last-wave span and not far
    above it, on every replay of the kept graph."""
    man = manifest("c2")
    insts = [synth.c2_instance(r["j"], r["attempt"]) for r in man["instances"]]
    th = ctx.load_target(insts[0].target)
    jobs = [(th, ctx.load_pattern(i.pattern), i.mode, i.labelled) for i in insts]
    try:
        for rep in range(4):
            st, res = ctx.batch_run(jobs)
            ev = ctx.last_kernel_ms()
            dev = ctx.last_launch_timing()[0]
            _note(f"batch replay {rep}: event {ev:.3f} ms, device clock {dev:.3f} ms; {ctx.last_error()}")
            assert dev > 0 and 0.9 * dev <= ev <= dev + 0.5
        ctx.set_mode(0)
        ctx.set_labelled(True)
        ctx.count(th, jobs[28][1])
        ev, dev = ctx.last_kernel_ms(), ctx.last_launch_timing()[0]
        _note(f"single search: event {ev:.3f} ms, device clock {dev:.3f} ms")
        assert dev > 0 and 0.9 * dev <= ev <= dev + 0.5
    finally:
        for j in jobs:
            ctx.unload_pattern(j[1])
        ctx.unload_target(th)
