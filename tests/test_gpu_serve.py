"""GPU tests of the server: results alone and in the mix are the same, and
equal to the oracle's; admission by slots and memory."""
from __future__ import annotations

import json
import os
import sys
import time

import pytest

import oracle
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C5_SAMPLE = 48   # the first queries of the serving workload's arrival stream


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def manifest(cfg):
    with open(os.path.join(GOLDEN, f"{cfg}.json")) as f:
        return json.load(f)


def serve_all(ctx, jobs, timeout_s=60.0):
    """Submit every job (retrying while not admissible), poll until all are done."""
    pending = list(enumerate(jobs))
    tickets = {}
    results = {}
    t_end = time.time() + timeout_s
    while (pending or tickets) and time.time() < t_end:
        while pending:
            i, (t, p, mode, lab) = pending[0]
            tk = ctx.serve_submit(t, p, mode, lab)
            if tk is None:
                break
            tickets[tk] = i
            pending.pop(0)
        for tk in list(tickets):
            r = ctx.serve_poll(tk)
            if r is not None:
                results[tickets.pop(tk)] = r
        time.sleep(0.0005)
    assert not pending and not tickets, "server did not finish in time"
    return [results[i] for i in range(len(jobs))]


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.close()


@pytest.mark.parametrize("where", [-1, 1])
def test_serve_c1_matches_oracle_and_alone(ctx, where):
    """where: -1 plans each query on the server's host threads, 1 in the plan
    kernel at the head of its launch."""
    man = manifest("c1")
    insts = [synth.c1_instance(r["j"], r["attempt"]) for r in man["instances"]]
    jobs = [(ctx.load_target(i.target), ctx.load_pattern(i.pattern), i.mode, True) for i in insts]
    ctx.set_plan_location(where)
    ctx.serve_start(32, 1 << 30)
    try:
        _note(f"serve c1 x100, plan {where}")
        mix = serve_all(ctx, jobs)
    finally:
        ctx.serve_stop()
        ctx.set_plan_location(-1)
    for r, w in zip(mix, man["instances"]):
        assert r.status == sge.OK
        assert (r.matches, r.states) == (w["matches"], w["states"])
    ctx.set_mode(0)
    ctx.set_labelled(True)
    for (t, p, _, _), r in list(zip(jobs, mix))[::10]:
        alone = ctx.count(t, p)
        assert (alone.matches, alone.states) == (r.matches, r.states)
    for t, p, _, _ in jobs:
        ctx.unload_pattern(p)
        ctx.unload_target(t)


@pytest.mark.parametrize("where", [-1, 1])
def test_serve_c5_sample_alone_and_mix(ctx, where):
    """The serving workload's first queries (resident 5k-20k-node targets,
    RI-DS-SI-FC, state cap 1e7) against the oracle, in the mix and alone,
    planned on the host (-1) or on the device (1)."""
    man = manifest("c5")
    sample = man["instances"][:C5_SAMPLE]
    _note("serve c5: loading 50 resident targets")
    targets = [synth.c5_target(t) for t in range(synth.C5_TARGETS)]
    th = [ctx.load_target(T) for T in targets]
    jobs, pats = [], []
    for r in sample:
        t, P, _ = synth.c5_query(r["j"], targets)
        assert t == r["target"]
        pats.append(P)
        jobs.append((th[t], ctx.load_pattern(P), sge.RIDS_SI_FC, True))
    ctx.set_state_cap(man["state_cap"])
    ctx.set_plan_location(where)
    try:
        ctx.serve_start(64, 4 << 30)
        try:
            _note(f"serve c5: {len(jobs)} queries in the mix, plan {where}")
            mix = serve_all(ctx, jobs)
        finally:
            ctx.serve_stop()
        ctx.set_mode(sge.RIDS_SI_FC)
        ctx.set_labelled(True)
        for (t, p, _, _), r, w in zip(jobs, mix, sample):
            if w["status"] == "ok":
                assert r.status == sge.OK, w["j"]
                assert (r.matches, r.states) == (w["matches"], w["states"]), w["j"]
            else:
                assert r.status == sge.E_ABORTED, w["j"]
            alone = ctx.count(t, p, allow=(sge.OK, sge.E_ABORTED))
            assert alone.status == r.status
            if r.status == sge.OK:
                assert (alone.matches, alone.states) == (r.matches, r.states)
    finally:
        ctx.set_state_cap(0)
        ctx.set_plan_location(-1)
        for _, p, _, _ in jobs:
            ctx.unload_pattern(p)
        for t in th:
            ctx.unload_target(t)


def test_serve_admission(ctx):
    """A slow query holds the only slot: the next submit is refused (BUSY)
    until the first completes; a query larger than the memory budget is
    refused outright."""
    T3 = synth.c3_target()
    slow = synth.c3_instance(0, 0)
    fast = synth.c1_instance(0)
    t3 = ctx.load_target(T3)
    p3 = ctx.load_pattern(slow.pattern)
    t1 = ctx.load_target(fast.target)
    p1 = ctx.load_pattern(fast.pattern)
    ctx.serve_start(1, 1 << 30)
    try:
        tk = ctx.serve_submit(t3, p3, sge.RIDS_SI_FC, True)
        assert tk is not None
        assert ctx.serve_submit(t1, p1, sge.RI, True) is None      # no slot free
        t_end = time.time() + 60
        r = None
        while r is None and time.time() < t_end:
            r = ctx.serve_poll(tk)
            time.sleep(0.001)
        assert r is not None and r.status == sge.OK and r.matches >= 1
        tk2 = None
        while tk2 is None and time.time() < t_end:
            tk2 = ctx.serve_submit(t1, p1, sge.RI, True)
        r2 = None
        while r2 is None and time.time() < t_end:
            r2 = ctx.serve_poll(tk2)
        want = oracle.run(fast.pattern, fast.target, sge.RI, True)
        assert (r2.matches, r2.states) == (want["matches"], want["states"])
    finally:
        ctx.serve_stop()
    ctx.serve_start(4, 1000)    # below one query's plan: refused outright
    try:
        with pytest.raises(sge.SgeError) as e:
            ctx.serve_submit(t1, p1, sge.RI, True)
        assert e.value.code == sge.E_NOMEM
    finally:
        ctx.serve_stop()
    for h in (p3, p1):
        ctx.unload_pattern(h)
    for h in (t3, t1):
        ctx.unload_target(h)


def test_unload_refused_while_queries_use_the_graphs(ctx):
    """A target or pattern that a query in flight uses cannot be unloaded
    (SGE_E_BUSY); once the query has completed the unload succeeds, and the
    query's result is the oracle's.  The query is a full dense search (about
    7e8 states, a fraction of a second on the device), so it is still running
    when the unloads are tried right after the submit."""
    man = json.load(open(os.path.join(GOLDEN, "c3full.json")))
    w = man["instances"][0]
    inst = synth.c3_instance(w["j"], 0)
    th, ph = ctx.load_target(inst.target), ctx.load_pattern(inst.pattern)
    other = ctx.load_pattern(synth.c3_instance(1, 0).pattern)
    ctx.set_state_cap(0)
    ctx.serve_start(8, 1 << 30)
    try:
        tk = ctx.serve_submit(th, ph, sge.RIDS_SI_FC, True)
        assert tk is not None
        for fn, h in ((ctx.unload_target, th), (ctx.unload_pattern, ph)):
            with pytest.raises(sge.SgeError) as e:
                fn(h)
            assert e.value.code == sge.E_BUSY
        ctx.unload_pattern(other)          # not used by any query: unloads at once
        t_end = time.time() + 60
        r = None
        while r is None and time.time() < t_end:
            r = ctx.serve_poll(tk)
            time.sleep(0.001)
        assert r is not None and r.status == sge.OK
        assert (r.matches, r.states, r.alg_bytes) == (w["matches"], w["states"], w["dense_bytes"])
    finally:
        ctx.serve_stop()
    ctx.unload_pattern(ph)
    ctx.unload_target(th)
