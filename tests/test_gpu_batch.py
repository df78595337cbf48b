"""GPU parity of the batched path (many jobs in one persistent launch in a HIP
graph) against the oracle's stored results for the full workloads."""
from __future__ import annotations

import json
import os
import sys

import pytest

import oracle
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def manifest(cfg):
    with open(os.path.join(GOLDEN, f"{cfg}.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)   # any launch ends within a minute
    yield c
    c.close()


def load_jobs(ctx, insts):
    tcache = {}
    jobs = []
    for inst in insts:
        key = id(inst.target)
        if key not in tcache:
            tcache[key] = ctx.load_target(inst.target)
        jobs.append((tcache[key], ctx.load_pattern(inst.pattern), inst.mode, inst.labelled))
    return jobs


def unload(ctx, jobs):
    for t in {j[0] for j in jobs}:
        ctx.unload_target(t)
    for j in jobs:
        ctx.unload_pattern(j[1])


@pytest.mark.parametrize("policy", [2, 1])
def test_small_batch_c1(ctx, policy):
    man = manifest("c1")
    rows = man["instances"][:6]
    _note(f"batch c1 x{len(rows)} policy {policy}")
    insts = [synth.c1_instance(r["j"], r["attempt"]) for r in rows]
    jobs = load_jobs(ctx, insts)
    ctx.set_batch_policy(policy)
    try:
        st, res = ctx.batch_run(jobs)
    finally:
        ctx.set_batch_policy(0)
        unload(ctx, jobs)
    assert st == sge.OK
    assert [(r.matches, r.states) for r in res] == [(w["matches"], w["states"]) for w in rows]


def test_batch_mixed_modes_vs_live_oracle(ctx):
    import graphs as G
    insts = [synth.c1_instance(j) for j in range(8)]
    for i, inst in enumerate(insts):
        inst.mode = i % 4
    # two small unlabelled jobs (an unlabelled 8-node pattern has ~1e9 embeddings here)
    for i, P in enumerate([G.path(3), G.cycle(4)]):
        insts.append(synth.Instance(insts[i].target, P, i * 3, False, None))
    jobs = load_jobs(ctx, insts)
    try:
        st, res = ctx.batch_run(jobs)
    finally:
        unload(ctx, jobs)
    for inst, r in zip(insts, res):
        w = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled)
        assert (r.matches, r.states) == (w["matches"], w["states"])


@pytest.mark.parametrize("cfg", ["c1", "c2"])
@pytest.mark.parametrize("policy", [0, 1, 2])
@pytest.mark.parametrize("where", [-1, 0])
def test_full_batch(ctx, cfg, policy, where):
    """where: -1 plans these 100-job batches on the device, 0 on the host."""
    man = manifest(cfg)
    _note(f"batch {cfg} full x{len(man['instances'])} policy {policy} plan {where}")
    make = {"c1": synth.c1_instance, "c2": synth.c2_instance}[cfg]
    insts = [make(r["j"], r["attempt"]) for r in man["instances"]]
    jobs = load_jobs(ctx, insts)
    ctx.set_batch_policy(policy)
    ctx.set_plan_location(where)
    try:
        st, res = ctx.batch_run(jobs)
    finally:
        ctx.set_batch_policy(0)
        ctx.set_plan_location(-1)
        unload(ctx, jobs)
    assert st == sge.OK
    got = [(r.matches, r.states) for r in res]
    want = [(w["matches"], w["states"]) for w in man["instances"]]
    assert got == want


@pytest.fixture(scope="module")
def c4_jobs(ctx):
    man = manifest("c4")
    _note("batch c4 x4096: generating")
    insts = [synth.c4_instance(r["j"], r["attempt"]) for r in man["instances"]]
    jobs = load_jobs(ctx, insts)
    yield man, jobs
    unload(ctx, jobs)


@pytest.mark.parametrize("where", [-1, 0])
def test_c4_full_batch(ctx, c4_jobs, where):
    """All 4096 pairs of the batching workload in one launch, planned on the
    device (-1: automatic for a batch this size) or on the host (0)."""
    man, jobs = c4_jobs
    _note(f"batch c4: running, plan {where}")
    ctx.set_plan_location(where)
    try:
        st, res = ctx.batch_run(jobs)
    finally:
        ctx.set_plan_location(-1)
    assert st == sge.OK
    bad = [(i, r.matches, r.states, w["matches"], w["states"])
           for i, (r, w) in enumerate(zip(res, man["instances"])) if (r.matches, r.states) != (w["matches"], w["states"])]
    assert not bad, bad[:10]


def test_batch_state_cap(ctx):
    man = manifest("c2")
    rows = man["instances"][:10]
    insts = [synth.c2_instance(r["j"], r["attempt"]) for r in rows]
    jobs = load_jobs(ctx, insts)
    cap = sorted(r["states"] for r in rows)[5]
    ctx.set_state_cap(cap)
    try:
        st, res = ctx.batch_run(jobs, allow=(sge.OK, sge.E_ABORTED))
    finally:
        ctx.set_state_cap(0)
        unload(ctx, jobs)
    assert st == sge.E_ABORTED
    for r, w in zip(res, rows):
        if w["states"] <= cap:
            assert (r.matches, r.states) == (w["matches"], w["states"])
        else:
            assert r.states > cap


def test_batch_graph_reuse(ctx):
    """The batch graph is launched again while the launch is unchanged: every
    repeat (with eager single searches between them) must match the oracle,
    a changed state cap must take effect at once and be lifted again, and a
    different job list of the same size must give its own results."""
    man = manifest("c2")
    rows = man["instances"][:10]
    other = man["instances"][10:20]
    insts = [synth.c2_instance(r["j"], r["attempt"]) for r in rows]
    insts2 = [synth.c2_instance(r["j"], r["attempt"]) for r in other]
    jobs = load_jobs(ctx, insts)
    jobs2 = load_jobs(ctx, insts2)
    want = [(w["matches"], w["states"]) for w in rows]
    want2 = [(w["matches"], w["states"]) for w in other]
    ctx.set_batch_policy(2)
    ctx.set_plan_location(1)
    ctx.set_mode(sge.RI)          # the single searches below: as the jobs (RI, labelled)
    ctx.set_labelled(True)
    try:
        for rep in range(3):
            _note(f"batch graph reuse: repeat {rep}")
            st, res = ctx.batch_run(jobs)
            assert st == sge.OK and [(r.matches, r.states) for r in res] == want
            single = ctx.count(jobs[rep][0], jobs[rep][1])   # eager work between the launches
            assert (single.matches, single.states) == want[rep]
        cap = sorted(w["states"] for w in rows)[5]
        ctx.set_state_cap(cap)
        st, res = ctx.batch_run(jobs, allow=(sge.OK, sge.E_ABORTED))
        assert st == sge.E_ABORTED
        for r, w in zip(res, rows):
            if w["states"] <= cap:
                assert (r.matches, r.states) == (w["matches"], w["states"])
            else:
                assert r.states > cap
        ctx.set_state_cap(0)
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK and [(r.matches, r.states) for r in res] == want
        st, res = ctx.batch_run(jobs2)
        assert st == sge.OK and [(r.matches, r.states) for r in res] == want2
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK and [(r.matches, r.states) for r in res] == want
    finally:
        ctx.set_state_cap(0)
        ctx.set_batch_policy(0)
        ctx.set_plan_location(-1)
        unload(ctx, jobs)
        unload(ctx, jobs2)


_UNITS = {}


@pytest.mark.parametrize("per_cu", [1, 2, 3])
def test_blocks_per_cu_cap(ctx, per_cu):
    # the same counts with fewer resident blocks; more blocks, no fewer units
    man = manifest("c2")
    _note(f"batch c2 with at most {per_cu} blocks per CU")
    insts = [synth.c2_instance(r["j"], r["attempt"]) for r in man["instances"]]
    jobs = load_jobs(ctx, insts)
    ctx.set_blocks_per_cu(per_cu)
    ctx.set_batch_policy(2)
    try:
        st, res = ctx.batch_run(jobs)
        busy, units = ctx.last_launch_occupancy()
    finally:
        ctx.set_blocks_per_cu(0)
        ctx.set_batch_policy(0)
        unload(ctx, jobs)
    assert st == sge.OK
    assert [(r.matches, r.states) for r in res] == [(w["matches"], w["states"]) for w in man["instances"]]
    assert units >= 1 and busy > 0
    assert units <= per_cu * 1024 * 32          # under 1024 CUs, at most 32 units per block
    _UNITS[per_cu] = units
    assert all(_UNITS[p] <= units for p in _UNITS if p < per_cu)


def test_blocks_per_cu_rejects_out_of_range(ctx):
    for bad in (-1, 65):
        with pytest.raises(sge.SgeError) as e:
            ctx.set_blocks_per_cu(bad)
        assert e.value.code == sge.E_INVAL
