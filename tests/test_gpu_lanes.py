"""The search units' state is kept per lane (every lane of a unit holds a copy
of its task, level, stack top and current frame).  With the library's
per-step check on, each copy is compared with the unit's first lane on every
step of every unit; the workloads below must finish with no disagreement and
with the oracle's counts, for every unit width and both kernel variants."""
from __future__ import annotations

import json
import os
import sys

import pytest

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
    c.set_time_limit(60000)
    c.set_checks(True)
    yield c
    c.set_checks(False)
    c.set_tuning(0, 0, 1, -1)
    c.close()


def jobs_of(ctx, insts):
    tc, jobs = {}, []
    for i in insts:
        if id(i.target) not in tc:
            tc[id(i.target)] = ctx.load_target(i.target)
        jobs.append((tc[id(i.target)], ctx.load_pattern(i.pattern), i.mode, i.labelled))
    return tc, jobs


def drop(ctx, tc, jobs):
    for j in jobs:
        ctx.unload_pattern(j[1])
    for t in tc.values():
        ctx.unload_target(t)


@pytest.mark.parametrize("lanes", [8, 16, 32, 64])
def test_batch_contact3000_every_width(ctx, lanes):
    man = manifest("c2")
    tc, jobs = jobs_of(ctx, [synth.c2_instance(r["j"], r["attempt"]) for r in man["instances"]])
    try:
        ctx.set_tuning(lanes, 0, 1, 0)
        ctx.set_batch_policy(2)
        _note(f"checked batch c2 lanes {lanes}")
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK
        assert res.states.tolist() == [r["states"] for r in man["instances"]]
        assert res.matches.tolist() == [r["matches"] for r in man["instances"]]
    finally:
        ctx.set_tuning(0, 0, 1, -1)
        ctx.set_batch_policy(0)
        drop(ctx, tc, jobs)


def test_single_contact3000_automatic_width(ctx):
    """Each contact-3000 pattern alone, all units on it (64-lane units)."""
    man = manifest("c2")
    T = synth.c2_target()
    th = ctx.load_target(T)
    try:
        for r in man["instances"]:
            inst = synth.c2_instance(r["j"], r["attempt"])
            ph = ctx.load_pattern(inst.pattern)
            try:
                ctx.set_mode(inst.mode)
                ctx.set_labelled(True)
                res = ctx.count(th, ph)
                assert (res.matches, res.states) == (r["matches"], r["states"]), r["j"]
            finally:
                ctx.unload_pattern(ph)
    finally:
        ctx.unload_target(th)


@pytest.mark.parametrize("lanes", [8, 64])
def test_dense_c1(ctx, lanes):
    man = manifest("c1")
    tc, jobs = jobs_of(ctx, [synth.c1_instance(r["j"], r["attempt"]) for r in man["instances"]])
    try:
        ctx.set_tuning(lanes, 0, 1, 1)
        _note(f"checked dense batch c1 lanes {lanes}")
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK
        assert res.states.tolist() == [r["states"] for r in man["instances"]]
    finally:
        ctx.set_tuning(0, 0, 1, -1)
        drop(ctx, tc, jobs)


def test_batching_workload(ctx):
    man = manifest("c4")
    tc, jobs = jobs_of(ctx, [synth.c4_instance(r["j"], r["attempt"]) for r in man["instances"]])
    try:
        _note("checked batch c4")
        ctx.set_batch_policy(2)
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK
        assert res.states.tolist() == [r["states"] for r in man["instances"]]
    finally:
        ctx.set_batch_policy(0)
        drop(ctx, tc, jobs)
