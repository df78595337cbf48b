"""GPU parity on targets above 65,536 nodes: no adjacency rows (back-edges are
binary searches in the CSR rows), and, where a used-node bitset per search
unit no longer fits in LDS beside four waves, candidates compared with the
mapped prefix instead.  Protein-contact-like targets of 70,000 and 600,000
nodes (the contact generator, 20 Zipf labels), random-walk patterns, full
searches against the oracle: matches, states, algorithmic bytes and the
digest of the sorted rows."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu

SIZES = {70_000: 0, 600_000: 1}


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.set_tuning(0, 0, 1, -1)
    c.close()


def workload(n):
    i = SIZES[n]
    T = synth.contact_target(synth.rng(99, 0, i, 0), n)
    g = synth.rng(99, 1, i, 0)
    pats = []
    for k in (8, 12, 16, 24):
        P, planted = synth.induced_pattern(g, T, synth.walk_selection(g, T, k))
        pats.append((P, planted))
    return T, pats


@pytest.mark.parametrize("n", sorted(SIZES))
@pytest.mark.parametrize("lanes", [32, 64])
def test_large_target_single(ctx, n, lanes):
    T, pats = workload(n)
    th = ctx.load_target(T)
    try:
        ctx.set_tuning(lanes, 0, 1, -1)
        for P, planted in pats:
            ph = ctx.load_pattern(P)
            try:
                for mode in (sge.RI, sge.RIDS_SI_FC):
                    _note(f"large n={n} k={P.n} mode={mode} lanes={lanes}")
                    want = oracle.run(P, T, mode, True, rows=True)
                    ctx.set_mode(mode)
                    ctx.set_labelled(True)
                    res, rows = ctx.enumerate(th, ph, P.n, cap_rows=want["matches"] + 1)
                    assert (res.matches, res.states) == (want["matches"], want["states"])
                    assert res.alg_bytes == want["alg_bytes"]
                    assert oracle.rows_digest(rows, P.n) == oracle.rows_digest(want["rows"], P.n)
                    assert any(np.array_equal(r, planted) for r in rows)
            finally:
                ctx.unload_pattern(ph)
    finally:
        ctx.set_tuning(0, 0, 1, -1)
        ctx.unload_target(th)


@pytest.mark.parametrize("where", [0, 1])
def test_large_target_batch(ctx, where):
    """All patterns of both targets in one launch, planned on the host (0) or
    by the plan kernel (1; support sets of the 600,000-node target do not fit
    its LDS and go to device memory)."""
    jobs, want = [], []
    loaded = []
    for n in sorted(SIZES):
        T, pats = workload(n)
        th = ctx.load_target(T)
        loaded.append(th)
        for P, _ in pats:
            ph = ctx.load_pattern(P)
            for mode in (sge.RI, sge.RIDS_SI_FC):
                jobs.append((th, ph, mode, True))
                want.append(oracle.run(P, T, mode, True))
    try:
        ctx.set_plan_location(where)
        _note(f"large batch x{len(jobs)} plan {where}")
        st, res = ctx.batch_run(jobs)
        assert st == sge.OK
        assert res.matches.tolist() == [w["matches"] for w in want]
        assert res.states.tolist() == [w["states"] for w in want]
        assert res.alg_bytes.tolist() == [w["alg_bytes"] for w in want]
    finally:
        ctx.set_plan_location(-1)
        for j in jobs[::2]:
            ctx.unload_pattern(j[1])
        for th in loaded:
            ctx.unload_target(th)
