"""GPU parity of the dense-bitset search (frames as candidate bitsets)."""
from __future__ import annotations

import json
import math
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
    c.set_tuning(0, 0, 1, 1)     # force the dense kernel
    yield c
    c.close()


def run(ctx, P, T, mode, labelled, rows=True, cap_rows=None):
    th = ctx.load_target(T)
    ph = ctx.load_pattern(P)
    try:
        ctx.set_mode(mode)
        ctx.set_labelled(labelled)
        if rows:
            return ctx.enumerate(th, ph, P.n, cap_rows=cap_rows or (1 << 16))
        return ctx.count(th, ph), None
    finally:
        ctx.unload_pattern(ph)
        ctx.unload_target(th)


@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_dense(ctx, seed):
    g = np.random.default_rng(500 + seed)
    n = int(g.integers(2, 14))
    k = int(g.integers(1, min(6, n) + 1))
    nlab = int(g.integers(1, 4))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.3, 1.0)), nlab)
    for mode in range(4):
        for labelled in (False, True):
            want = oracle.run(P, T, mode, labelled, rows=True)
            res, rows = run(ctx, P, T, mode, labelled, cap_rows=want["matches"] + 1)
            assert (res.matches, res.states) == (want["matches"], want["states"]), (seed, mode, labelled)
            assert np.array_equal(_sorted(rows), _sorted(want["rows"]))


@pytest.mark.parametrize("n,k", [(8, 3), (70, 3), (130, 2), (9, 5)])
def test_clique_closed_form_dense(ctx, n, k):
    res, _ = run(ctx, G.complete(k), G.complete(n), 0, False, rows=False)
    assert res.matches == math.perm(n, k)
    assert res.states == sum(math.perm(n, d) for d in range(1, k + 1))


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_manifest_dense(ctx, cfg):
    with open(os.path.join(GOLDEN, f"{cfg}.json")) as f:
        man = json.load(f)
    make = {"c1": synth.c1_instance, "c2": synth.c2_instance}[cfg]
    for r in man["instances"][::3]:
        inst = make(r["j"], r["attempt"])
        _note(f"dense {cfg}/{r['j']}")
        res, rows = run(ctx, inst.pattern, inst.target, inst.mode, True, cap_rows=r["matches"] + 1)
        assert (res.matches, res.states) == (r["matches"], r["states"])
        assert oracle.rows_digest(rows, inst.pattern.n) == r["sha256"]


def test_dense_rids_modes_c1(ctx):
    for j in range(0, 100, 10):
        inst = synth.c1_instance(j)
        for mode in (1, 2, 3):
            want = oracle.run(inst.pattern, inst.target, mode, True)
            res, _ = run(ctx, inst.pattern, inst.target, mode, True, rows=False)
            assert (res.matches, res.states) == (want["matches"], want["states"])


def _c3():
    with open(os.path.join(GOLDEN, "c3.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ctx_auto():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.close()


def test_c3_shards(ctx_auto):
    """The dense workload against the oracle on root shards (first node of the
    order restricted to a range of target ids)."""
    man = _c3()
    T = synth.c3_target()
    th = ctx_auto.load_target(T)
    ctx_auto.set_mode(3)
    ctx_auto.set_labelled(True)
    try:
        for r in man["instances"]:
            inst = synth.c3_instance(r["j"], 0)
            _note(f"c3 shard {r['j']} [{r['root_lo']},{r['root_hi']})")
            ph = ctx_auto.load_pattern(inst.pattern)
            ctx_auto.set_root_range(r["root_lo"], r["root_hi"])
            try:
                res, rows = ctx_auto.enumerate(th, ph, inst.pattern.n, cap_rows=r["matches"] + 1)
            finally:
                ctx_auto.set_root_range()
                ctx_auto.unload_pattern(ph)
            assert (res.matches, res.states) == (r["matches"], r["states"]), r["j"]
            assert oracle.rows_digest(rows, inst.pattern.n) == r["sha256"]
    finally:
        ctx_auto.unload_target(th)


@pytest.mark.parametrize("j", [0, 7])
def test_c3_full_size_properties(ctx_auto, j):
    """Full-size dense searches (~1e9 states, beyond the oracle): the planted
    embedding is found, every row satisfies the definition, and a partition of
    the root candidates adds up to the whole search."""
    T = synth.c3_target()
    inst = synth.c3_instance(j, 0)
    th = ctx_auto.load_target(T)
    ph = ctx_auto.load_pattern(inst.pattern)
    ctx_auto.set_mode(3)
    ctx_auto.set_labelled(True)
    try:
        _note(f"c3/{j} full")
        full, rows = ctx_auto.enumerate(th, ph, inst.pattern.n, cap_rows=4096)
        assert full.matches >= 1 and full.states > 10 ** 7
        assert any(np.array_equal(r, inst.planted) for r in rows)
        A = G.adjacency(T)
        for r in rows:
            assert len(set(r.tolist())) == inst.pattern.n
            assert all(T.labels[r[u]] == inst.pattern.labels[u] for u in range(inst.pattern.n))
            assert all(A[r[u], r[int(w)]] for u in range(inst.pattern.n) for w in inst.pattern.neighbours(u))
        tot = [0, 0]
        for lo, hi in [(0, 250), (250, 600), (600, 1000)]:
            ctx_auto.set_root_range(lo, hi)
            try:
                part = ctx_auto.count(th, ph)
            finally:
                ctx_auto.set_root_range()
            tot[0] += part.matches
            tot[1] += part.states
        assert tot == [full.matches, full.states]
    finally:
        ctx_auto.unload_pattern(ph)
        ctx_auto.unload_target(th)


@pytest.mark.parametrize("i", range(4))
def test_c3_full_size_against_oracle(ctx_auto, i):
    """The four dense patterns the benchmark times, searched whole (2.7e9
    states together): matches, states, the digest of the sorted rows and the
    dense algorithmic bytes equal the oracle's full-size values (stored, each
    the sum of the oracle's root shards)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3full.json")) as f:
        w = json.load(f)["instances"][i]
    T = synth.c3_target()
    inst = synth.c3_instance(w["j"], w["attempt"])
    th = ctx_auto.load_target(T)
    ph = ctx_auto.load_pattern(inst.pattern)
    ctx_auto.set_mode(w["mode"])
    ctx_auto.set_labelled(w["labelled"])
    try:
        _note(f"c3 full/{w['j']} against the oracle")
        res, rows = ctx_auto.enumerate(th, ph, inst.pattern.n, cap_rows=max(1, w["matches"]))
        assert (res.matches, res.states) == (w["matches"], w["states"])
        assert oracle.rows_digest(rows, inst.pattern.n) == w["sha256"]
        cnt = ctx_auto.count(th, ph)
        assert (cnt.matches, cnt.states) == (w["matches"], w["states"])
        assert cnt.alg_bytes == w["dense_bytes"]
    finally:
        ctx_auto.unload_pattern(ph)
        ctx_auto.unload_target(th)
