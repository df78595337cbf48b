"""The paper's parallel CPU search (the measurement baseline) against the
oracle: match and canonical state counts for any number of workers and any
task-group size (work stealing must neither lose nor repeat work)."""
from __future__ import annotations

import numpy as np
import pytest

import graphs as G
from paper_1705_09358_amd import cpu_baseline, synth


@pytest.mark.parametrize("seed", range(25))
def test_tiny_random_any_worker_count(orc, seed):
    g = np.random.default_rng(31000 + seed)
    n = int(g.integers(2, 14))
    k = int(g.integers(1, min(6, n) + 1))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), int(g.integers(1, 3)))
    P = G.random_graph(g, k, float(g.uniform(0.3, 1.0)), int(g.integers(1, 3)))
    for mode in (0, 3):
        for labelled in (False, True):
            w = orc.run(P, T, mode, labelled)
            for threads, group in [(1, 1), (2, 4), (5, 2), (8, 4)]:
                r = cpu_baseline.count(P, T, mode, labelled, threads, group)
                assert (r["matches"], r["states"]) == (w["matches"], w["states"]), (mode, labelled, threads)


@pytest.mark.parametrize("j", [0, 5, 28, 41, 77])
def test_contact_patterns(orc, j):
    inst = synth.c2_instance(j)
    w = orc.run(inst.pattern, inst.target, inst.mode, inst.labelled)
    for threads in (1, 4, 16):
        r = cpu_baseline.count(inst.pattern, inst.target, inst.mode, inst.labelled, threads)
        assert (r["matches"], r["states"]) == (w["matches"], w["states"])


def test_many_workers_steal_and_agree(orc):
    # a search large enough that idle workers must steal; repeated to shake out races
    T = G.complete(11)
    P = G.cycle(5)
    w = orc.run(P, T, 0, False)
    for rep in range(5):
        r = cpu_baseline.count(P, T, 0, False, 12, 4)
        assert (r["matches"], r["states"]) == (w["matches"], w["states"])
    assert r["matches"] == 11 * 10 * 9 * 8 * 7


def test_edge_cases(orc):
    T = G.petersen()
    assert cpu_baseline.count(G.edgeless(0), T, 0, False, 4)["matches"] == 1      # k = 0
    assert cpu_baseline.count(G.complete(11), T, 0, False, 4)["matches"] == 0     # k > n
    r = cpu_baseline.count(G.edgeless(1), T, 0, False, 3)
    assert (r["matches"], r["states"]) == (10, 10)
