"""Pins of the oracle on directed and edge-labelled graphs (the paper's general
problem, Section 2.1, eqs. (2)-(4); RI's rules 3-4 with in- and out-degree and
edge-label compatibility; RI-DS domains on in- and out-degree, Section 4.1).

Every pin checks the oracle against something other than itself: brute force
over all injections, the undirected oracle on symmetric inputs, closed forms,
and invariants (arc reversal, label coarsening, domain soundness)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import graphs as G


def _rows(r):
    r = np.asarray(r, dtype=np.uint32)
    return r[np.lexsort(r.T[::-1])] if r.shape[0] > 1 else r


@pytest.mark.parametrize("seed", range(50))
def test_brute_force_directed_edge_labelled(orc, seed):
    g = np.random.default_rng(5000 + seed)
    n = int(g.integers(2, 8))
    k = int(g.integers(1, min(5, n) + 1))
    nlab = int(g.integers(1, 3))
    nelab = int(g.integers(1, 4))
    T = G.random_digraph(g, n, float(g.uniform(0.2, 0.7)), nlab, nelab)
    P = G.random_digraph(g, k, float(g.uniform(0.3, 0.9)), nlab, nelab)
    for labelled in (False, True):
        want = G.brute_matches_ex(P, T, labelled)
        for mode in range(4):
            got = orc.run(P, T, mode, labelled, rows=True)
            assert got["matches"] == want.shape[0], (mode, labelled)
            assert np.array_equal(_rows(got["rows"]), want), (mode, labelled)
            pl = orc.plan(P, T, mode, labelled)
            if pl["empty"]:
                assert got["states"] == 0
                continue
            assert got["states"] == G.brute_states_ex(P, T, labelled, pl["order"], pl["domains"]), (mode, labelled)


@pytest.mark.parametrize("seed", range(20))
def test_brute_force_undirected_edge_labelled(orc, seed):
    g = np.random.default_rng(6000 + seed)
    n = int(g.integers(2, 8))
    k = int(g.integers(1, min(5, n) + 1))
    T = G.random_undirected_elabelled(g, n, float(g.uniform(0.3, 0.8)), 2, 3)
    P = G.random_undirected_elabelled(g, k, float(g.uniform(0.4, 1.0)), 2, 3)
    for labelled in (False, True):
        want = G.brute_matches_ex(P, T, labelled)
        for mode in (0, 3):
            got = orc.run(P, T, mode, labelled, rows=True)
            assert np.array_equal(_rows(got["rows"]), want), (mode, labelled)
            pl = orc.plan(P, T, mode, labelled)
            if not pl["empty"]:
                assert got["states"] == G.brute_states_ex(P, T, labelled, pl["order"], pl["domains"])


@pytest.mark.parametrize("seed", range(15))
def test_mixed_directed_pattern_undirected_target(orc, seed):
    g = np.random.default_rng(7000 + seed)
    T = G.random_graph(g, int(g.integers(3, 8)), 0.5, 2)        # undirected: both arcs of every edge
    P = G.random_digraph(g, int(g.integers(1, 4)), 0.6, 2, 1)
    for labelled in (False, True):
        want = G.brute_matches_ex(P, T, labelled)
        got = orc.run(P, T, 3, labelled, rows=True)
        assert np.array_equal(_rows(got["rows"]), want)


@pytest.mark.parametrize("seed", range(15))
def test_symmetric_inputs_as_directed_equal_undirected(orc, seed):
    # an undirected graph is the directed graph with both arcs of every edge
    g = np.random.default_rng(8000 + seed)
    T = G.random_graph(g, int(g.integers(4, 12)), 0.4, 2)
    P = G.random_graph(g, int(g.integers(2, 6)), 0.6, 2)
    Td = G.Graph(T.n, T.row_ptr, T.col, T.labels, None, True)
    Pd = G.Graph(P.n, P.row_ptr, P.col, P.labels, None, True)
    for mode in range(4):
        for labelled in (False, True):
            a = orc.run(P, T, mode, labelled)
            b = orc.run(Pd, Td, mode, labelled)
            assert (a["matches"], a["states"], a["candidates"]) == (b["matches"], b["states"], b["candidates"])


@pytest.mark.parametrize("seed", range(10))
def test_uniform_edge_labels_change_nothing(orc, seed):
    g = np.random.default_rng(9000 + seed)
    T = G.random_digraph(g, 7, 0.4, 2, 1)
    P = G.random_digraph(g, 3, 0.7, 2, 1)
    T7 = G.Graph(T.n, T.row_ptr, T.col, T.labels, np.full(T.col.size, 7, np.uint32), True)
    P7 = G.Graph(P.n, P.row_ptr, P.col, P.labels, np.full(P.col.size, 7, np.uint32), True)
    for mode in range(4):
        a = orc.run(P, T, mode, True)
        b = orc.run(P7, T7, mode, True)
        assert (a["matches"], a["states"]) == (b["matches"], b["states"])


def _dicycle(n):
    return G.from_arcs(n, [(i, (i + 1) % n) for i in range(n)])


def _tournament(n):
    return G.from_arcs(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def _dipath(n):
    return G.from_arcs(n, [(i, i + 1) for i in range(n - 1)])


@pytest.mark.parametrize("n", [3, 5, 8])
def test_directed_cycle_automorphisms(orc, n):
    # the rotations only (a reflection reverses the arcs)
    for mode in range(4):
        assert orc.run(_dicycle(n), _dicycle(n), mode, False)["matches"] == n


@pytest.mark.parametrize("n,k", [(5, 3), (7, 4), (8, 2), (6, 6)])
def test_transitive_tournament_closed_forms(orc, n, k):
    # an order-preserving injection for each k-subset: C(n, k) copies of TT_k,
    # and the directed path P_k also maps onto every increasing k-sequence
    for mode in (0, 3):
        assert orc.run(_tournament(k), _tournament(n), mode, False)["matches"] == math.comb(n, k)
        assert orc.run(_dipath(k), _tournament(n), mode, False)["matches"] == math.comb(n, k)


def test_directed_cycle_not_in_tournament(orc):
    # a transitive tournament is acyclic
    for mode in range(4):
        assert orc.run(_dicycle(3), _tournament(6), mode, False)["matches"] == 0


def test_single_arc_counts_by_label(orc):
    g = np.random.default_rng(31)
    T = G.random_digraph(g, 9, 0.35, 1, 3)
    arcs = G.arcs_of(T)
    for b in range(3):
        P = G.from_arcs(2, [(0, 1)], None, [b])
        want = sum(1 for lb in arcs.values() if lb == b)
        for mode in range(4):
            assert orc.run(P, T, mode, True)["matches"] == want
            assert orc.run(P, T, mode, False)["matches"] == len(arcs)


@pytest.mark.parametrize("seed", range(12))
def test_reversal_invariance(orc, seed):
    g = np.random.default_rng(3300 + seed)
    T = G.random_digraph(g, 8, 0.3, 2, 2)
    P = G.random_digraph(g, 4, 0.5, 2, 2)
    for mode in (0, 3):
        a = orc.run(P, T, mode, True, rows=True)
        b = orc.run(G.reverse(P), G.reverse(T), mode, True, rows=True)
        assert np.array_equal(_rows(a["rows"]), _rows(b["rows"]))


@pytest.mark.parametrize("seed", range(12))
def test_labelled_subset_of_unlabelled_and_domain_soundness(orc, seed):
    g = np.random.default_rng(4400 + seed)
    T = G.random_digraph(g, 9, 0.35, 2, 2)
    P = G.random_digraph(g, 4, 0.45, 2, 2)
    lab = {tuple(r) for r in orc.run(P, T, 0, True, rows=True)["rows"].tolist()}
    unl = {tuple(r) for r in orc.run(P, T, 0, False, rows=True)["rows"].tolist()}
    assert lab <= unl
    for mode in (1, 3):
        pl = orc.plan(P, T, mode, True)
        if pl["empty"]:
            assert not lab
            continue
        for r in lab:
            for u, v in enumerate(r):
                assert pl["domains"][u, v]


def test_arc_consistency_follows_arc_direction(orc):
    # pattern a -> b; target x -> y and a lone z: only x can host a, only y b
    P = G.from_arcs(2, [(0, 1)])
    T = G.from_arcs(3, [(0, 1)])
    pl = orc.plan(P, T, 1, False)
    assert pl["domains"].tolist() == [[True, False, False], [False, True, False]]
    # an incoming pattern arc needs an incoming target arc from the neighbour's domain
    T2 = G.from_arcs(4, [(0, 1), (2, 3), (3, 2)], [0, 1, 0, 1])
    P2 = G.from_arcs(2, [(1, 0)], [1, 0])          # node 1 (label 0) -> node 0 (label 1)
    pl = orc.plan(P2, T2, 1, True)
    # node 0 of the pattern needs an in-arc from a label-0 node: targets 1 (from 0) and 3 (from 2)
    assert pl["domains"][0].tolist() == [False, True, False, True]
    assert pl["domains"][1].tolist() == [True, False, True, False]


def test_edge_labels_prune_domains(orc):
    # same shape, one arc label differs: the mismatching target arc cannot host it
    P = G.from_arcs(2, [(0, 1)], None, [5])
    T = G.from_arcs(4, [(0, 1), (2, 3)], None, [5, 6])
    pl = orc.plan(P, T, 1, True)
    assert pl["domains"].tolist() == [[True, False, False, False], [False, True, False, False]]
    assert orc.run(P, T, 0, True)["matches"] == 1
    assert orc.run(P, T, 0, False)["matches"] == 2


@pytest.mark.parametrize("seed", range(40))
def test_arc_consistency_is_the_greatest_fixpoint(orc, seed):
    g = np.random.default_rng(12000 + seed)
    T = G.random_digraph(g, int(g.integers(3, 9)), float(g.uniform(0.15, 0.5)), 2, 3)
    P = G.random_digraph(g, int(g.integers(2, 5)), float(g.uniform(0.3, 0.8)), 2, 3)
    for labelled in (False, True):
        want = G.brute_ac_domains(P, T, labelled)
        pl = orc.plan(P, T, 1, labelled)
        if pl["empty"]:
            assert not want.any(axis=1).all()
        else:
            assert np.array_equal(pl["domains"], want)
