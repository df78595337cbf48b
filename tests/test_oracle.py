"""Pins for the oracle: brute force, closed forms, the paper's worked example,
the ordering rules, and invariants.  Nothing here uses the GPU library."""
from __future__ import annotations

import math

import numpy as np
import pytest

import graphs as G
from paper_1705_09358_amd import synth

MODES = [0, 1, 2, 3]


def _sorted(rows):
    rows = np.asarray(rows, dtype=np.uint32)
    return rows[np.lexsort(rows.T[::-1])] if rows.shape[0] > 1 else rows


# ------------------------------------------------------------------ brute force
@pytest.mark.parametrize("seed", range(120))
def test_brute_force_tiny(orc, seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(2, 9))
    k = int(g.integers(1, min(5, n) + 1))
    nlab = int(g.integers(1, 4))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.3, 1.0)), nlab)
    labelled = bool(g.integers(0, 2))
    want = G.brute_matches(P, T, labelled)
    for mode in MODES:
        r = orc.run(P, T, mode, labelled, rows=True)
        assert r["status"] == 0
        assert r["matches"] == want.shape[0]
        assert np.array_equal(_sorted(r["rows"]), want)
        pl = orc.plan(P, T, mode, labelled)
        if pl["empty"]:
            assert r["states"] == 0 and want.shape[0] == 0
            continue
        assert sorted(pl["order"].tolist()) == list(range(k))
        assert r["states"] == G.brute_states(P, T, labelled, pl["order"], pl["domains"])


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,k", [(6, 1), (6, 3), (7, 4), (6, 6), (5, 6)])
def test_clique_in_clique(orc, n, k):
    r = orc.run(G.complete(k), G.complete(n), 0, False)
    want = math.perm(n, k) if k <= n else 0
    assert r["matches"] == want
    if k <= n:
        assert r["states"] == sum(math.perm(n, d) for d in range(1, k + 1))


@pytest.mark.parametrize("pat", ["path4", "star3", "cycle5", "edgeless3", "k23"])
@pytest.mark.parametrize("mode", MODES)
def test_any_pattern_in_clique(orc, pat, mode):
    P = dict(path4=G.path(4), star3=G.star(3), cycle5=G.cycle(5), edgeless3=G.edgeless(3),
             k23=G.complete_bipartite(2, 3))[pat]
    n = 7
    r = orc.run(P, G.complete(n), mode, False)
    assert r["matches"] == math.perm(n, P.n)
    assert r["states"] == sum(math.perm(n, d) for d in range(1, P.n + 1))


AUT = [
    ("K5", G.complete(5), 120), ("C7", G.cycle(7), 14), ("P6", G.path(6), 2), ("K1,4", G.star(4), 24),
    ("K2,3", G.complete_bipartite(2, 3), 12), ("K3,3", G.complete_bipartite(3, 3), 72),
    ("Petersen", G.petersen(), 120), ("Q3", G.hypercube(3), 48), ("E4", G.edgeless(4), 24),
]


@pytest.mark.parametrize("name,g,aut", AUT, ids=[a[0] for a in AUT])
@pytest.mark.parametrize("mode", MODES)
def test_automorphisms(orc, name, g, aut, mode):
    assert orc.run(g, g, mode, False)["matches"] == aut
    uniq = G.relabel(g, np.arange(g.n))
    r = orc.run(uniq, uniq, mode, True, rows=True)
    assert r["matches"] == 1
    assert np.array_equal(r["rows"][0], np.arange(g.n))


def _target_stats(T):
    import scipy.sparse as sp
    A = sp.csr_matrix((np.ones(T.m2, dtype=np.int64), T.col.astype(np.int64), T.row_ptr.astype(np.int64)),
                      shape=(T.n, T.n))
    d = np.asarray(A.sum(1)).ravel()
    A2 = A @ A
    tr3 = int(A2.multiply(A).sum())          # trace(A^3) = sum_ij (A^2)_ij A_ji, A symmetric
    tr4 = int(A2.multiply(A2).sum())         # trace(A^4) = ||A^2||_F^2
    return A, d, tr3, tr4


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_closed_forms_on_config_targets(orc, which):
    T = synth.c1_instance(0).target if which == "c1" else synth.c2_target()
    A, d, tr3, tr4 = _target_stats(T)
    m = int(d.sum()) // 2
    cases = [
        (G.complete(2), 2 * m),
        (G.path(3), int((d * (d - 1)).sum())),
        (G.star(3), int((d * (d - 1) * (d - 2)).sum())),
        (G.complete(3), tr3),
        (G.cycle(4), tr4 - 2 * int((d * d).sum()) + 2 * m),
    ]
    for P, want in cases:
        for mode in (0, 3):
            assert orc.run(P, T, mode, False)["matches"] == want
    if which == "c1":
        assert orc.run(G.edgeless(2), T, 0, False)["matches"] == T.n * (T.n - 1)
    # labelled K2 with labels (a, b): ordered adjacent pairs with those labels
    for a, b in [(0, 1), (1, 1), (2, 0)]:
        P = G.from_edges(2, [(0, 1)], [a, b])
        la, lb = T.labels == a, T.labels == b
        want = int(A[la][:, lb].sum())
        for mode in MODES:
            assert orc.run(P, T, mode, True)["matches"] == want


# ------------------------------------------------ forward checking (Section 4.2.2)
def test_forward_check_paper_example(orc):
    """The worked example of forward checking: initial domains n0 {0}, n1 {4},
    n2 {0,3,7}, n3 {2,8,9}, n4 {0,4,7}; two rounds leave n2 {3} and n4 {7}."""
    init = [{0}, {4}, {0, 3, 7}, {2, 8, 9}, {0, 4, 7}]
    want = [{0}, {4}, {3}, {2, 8, 9}, {7}]
    dom = np.zeros((5, 10), dtype=bool)
    for u, s in enumerate(init):
        dom[u, list(s)] = True
    emptied, out = orc.forward_check(dom)
    assert not emptied
    assert [set(np.flatnonzero(out[u]).tolist()) for u in range(5)] == want


def test_forward_check_collision_empties(orc):
    dom = np.zeros((3, 4), dtype=bool)
    dom[0, 1] = dom[1, 1] = True
    dom[2, [1, 2]] = True
    emptied, _ = orc.forward_check(dom)
    assert emptied


# ------------------------------------------------ arc-consistency (Section 4.1)
def test_arc_consistency_cascades(orc):
    """Path a-b-c labelled A,B,C.  The B-node 4 has no C neighbour, so it leaves
    D(b); then the A-nodes 3 and 5, whose only B neighbour was 4, lose support."""
    A_, B_, C_ = 0, 1, 2
    T = G.from_edges(6, [(0, 1), (1, 2), (3, 4), (4, 5)], [A_, B_, C_, A_, B_, A_])
    P = G.from_edges(3, [(0, 1), (1, 2)], [A_, B_, C_])
    pl = orc.plan(P, T, 1, True)
    dom = pl["domains"]
    assert np.flatnonzero(dom[0]).tolist() == [0]
    assert np.flatnonzero(dom[1]).tolist() == [1]
    assert np.flatnonzero(dom[2]).tolist() == [2]


def test_arc_consistency_empty_domain(orc):
    T = G.from_edges(4, [(0, 1), (2, 3)], [0, 1, 1, 1])
    P = G.from_edges(3, [(0, 1), (1, 2)], [1, 0, 0])   # needs two 0-labelled nodes around a 1
    for mode in (1, 2, 3):
        pl = orc.plan(P, T, mode, True)
        assert pl["empty"]
        r = orc.run(P, T, mode, True)
        assert r["matches"] == 0 and r["states"] == 0


# --------------------------------------------------- ordering (Section "RI")
def test_order_highest_degree_first_and_more_wm_wins(orc):
    # triangle 0-1-2 plus pendant 3 on 0
    P = G.from_edges(4, [(0, 1), (1, 2), (0, 2), (0, 3)])
    pl = orc.plan(P, G.complete(6), 0, False)
    assert pl["order"].tolist() == [0, 1, 2, 3]
    assert pl["parent"].tolist() == [-1, 0, 0, 0]


def test_order_wn_breaks_wm_tie(orc):
    # after [0], nodes 1, 2, 4 have one neighbour in the order; 2 and 4 share the
    # unplaced neighbour 4 / 2 with node 0, node 1 shares none: w_n picks 2 over 1
    P = G.from_edges(5, [(0, 1), (0, 2), (0, 4), (2, 4), (1, 3)])
    pl = orc.plan(P, G.complete(6), 0, False)
    assert pl["order"].tolist() == [0, 2, 4, 1, 3]
    assert pl["parent"].tolist() == [-1, 0, 0, 0, 3]


def test_order_degree_breaks_wm_wn_tie(orc):
    P = G.from_edges(8, [(0, 1), (0, 2), (0, 3), (0, 6), (1, 7), (2, 4), (2, 5)])
    pl = orc.plan(P, G.complete(9), 0, False)
    assert pl["order"].tolist() == [0, 2, 1, 3, 4, 5, 6, 7]
    assert pl["parent"].tolist() == [-1, 0, 0, 0, 1, 1, 0, 2]


def test_order_domain_size_tie_break_and_singletons_first(orc):
    # pattern a(0)-b(1)-c(2) labelled X,Z,Y; target star centre Z with three X and two Y leaves
    X, Y, Z = 0, 1, 2
    T = G.from_edges(6, [(0, i) for i in range(1, 6)], [Z, X, X, X, Y, Y])
    P = G.from_edges(3, [(0, 1), (1, 2)], [X, Z, Y])
    assert orc.plan(P, T, 0, True)["order"].tolist() == [1, 0, 2]      # RI: degree, then lowest id
    assert orc.plan(P, T, 1, True)["order"].tolist() == [1, 0, 2]      # RI-DS: singleton D(b) first
    assert orc.plan(P, T, 2, True)["order"].tolist() == [1, 2, 0]      # SI: |D(c)|=2 < |D(a)|=3
    assert orc.plan(P, T, 3, True)["order"].tolist() == [1, 2, 0]


def test_singletons_first_in_id_order(orc):
    # unique labels make every domain a singleton: order is ascending id
    P = G.relabel(G.path(4), [3, 2, 1, 0])
    T = G.relabel(G.path(4), [3, 2, 1, 0])
    for mode in (1, 2, 3):
        assert orc.plan(P, T, mode, True)["order"].tolist() == [0, 1, 2, 3]


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("j", range(0, 100, 7))
def test_c1_invariants(orc, j):
    inst = synth.c1_instance(j)
    P, T = inst.pattern, inst.target
    res = {m: orc.run(P, T, m, True, rows=True) for m in MODES}
    base = _sorted(res[0]["rows"])
    assert res[0]["matches"] >= 1
    for m in MODES:
        assert np.array_equal(_sorted(res[m]["rows"]), base)
    # planted embedding present; every row verifies
    assert any(np.array_equal(r, inst.planted) for r in base)
    AT = G.adjacency(T)
    for r in base:
        assert len(set(r.tolist())) == P.n
        assert all(T.labels[r[u]] == P.labels[u] for u in range(P.n))
        assert all(AT[r[u], r[int(w)]] for u in range(P.n) for w in P.neighbours(u))
    # labelled matches are a subset of unlabelled ones
    un = orc.run(P, T, 0, False, state_cap=2 * 10**6)
    if un["status"] == 0:
        assert un["matches"] >= base.shape[0]
    # forward checking never grows the search (same order rules, smaller domains)
    assert res[3]["states"] <= res[2]["states"]
    # domain soundness
    for mode in (1, 2, 3):
        dom = orc.plan(P, T, mode, True)["domains"]
        for r in base:
            assert all(dom[u, r[u]] for u in range(P.n))


@pytest.mark.parametrize("j", [0, 5, 11])
def test_relabelling_equivariance(orc, j):
    inst = synth.c1_instance(j)
    P, T = inst.pattern, inst.target
    g = np.random.default_rng(j)
    pi = g.permutation(T.n)                      # new id of target node v is pi[v]
    e = [(int(pi[v]), int(pi[w])) for v in range(T.n) for w in T.neighbours(v) if v < w]
    lab = np.empty(T.n, dtype=np.uint32)
    lab[pi] = T.labels
    T2 = G.from_edges(T.n, e, lab)
    a = orc.run(P, T, 0, True, rows=True)
    b = orc.run(P, T2, 0, True, rows=True)
    assert np.array_equal(_sorted(pi[a["rows"]].astype(np.uint32)), _sorted(b["rows"]))
    # pattern relabelling permutes columns
    sg = g.permutation(P.n)                      # new pattern id of u is sg[u]
    pe = [(int(sg[u]), int(sg[w])) for u in range(P.n) for w in P.neighbours(u) if u < w]
    plab = np.empty(P.n, dtype=np.uint32)
    plab[sg] = P.labels
    P2 = G.from_edges(P.n, pe, plab)
    c = orc.run(P2, T, 0, True, rows=True)
    cols = np.empty(P.n, dtype=np.int64)
    cols[sg] = np.arange(P.n)
    assert np.array_equal(_sorted(c["rows"][:, sg]), _sorted(a["rows"]))


def _arc_consistent(P, T, dom):
    for u in range(P.n):
        for v in np.flatnonzero(dom[u]):
            for w in P.neighbours(u):
                if not dom[int(w), T.neighbours(int(v))].any():
                    return False
    return True


@pytest.mark.parametrize("j", range(8))
def test_domains_arc_consistent_and_sound(orc, j):
    inst = synth.c2_instance(j)
    P, T = inst.pattern, inst.target
    r = orc.run(P, T, 0, True, rows=True)
    for mode in (1, 2):
        pl = orc.plan(P, T, mode, True)
        assert _arc_consistent(P, T, pl["domains"])
        for row in r["rows"]:
            assert all(pl["domains"][u, row[u]] for u in range(P.n))


# ----------------------------------------------------------------- edge cases
def test_empty_pattern_single_match(orc):
    r = orc.run(G.edgeless(0), G.complete(3), 0, False, rows=True)
    assert r["matches"] == 1 and r["states"] == 0


def test_pattern_larger_than_target(orc):
    for mode in MODES:
        assert orc.run(G.path(5), G.complete(4), mode, False)["matches"] == 0


def test_self_loop_rejected(orc):
    bad = synth.Graph(2, np.array([0, 2, 3], np.uint32), np.array([0, 1, 0], np.uint32), np.zeros(2, np.uint32))
    with pytest.raises(ValueError):
        orc.run(G.path(2), bad, 0, False)


def test_asymmetric_rejected(orc):
    bad = synth.Graph(2, np.array([0, 1, 1], np.uint32), np.array([1], np.uint32), np.zeros(2, np.uint32))
    with pytest.raises(ValueError):
        orc.run(G.path(2), bad, 0, False)


def test_state_cap(orc):
    inst = synth.c2_instance(2)
    full = orc.run(inst.pattern, inst.target, 0, True)
    assert full["status"] == 0
    at = orc.run(inst.pattern, inst.target, 0, True, state_cap=full["states"])
    assert at["status"] == 0 and at["matches"] == full["matches"]
    below = orc.run(inst.pattern, inst.target, 0, True, state_cap=full["states"] - 1)
    assert below["status"] == 2


def test_row_capacity(orc):
    full = orc.run(G.path(3), G.complete(5), 0, False, rows=True)
    part = orc.run(G.path(3), G.complete(5), 0, False, rows=True, cap_rows=7)
    assert part["matches"] == full["matches"] == 60
    assert part["rows"].shape == (7, 3)
    fullset = {tuple(r) for r in full["rows"].tolist()}
    assert all(tuple(r) in fullset for r in part["rows"].tolist())


def test_root_shards_partition_the_search(orc):
    """Restricting the first node of the order to disjoint ranges of target ids
    splits the search tree by its first level: counts add up to the whole."""
    inst = synth.c2_instance(5)
    full = orc.run(inst.pattern, inst.target, 0, True, rows=True)
    parts = [orc.run(inst.pattern, inst.target, 0, True, rows=True, root_range=(lo, hi))
             for lo, hi in [(0, 1000), (1000, 1001), (1001, 3000)]]
    assert sum(p["matches"] for p in parts) == full["matches"]
    assert sum(p["states"] for p in parts) == full["states"]
    allrows = np.concatenate([p["rows"] for p in parts])
    assert np.array_equal(_sorted(allrows), _sorted(full["rows"]))
    order0 = orc.plan(inst.pattern, inst.target, 0, True)["order"][0]
    for p, (lo, hi) in zip(parts, [(0, 1000), (1000, 1001), (1001, 3000)]):
        assert all(lo <= r[order0] < hi for r in p["rows"])


# ------------------------------------------------- algorithmic bytes (roofline numerator)
# The byte model (bytes a search must read, per unit of work): sparse, per
# expansion with a parent 8 + 4 deg(parent image); per candidate 5 B (RI) or
# 8 B (RI-DS); per parentless RI-DS candidate 4 B more (the domain list); 8 B
# per back-edge probe up to the first failure.  Dense, per expansion 8W bytes
# per row read: domain, parent (if any), each back-edge.  Neither counts rows.

@pytest.mark.parametrize("seed", range(60))
def test_bytes_brute_force_tiny(orc, seed):
    """The oracle's byte counters equal the model summed over the consistent
    prefixes that a brute force finds (the DFS itself is not used)."""
    g = np.random.default_rng(10_000 + seed)
    n = int(g.integers(3, 8))
    k = int(g.integers(2, min(5, n) + 1))
    nlab = int(g.integers(1, 3))
    T = G.random_graph(g, n, float(g.uniform(0.3, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.4, 1.0)), nlab)
    labelled = bool(g.integers(0, 2))
    for mode in MODES:
        pl = orc.plan(P, T, mode, labelled)
        r = orc.run(P, T, mode, labelled)
        if pl["empty"]:
            assert r["alg_bytes"] == 0 and r["dense_bytes"] == 0
            continue
        want = G.brute_bytes(P, T, labelled, mode, pl["order"], pl["parent"], pl["domains"])
        assert (r["alg_bytes"], r["dense_bytes"]) == want, (seed, mode)


@pytest.mark.parametrize("n,k", [(6, 1), (6, 3), (7, 4), (6, 6), (9, 5), (70, 3)])
@pytest.mark.parametrize("mode", MODES)
def test_bytes_clique_in_clique_closed_form(orc, n, k, mode):
    """K_k in K_n, unlabelled.  The order is 0..k-1 with every parent at
    position 0 and back(i) = {1..i-1}.  Position 0 reads no list: its n
    candidates cost 5 B each in RI, 4 + 8 B in RI-DS.  Position i >= 1 is
    expanded once per injective i-prefix (P(n, i) of them): 8 + 4(n-1) bytes
    of the parent's list, n-1 candidates, of which n-i are unused and probe all
    i-1 back-edges successfully."""
    r = orc.run(G.complete(k), G.complete(n), mode, False)
    per_cand = 5 if mode == 0 else 8
    root = 5 * n if mode == 0 else 12 * n
    want = root + sum(math.perm(n, i) * (8 + 4 * (n - 1) + per_cand * (n - 1) + 8 * (i - 1) * (n - i))
                      for i in range(1, k))
    W = (n + 63) // 64
    want_dense = 8 * W * (1 + sum(math.perm(n, i) * (i + 1) for i in range(1, k)))
    assert r["alg_bytes"] == want
    assert r["dense_bytes"] == want_dense


def _k4_bytes(T):
    """Closed form of the byte counters for K_4 in a target T (RI, unlabelled),
    from the adjacency matrix.  The order is 0,1,2,3, every parent at position
    0, back(2) = {1}, back(3) = {1, 2}.  s = nodes of degree >= 3 (rule 3),
    B = A restricted to them.  A state (v0, v1) probes v1's row once for each
    other qualifying neighbour v2 of v0 ((B1)_v0 - 1 of them); a state
    (v0, v1, v2) probes v1's row for each qualifying neighbour v3 of v0 other
    than v1 and v2, and v2's row only when that first probe succeeds
    ((B^2)_{v0 v1} - 1 of them: v2 itself is a common neighbour)."""
    A = G.adjacency(T).astype(np.int64)
    n = T.n
    d = A.sum(1)
    s = (d >= 3).astype(np.int64)
    B = A * np.outer(s, s)
    B2 = B @ B
    r1 = B.sum(1)
    f = 8 + 9 * d                                      # list bounds + 4 B/id + 5 B/candidate
    pos0 = 5 * n
    pos1 = int((s * f).sum())
    pos2 = int((B * (f + 8 * (r1 - 1))[:, None]).sum())
    tri = B * B2                                       # (v0, v1) -> number of v2 closing a triangle
    pos3 = int((tri * (f[:, None] + 8 * ((r1 - 2)[:, None] + B2 - 1))).sum())
    W = (n + 63) // 64
    states0, states1, states2 = int(s.sum()), int(B.sum()), int(tri.sum())
    dense = 8 * W * (1 + 2 * states0 + 3 * states1 + 4 * states2)
    return pos0 + pos1 + pos2 + pos3, dense


@pytest.mark.parametrize("seed", range(4))
def test_bytes_k4_closed_form(orc, seed):
    g = np.random.default_rng(seed)
    T = G.random_graph(g, 40, 0.3, 1)
    r = orc.run(G.complete(4), T, 0, False)
    assert (r["alg_bytes"], r["dense_bytes"]) == _k4_bytes(T)


def test_bytes_k4_closed_form_c1_target(orc):
    T = synth.c1_instance(0).target
    r = orc.run(G.complete(4), T, 0, False)
    assert (r["alg_bytes"], r["dense_bytes"]) == _k4_bytes(T)


def test_bytes_exclude_rows(orc):
    """The byte counters are those of a count-only search: asking for the rows
    (4k bytes written per match) changes neither."""
    inst = synth.c1_instance(3)
    for mode in (0, 3):
        a = orc.run(inst.pattern, inst.target, mode, True)
        b = orc.run(inst.pattern, inst.target, mode, True, rows=True)
        assert b["matches"] > 0
        assert (a["alg_bytes"], a["dense_bytes"]) == (b["alg_bytes"], b["dense_bytes"])


def test_bytes_over_root_shards(orc):
    """Disjoint root ranges partition a search: states, matches and the
    sparse bytes add up exactly; the bitset model charges each search's root
    expansion (one domain row) once, so the shards' dense bytes exceed the
    whole search's by one row per extra shard (the rule the full-size dense
    golden values are summed by)."""
    inst = synth.c1_instance(7)
    T, P = inst.target, inst.pattern
    W = (T.n + 63) // 64
    for mode in (0, 3):
        whole = orc.run(P, T, mode, True)
        cuts = [0, 37, 90, 150, T.n]
        parts = [orc.run(P, T, mode, True, root_range=(a, b)) for a, b in zip(cuts, cuts[1:])]
        for key in ("states", "matches", "alg_bytes"):
            assert sum(p[key] for p in parts) == whole[key]
        assert sum(p["dense_bytes"] for p in parts) - (len(parts) - 1) * 8 * W == whole["dense_bytes"]
