"""Small named graphs and a brute-force enumerator used to pin the oracle.

The brute force checks only the problem definition (Section 2.1, eqs. (2)-(3),
non-induced): every injection V_p -> V_t is tried and kept when labels agree
(if labelled) and every pattern edge lands on a target edge.
"""
from __future__ import annotations

import itertools

import numpy as np

from paper_1705_09358_amd.synth import Graph, csr_from_edges


def from_edges(n: int, edges, labels=None) -> Graph:
    e = np.array(list(edges), dtype=np.int64).reshape(-1, 2)
    rp, col = csr_from_edges(n, e[:, 0], e[:, 1])
    lab = np.zeros(n, dtype=np.uint32) if labels is None else np.asarray(labels, dtype=np.uint32)
    return Graph(n, rp, col, lab)


def complete(n: int) -> Graph:
    return from_edges(n, itertools.combinations(range(n), 2))


def cycle(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def path(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def star(m: int) -> Graph:
    return from_edges(m + 1, [(0, i) for i in range(1, m + 1)])


def complete_bipartite(a: int, b: int) -> Graph:
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def edgeless(n: int) -> Graph:
    return from_edges(n, [])


def petersen() -> Graph:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return from_edges(10, outer + spokes + inner)


def hypercube(d: int) -> Graph:
    n = 1 << d
    return from_edges(n, [(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)])


def relabel(g: Graph, labels) -> Graph:
    return Graph(g.n, g.row_ptr, g.col, np.asarray(labels, dtype=np.uint32))


def adjacency(g: Graph) -> np.ndarray:
    A = np.zeros((g.n, g.n), dtype=bool)
    for v in range(g.n):
        A[v, g.neighbours(v)] = True
    return A


def brute_matches(P: Graph, T: Graph, labelled: bool) -> np.ndarray:
    """All edge- and label-preserving injections, rows in pattern-id order, sorted."""
    AT = adjacency(T)
    pe = [(u, int(w)) for u in range(P.n) for w in P.neighbours(u) if u < w]
    rows = []
    for m in itertools.permutations(range(T.n), P.n):
        if labelled and any(P.labels[u] != T.labels[m[u]] for u in range(P.n)):
            continue
        if all(AT[m[u], m[w]] for u, w in pe):
            rows.append(m)
    r = np.array(rows, dtype=np.uint32).reshape(-1, P.n)
    return r[np.lexsort(r.T[::-1])] if len(rows) > 1 else r


def brute_states(P: Graph, T: Graph, labelled: bool, order, domains) -> int:
    """Number of consistent prefix assignments summed over prefix lengths 1..k.

    A prefix assignment of positions 0..d-1 is consistent when it is injective,
    each assigned pair passes the unary checks (label when labelled, pattern
    degree <= target degree, membership in the domain when domains are given)
    and every pattern edge inside the prefix maps onto a target edge.
    """
    AT = adjacency(T)
    AP = adjacency(P)
    tdeg = T.degrees()
    pdeg = P.degrees()
    total = 0
    order = [int(u) for u in order]

    def unary(u, v):
        if labelled and P.labels[u] != T.labels[v]:
            return False
        if pdeg[u] > tdeg[v]:
            return False
        return domains is None or bool(domains[u, v])

    for d in range(1, P.n + 1):
        us = order[:d]
        for m in itertools.permutations(range(T.n), d):
            if not all(unary(us[i], m[i]) for i in range(d)):
                continue
            if all(AT[m[i], m[j]] for i in range(d) for j in range(i) if AP[us[i], us[j]]):
                total += 1
    return total


def random_graph(g: np.random.Generator, n: int, p: float, nlab: int) -> Graph:
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if g.random() < p]
    return from_edges(n, edges, g.integers(0, nlab, size=n))


# ---------------------------------------------------------------- directed and edge-labelled graphs

def from_arcs(n: int, arcs, labels=None, elabels=None, directed: bool = True) -> Graph:
    """CSR of the arcs (a, b) (sorted rows); elabels[i] is the label of arcs[i].
    With directed=False every arc must appear in both directions."""
    arcs = [tuple(int(x) for x in a) for a in arcs]
    el = [0] * len(arcs) if elabels is None else [int(x) for x in elabels]
    order = sorted(range(len(arcs)), key=lambda i: arcs[i])
    rp = np.zeros(n + 1, dtype=np.uint32)
    for a, _ in arcs:
        rp[a + 1] += 1
    rp = np.cumsum(rp).astype(np.uint32)
    col = np.array([arcs[i][1] for i in order], dtype=np.uint32)
    elab = np.array([el[i] for i in order], dtype=np.uint32) if elabels is not None else None
    lab = np.zeros(n, dtype=np.uint32) if labels is None else np.asarray(labels, dtype=np.uint32)
    return Graph(n, rp, col, lab, elab, directed)


def arcs_of(g: Graph):
    """{(a, b): label} over the CSR entries."""
    out = {}
    for a in range(g.n):
        for e in range(int(g.row_ptr[a]), int(g.row_ptr[a + 1])):
            out[(a, int(g.col[e]))] = 0 if g.elabels is None else int(g.elabels[e])
    return out


def reverse(g: Graph) -> Graph:
    arcs = arcs_of(g)
    return from_arcs(g.n, [(b, a) for a, b in arcs], g.labels, [arcs[x] for x in arcs] if g.elabels is not None
                     else None, g.directed)


def random_digraph(g: np.random.Generator, n: int, p: float, nlab: int, nelab: int) -> Graph:
    arcs, el = [], []
    for a in range(n):
        for b in range(n):
            if a != b and g.random() < p:
                arcs.append((a, b))
                el.append(int(g.integers(0, nelab)))
    return from_arcs(n, arcs, g.integers(0, nlab, size=n), el if nelab > 1 else None)


def random_undirected_elabelled(g: np.random.Generator, n: int, p: float, nlab: int, nelab: int) -> Graph:
    arcs, el = [], []
    for a in range(n):
        for b in range(a + 1, n):
            if g.random() < p:
                lb = int(g.integers(0, nelab))
                arcs += [(a, b), (b, a)]
                el += [lb, lb]
    return from_arcs(n, arcs, g.integers(0, nlab, size=n), el, directed=False)


def brute_matches_ex(P: Graph, T: Graph, labelled: bool) -> np.ndarray:
    """All injections mapping every pattern arc onto a target arc (with equal
    node and edge labels when labelled), rows in pattern-id order, sorted."""
    pa, ta = arcs_of(P), arcs_of(T)
    rows = []
    for m in itertools.permutations(range(T.n), P.n):
        if labelled and any(P.labels[u] != T.labels[m[u]] for u in range(P.n)):
            continue
        if all((m[a], m[b]) in ta and (not labelled or ta[(m[a], m[b])] == lb) for (a, b), lb in pa.items()):
            rows.append(m)
    r = np.array(rows, dtype=np.uint32).reshape(-1, P.n)
    return r[np.lexsort(r.T[::-1])] if len(rows) > 1 else r


def brute_states_ex(P: Graph, T: Graph, labelled: bool, order, domains) -> int:
    """Consistent prefix assignments (summed over prefix lengths 1..k): injective,
    unary checks (label, out-degree, in-degree, domain) and every pattern arc
    inside the prefix on a target arc of the same label (labelled)."""
    pa, ta = arcs_of(P), arcs_of(T)
    pout = np.diff(P.row_ptr.astype(np.int64))
    tout = np.diff(T.row_ptr.astype(np.int64))
    pin = np.bincount(P.col.astype(np.int64), minlength=P.n) if P.col.size else np.zeros(P.n, np.int64)
    tin = np.bincount(T.col.astype(np.int64), minlength=T.n) if T.col.size else np.zeros(T.n, np.int64)
    order = [int(u) for u in order]

    def unary(u, v):
        if labelled and P.labels[u] != T.labels[v]:
            return False
        if pout[u] > tout[v] or pin[u] > tin[v]:
            return False
        return domains is None or bool(domains[u, v])

    total = 0
    for d in range(1, P.n + 1):
        us = order[:d]
        pos = {u: i for i, u in enumerate(us)}
        inner = [(pos[a], pos[b], lb) for (a, b), lb in pa.items() if a in pos and b in pos]
        for m in itertools.permutations(range(T.n), d):
            if not all(unary(us[i], m[i]) for i in range(d)):
                continue
            if all((m[i], m[j]) in ta and (not labelled or ta[(m[i], m[j])] == lb) for i, j, lb in inner):
                total += 1
    return total


def brute_ac_domains(P: Graph, T: Graph, labelled: bool) -> np.ndarray:
    """Greatest arc-consistent domains by naive iteration: start from label,
    out-degree and in-degree compatibility; remove v from D(u) while some
    pattern arc u -> w (w -> u) has no target arc v -> x (x -> v) of the same
    label (labelled) with x in D(w).  Returns bool [k, n]."""
    pa, ta = arcs_of(P), arcs_of(T)
    pout = np.diff(P.row_ptr.astype(np.int64))
    tout = np.diff(T.row_ptr.astype(np.int64))
    pin = np.bincount(P.col.astype(np.int64), minlength=P.n) if P.col.size else np.zeros(P.n, np.int64)
    tin = np.bincount(T.col.astype(np.int64), minlength=T.n) if T.col.size else np.zeros(T.n, np.int64)
    D = np.zeros((P.n, T.n), dtype=bool)
    for u in range(P.n):
        for v in range(T.n):
            D[u, v] = (not labelled or P.labels[u] == T.labels[v]) and pout[u] <= tout[v] and pin[u] <= tin[v]
    changed = True
    while changed:
        changed = False
        for u in range(P.n):
            for v in range(T.n):
                if not D[u, v]:
                    continue
                ok = True
                for (a, b), lb in pa.items():
                    if a == u:
                        ok = any(x == v and D[b, y] and (not labelled or tl == lb) for (x, y), tl in ta.items())
                    elif b == u:
                        ok = any(y == v and D[a, x] and (not labelled or tl == lb) for (x, y), tl in ta.items())
                    if not ok:
                        break
                if not ok:
                    D[u, v] = False
                    changed = True
    return D


def brute_bytes(P: Graph, T: Graph, labelled: bool, mode: int, order, parent, domains) -> tuple[int, int]:
    """Algorithmic bytes of a count-only search by the per-unit model, summed
    over the consistent prefixes found by brute force (undirected graphs
    without edge labels).  Every consistent prefix of positions 0..i-1 (the
    empty prefix for i = 0) is expanded once at position i < k.

    Sparse model, per expansion: with a parent, 8 bytes of list bounds and 4
    per id in the parent image's neighbour list; without one, nothing (RI: all
    target ids) or 4 bytes per member of the domain (RI-DS).  Per candidate, 5
    bytes (RI) or 8 (RI-DS); a candidate that passes the unary checks and is
    unused has its back-edges probed at 8 bytes each, earliest position first,
    up to and including the first one that fails.  Dense model, per expansion:
    8W bytes for the domain row, 8W for the parent row (when there is a
    parent) and 8W per back-edge row.  Returns (sparse, dense)."""
    AT = adjacency(T)
    AP = adjacency(P)
    tdeg = T.degrees()
    pdeg = P.degrees()
    k, n = P.n, T.n
    use_dom = mode != 0
    W = (n + 63) // 64
    order = [int(u) for u in order]

    def unary(u, v):
        if labelled and P.labels[u] != T.labels[v]:
            return False
        if pdeg[u] > tdeg[v]:
            return False
        return not use_dom or bool(domains[u, v])

    def consistent(m):
        us = order[:len(m)]
        if not all(unary(us[i], m[i]) for i in range(len(m))):
            return False
        return all(AT[m[i], m[j]] for i in range(len(m)) for j in range(i) if AP[us[i], us[j]])

    sparse = dense = 0
    for i in range(k):
        u = order[i]
        par = int(parent[i])
        back = [j for j in range(i) if j != par and AP[order[j], u]]
        for m in itertools.permutations(range(n), i):
            if not consistent(m):
                continue
            dense += 8 * W * (1 + (par >= 0) + len(back))
            if par >= 0:
                cands = np.flatnonzero(AT[m[par]])
                sparse += 8 + 4 * len(cands)
            elif use_dom:
                cands = np.flatnonzero(domains[u])
                sparse += 4 * len(cands)
            else:
                cands = range(n)
            for v in cands:
                sparse += 8 if use_dom else 5
                if v in m or not unary(u, v):
                    continue
                for j in back:
                    sparse += 8
                    if not AT[m[j], v]:
                        break
    return sparse, dense
