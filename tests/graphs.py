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
