"""Seeded synthetic workloads for subgraph enumeration.

This module only *generates inputs*: target graphs, pattern graphs extracted
from them, labels, run modes and query arrival times.  It holds none of the
enumeration method's arithmetic and is shared by the tests, the benchmark and
the oracle harness.

Every draw comes from ``numpy.random.Generator(PCG64(SeedSequence([1705, 9358,
cfg, role, j, attempt])))`` with role 0 = target, 1 = pattern, 2 = mode or
arrival.  Graphs are simple and undirected and are returned as CSR with sorted
``uint32`` rows.

The paper's biochemical collections (PDBSv1, PPIS32, GRAEMLIN32; Section 5.1,
Table 1) are not available; the generators below stand in for them with the
shapes the paper reports: sparse labelled protein-contact-like targets (a
confined 3-D self-avoiding walk with a contact cutoff) and dense random
targets.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

MODE_RI, MODE_RIDS, MODE_RIDS_SI, MODE_RIDS_SI_FC = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_WALK_SO = os.path.join(_HERE, "_lib", "libsynth_walk.so")
_walk_lib = None


def _walk():
    global _walk_lib
    if _walk_lib is None:
        if not os.path.exists(_WALK_SO):
            from . import _build
            _build.build_synth()
        lib = ctypes.CDLL(_WALK_SO)
        lib.synth_saw.restype = ctypes.c_int
        lib.synth_saw.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p]
        lib.synth_contacts.restype = ctypes.c_int64
        lib.synth_contacts.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p]
        _walk_lib = lib
    return _walk_lib


def rng(cfg: int, role: int, j: int, attempt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1705, 9358, cfg, role, j, attempt])))


@dataclasses.dataclass
class Graph:
    """Simple graph in CSR form with sorted rows: both directions of every edge
    when undirected, the out-edges when ``directed``.  ``labels``: one uint32
    per node; ``elabels``: one uint32 per CSR entry (edge labels), or None."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    labels: np.ndarray
    elabels: np.ndarray | None = None
    directed: bool = False

    @property
    def m2(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def neighbours(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]


@dataclasses.dataclass
class Instance:
    """One (pattern, target) pair plus how it was drawn."""
    target: Graph
    pattern: Graph
    mode: int
    labelled: bool
    planted: np.ndarray          # planted[u] = target node of pattern node u
    name: str = ""


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR with sorted, de-duplicated rows from an undirected edge list (u != v)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * max(n, 1) + b)
    a = key // max(n, 1)
    b = key % max(n, 1)
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    np.add.at(row_ptr, a + 1, 1)
    row_ptr = np.cumsum(row_ptr, dtype=np.uint64).astype(np.uint32)
    return row_ptr, b.astype(np.uint32)


def er_edges(g: np.random.Generator, n: int, p: float) -> tuple[np.ndarray, np.ndarray]:
    """G(n, p): each of the n(n-1)/2 pairs independently with probability p."""
    iu, ju = np.triu_indices(n, k=1)
    keep = g.random(iu.shape[0]) < p
    return iu[keep], ju[keep]


def contact_xyz(g: np.random.Generator, n: int, c: float, step: float = 3.8) -> np.ndarray:
    """3-D self-avoiding walk, step 3.8, confined to a ball of radius c*2.2*n^0.38."""
    radius = c * 2.2 * (max(n, 2) ** 0.38)
    for _ in range(64):
        seed = int(g.integers(0, 2 ** 63))
        xyz = np.empty((n, 3), dtype=np.float64)
        rc = _walk().synth_saw(n, step, step, radius, seed, 64, 50 * n + 1000, xyz.ctypes.data)
        if rc == 0:
            return xyz
    raise RuntimeError("self-avoiding walk failed repeatedly")


def contact_csr(xyz: np.ndarray, cutoff: float = 8.0) -> tuple[np.ndarray, np.ndarray]:
    n = xyz.shape[0]
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    m2 = _walk().synth_contacts(n, xyz.ctypes.data, cutoff, row_ptr.ctypes.data, None)
    if m2 < 0:
        raise MemoryError("contact graph")
    col = np.empty(max(m2, 1), dtype=np.uint32)
    _walk().synth_contacts(n, xyz.ctypes.data, cutoff, row_ptr.ctypes.data, col.ctypes.data)
    return row_ptr, col[:m2]


# Confinement constant of the contact generator, chosen once so that the
# 3000-node target has mean degree in [8, 12] (measured value in the design notes).
CONTACT_C = 1.3


def zipf_labels(g: np.random.Generator, n: int, nsym: int = 20, s: float = 1.1) -> np.ndarray:
    w = np.arange(1, nsym + 1, dtype=np.float64) ** (-s)
    return g.choice(nsym, size=n, p=w / w.sum()).astype(np.uint32)


def contact_target(g: np.random.Generator, n: int, c: float = CONTACT_C) -> Graph:
    xyz = contact_xyz(g, n, c)
    rp, col = contact_csr(xyz)
    return Graph(n, rp, col, zipf_labels(g, n))


def er_target(g: np.random.Generator, n: int, p: float, nlab: int) -> Graph:
    u, v = er_edges(g, n, p)
    rp, col = csr_from_edges(n, u, v)
    return Graph(n, rp, col, g.integers(0, nlab, size=n).astype(np.uint32))


def induced_pattern(g: np.random.Generator, T: Graph, sel: list[int]) -> tuple[Graph, np.ndarray]:
    """Pattern on the selected target nodes with every target edge among them and
    their labels kept; pattern ids are a seeded permutation of selection order."""
    k = len(sel)
    perm = g.permutation(k)                 # pattern id of sel[j] is perm[j]
    pos = {int(t): int(perm[j]) for j, t in enumerate(sel)}
    us, vs = [], []
    for t in sel:
        for w in T.neighbours(int(t)):
            w = int(w)
            if w in pos and pos[int(t)] < pos[w]:
                us.append(pos[int(t)])
                vs.append(pos[w])
    rp, col = csr_from_edges(k, np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64))
    planted = np.empty(k, dtype=np.uint32)
    for j, t in enumerate(sel):
        planted[perm[j]] = t
    return Graph(k, rp, col, T.labels[planted].astype(np.uint32)), planted


def bfs_selection(g: np.random.Generator, T: Graph, k: int) -> list[int]:
    """First k nodes visited by a BFS from a uniform root with shuffled neighbour order."""
    for _ in range(10000):
        root = int(g.integers(0, T.n))
        seen = {root}
        order = [root]
        head = 0
        while head < len(order) and len(order) < k:
            v = order[head]
            head += 1
            nb = T.neighbours(v).copy()
            g.shuffle(nb)
            for w in nb:
                w = int(w)
                if w not in seen:
                    seen.add(w)
                    order.append(w)
                    if len(order) == k:
                        break
        if len(order) == k:
            return order
    raise RuntimeError("no component with k nodes")


def walk_selection(g: np.random.Generator, T: Graph, k: int, max_steps: int = 200000) -> list[int]:
    """Random walk from a uniform start to uniform neighbours until k distinct nodes."""
    for _ in range(10000):
        v = int(g.integers(0, T.n))
        if T.row_ptr[v + 1] == T.row_ptr[v] and k > 1:
            continue
        seen = {v}
        order = [v]
        steps = 0
        while len(order) < k and steps < max_steps:
            nb = T.neighbours(v)
            v = int(nb[int(g.integers(0, nb.shape[0]))])
            if v not in seen:
                seen.add(v)
                order.append(v)
            steps += 1
        if len(order) == k:
            return order
    raise RuntimeError("random walk could not reach k nodes")


def greedy_dense_selection(g: np.random.Generator, T: Graph, k: int) -> list[int]:
    """Connected subset grown from a uniform start by repeatedly adding the frontier
    node with the most edges into the current set (ties by a seeded shuffle)."""
    start = int(g.integers(0, T.n))
    sel = [start]
    inset = np.zeros(T.n, dtype=bool)
    inset[start] = True
    links = np.zeros(T.n, dtype=np.int64)
    links[T.neighbours(start)] += 1
    while len(sel) < k:
        cand = np.flatnonzero((links > 0) & ~inset)
        if cand.size == 0:
            raise RuntimeError("component smaller than k")
        best = cand[links[cand] == links[cand].max()]
        pick = int(best[g.permutation(best.size)[0]])
        sel.append(pick)
        inset[pick] = True
        links[T.neighbours(pick)] += 1
    return sel


# ---------------------------------------------------------------- configurations
# The five workloads: (1) plain RI on G(200, 0.05) with 8-node BFS patterns;
# (2) plain RI on a 3000-node contact graph with 100 random-walk patterns of
# 16-48 nodes; (3) RI-DS on dense G(1000, 0.3) with 50 dense patterns of 12-24
# nodes; (4) 4096 mixed-mode pairs on contact graphs with 100-5000 nodes and
# 8-64-node patterns; (5) serving queries of 4-64 nodes on 50 resident contact
# graphs of 5000-20000 nodes arriving as a Poisson process.

C1_COUNT, C2_COUNT, C3_COUNT, C4_COUNT = 100, 100, 50, 4096


def c1_instance(j: int, attempt: int = 0) -> Instance:
    T = er_target(rng(1, 0, j, attempt), 200, 0.05, 4)
    gp = rng(1, 1, j, attempt)
    P, planted = induced_pattern(gp, T, bfs_selection(gp, T, 8))
    return Instance(T, P, MODE_RI, True, planted, f"c1/{j}/{attempt}")


_c2_target = None


def c2_target() -> Graph:
    global _c2_target
    if _c2_target is None:
        _c2_target = contact_target(rng(2, 0, 0, 0), 3000)
    return _c2_target


def c2_instance(j: int, attempt: int = 0) -> Instance:
    T = c2_target()
    gp = rng(2, 1, j, attempt)
    k = int(gp.integers(16, 49))
    P, planted = induced_pattern(gp, T, walk_selection(gp, T, k))
    return Instance(T, P, MODE_RI, True, planted, f"c2/{j}/{attempt}")


_c3_target = None


def c3_target() -> Graph:
    global _c3_target
    if _c3_target is None:
        _c3_target = er_target(rng(3, 0, 0, 0), 1000, 0.3, 2)
    return _c3_target


def c3_instance(j: int, attempt: int = 0) -> Instance:
    T = c3_target()
    gp = rng(3, 1, j, attempt)
    k = int(gp.integers(12, 25))
    P, planted = induced_pattern(gp, T, greedy_dense_selection(gp, T, k))
    return Instance(T, P, MODE_RIDS_SI_FC, True, planted, f"c3/{j}/{attempt}")


def c4_instance(j: int, attempt: int = 0) -> Instance:
    gt = rng(4, 0, j, attempt)
    n = int(math.floor(math.exp(gt.uniform(math.log(100), math.log(5000)))))
    T = contact_target(gt, n)
    gp = rng(4, 1, j, attempt)
    k = min(n, int(math.floor(math.exp(gp.uniform(math.log(8), math.log(64))))))
    P, planted = induced_pattern(gp, T, walk_selection(gp, T, k))
    mode = MODE_RI if rng(4, 2, j, attempt).random() < 0.5 else MODE_RIDS_SI_FC
    return Instance(T, P, mode, True, planted, f"c4/{j}/{attempt}")


C5_TARGETS = 50
C5_RATE = 200.0


def c5_target(t: int) -> Graph:
    gt = rng(5, 0, t, 0)
    n = int(gt.integers(5000, 20001))
    return contact_target(gt, n)


def c5_arrivals(seconds: float, rate: float = C5_RATE) -> np.ndarray:
    """Open-loop Poisson arrival times (s) over [0, seconds)."""
    g = rng(5, 2, 0, 0)
    out = []
    t = 0.0
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= seconds:
            break
        out.append(t)
    return np.array(out, dtype=np.float64)


def c5_query(q: int, targets: list[Graph]) -> tuple[int, Graph, np.ndarray]:
    """Query q: (resident target index, pattern, planted embedding)."""
    g = rng(5, 1, q, 0)
    t = int(g.integers(0, len(targets)))
    k = int(g.integers(4, 65))
    P, planted = induced_pattern(g, targets[t], walk_selection(g, targets[t], k))
    return t, P, planted


# ---------------------------------------------------------------- directed workload
# The general problem (directed graphs, edge labels) on contact-like data: the
# 3000-node contact graph with each edge kept in both directions with
# probability 1/4 and otherwise in one uniformly chosen direction, every arc
# labelled with one of three bond types (uniform, drawn per arc).  100
# patterns, selected by a random walk over the undirected graph, with every
# arc among the selected nodes and its label: even j labelled (node and edge
# labels), 8-24 nodes, RI; odd j unlabelled (directions only), 4-7 nodes,
# RI-DS-SI-FC.
C2D_COUNT = 100
C2D_BOTH = 0.25
C2D_EDGE_LABELS = 3
_c2d_target = None


def arcs_csr(n: int, a: np.ndarray, b: np.ndarray, lab: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Out-edge CSR (sorted rows) of the arcs a[i] -> b[i] with labels lab[i] (no duplicates)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    order = np.argsort(a * max(n, 1) + b, kind="stable")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, a + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.uint32)
    return row_ptr, b[order].astype(np.uint32), np.asarray(lab, dtype=np.uint32)[order]


def orient(g: np.random.Generator, T: Graph, p_both: float = C2D_BOTH, nelab: int = C2D_EDGE_LABELS) -> Graph:
    """Directed, arc-labelled version of an undirected graph (see above)."""
    src = np.repeat(np.arange(T.n, dtype=np.int64), np.diff(T.row_ptr.astype(np.int64)))
    dst = T.col.astype(np.int64)
    keep = src < dst
    u, v = src[keep], dst[keep]
    r = g.random(u.shape[0])
    both = r < p_both
    fwd = (~both) & (r < p_both + (1.0 - p_both) / 2)
    bwd = ~(both | fwd)
    a = np.concatenate([u[both], v[both], u[fwd], v[bwd]])
    b = np.concatenate([v[both], u[both], v[fwd], u[bwd]])
    lab = g.integers(0, nelab, size=a.shape[0])
    rp, col, el = arcs_csr(T.n, a, b, lab)
    return Graph(T.n, rp, col, T.labels, el, True)


def induced_directed_pattern(g: np.random.Generator, T: Graph, sel: list[int]) -> tuple[Graph, np.ndarray]:
    """Pattern on the selected nodes of a directed target with every arc among
    them and its label; pattern ids are a seeded permutation of selection order."""
    k = len(sel)
    perm = g.permutation(k)
    pos = {int(t): int(perm[j]) for j, t in enumerate(sel)}
    a, b, lab = [], [], []
    for t in sel:
        t = int(t)
        for e in range(int(T.row_ptr[t]), int(T.row_ptr[t + 1])):
            w = int(T.col[e])
            if w in pos:
                a.append(pos[t])
                b.append(pos[w])
                lab.append(int(T.elabels[e]) if T.elabels is not None else 0)
    rp, col, el = arcs_csr(k, np.array(a, dtype=np.int64), np.array(b, dtype=np.int64), np.array(lab))
    planted = np.empty(k, dtype=np.uint32)
    for j, t in enumerate(sel):
        planted[perm[j]] = t
    return Graph(k, rp, col, T.labels[planted].astype(np.uint32), el, True), planted


def c2d_target() -> Graph:
    global _c2d_target
    if _c2d_target is None:
        _c2d_target = orient(rng(6, 0, 0, 0), c2_target())
    return _c2d_target


def c2d_instance(j: int, attempt: int = 0) -> Instance:
    T = c2d_target()
    gp = rng(6, 1, j, attempt)
    labelled = j % 2 == 0
    k = int(gp.integers(8, 25)) if labelled else int(gp.integers(4, 8))
    P, planted = induced_directed_pattern(gp, T, walk_selection(gp, c2_target(), k))
    mode = MODE_RI if labelled else MODE_RIDS_SI_FC
    return Instance(T, P, mode, labelled, planted, f"c2d/{j}/{attempt}")
