"""GPU parity of the plan kernel: the order, parents, final domains and root
count that the device computes before every search, against the oracle's plan
(ordering of Section "RI", domains of Section 4.1, forward checking of
Section 4.2.2, SI tie-break of Section 4.2.1)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphs as G
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.close()


class Planner:
    def __init__(self, ctx):
        self.ctx = ctx
        self.tcache = {}

    def target(self, T):
        if id(T) not in self.tcache:
            self.tcache[id(T)] = (T, self.ctx.load_target(T))
        return self.tcache[id(T)][1]

    def check(self, orc, P, T, mode, labelled, root=None):
        th = self.target(T)
        ph = self.ctx.load_pattern(P)
        try:
            if root is not None:
                self.ctx.set_root_range(*root)
            b = self.ctx.plan_device(th, ph, P.n, T.n, mode, labelled)
        finally:
            if root is not None:
                self.ctx.set_root_range(0, 0xFFFFFFFF)
            self.ctx.unload_pattern(ph)
        a = orc.plan(P, T, mode, labelled)
        assert a["empty"] == b["empty"], (mode, labelled)
        if a["empty"] or P.n == 0:
            return b
        assert a["order"].tolist() == b["order"].tolist(), (mode, labelled)
        assert a["parent"].tolist() == b["parent"].tolist(), (mode, labelled)
        if mode != sge.RI:
            assert np.array_equal(a["domains"], b["domains"]), (mode, labelled)
        # root candidates: the first position's domain (RI-DS) or the nodes
        # passing its label and degree rules (RI), within the root range
        u0 = int(a["order"][0])
        if mode != sge.RI:
            cand = a["domains"][u0]
        else:
            tdeg, pdeg = T.degrees(), P.degrees()
            cand = tdeg >= pdeg[u0]
            if labelled:
                cand &= T.labels == P.labels[u0]
        lo, hi = root if root is not None else (0, T.n)
        idx = np.arange(T.n)
        assert b["nroot"] == int((cand & (idx >= lo) & (idx < hi)).sum())
        return b


@pytest.fixture(scope="module")
def planner(ctx):
    return Planner(ctx)


@pytest.mark.parametrize("seed", range(40))
def test_plan_tiny_random(planner, orc, seed):
    _note(f"plan tiny seed {seed}")
    g = np.random.default_rng(2000 + seed)
    n = int(g.integers(2, 14))
    k = int(g.integers(1, min(8, n) + 1))
    nlab = int(g.integers(1, 4))
    T = G.random_graph(g, n, float(g.uniform(0.2, 0.9)), nlab)
    P = G.random_graph(g, k, float(g.uniform(0.2, 1.0)), nlab)
    for mode in range(4):
        for labelled in (False, True):
            planner.check(orc, P, T, mode, labelled)


def test_plan_paper_forward_checking_example(planner, orc):
    # singletons first and the forward-checking cascade on the star target
    X, Y, Z = 0, 1, 2
    T = G.from_edges(6, [(0, i) for i in range(1, 6)], [Z, X, X, X, Y, Y])
    P = G.from_edges(3, [(0, 1), (1, 2)], [X, Z, Y])
    b = planner.check(orc, P, T, sge.RIDS_SI_FC, True)
    assert b["order"].tolist() == [1, 2, 0]


@pytest.mark.parametrize("cfg,j", [("c1", 0), ("c1", 37), ("c2", 0), ("c2", 28), ("c2", 61), ("c3", 0), ("c3", 7),
                                   ("c4", 0), ("c4", 3), ("c4", 17), ("c4", 1000)])
def test_plan_workloads(planner, orc, cfg, j):
    inst = {"c1": synth.c1_instance, "c2": synth.c2_instance, "c3": synth.c3_instance,
            "c4": synth.c4_instance}[cfg](j)
    _note(f"plan {cfg}/{j}: n={inst.target.n} k={inst.pattern.n}")
    for mode in range(4):
        planner.check(orc, inst.pattern, inst.target, mode, True)
    planner.check(orc, inst.pattern, inst.target, sge.RIDS_SI_FC, False)


def test_plan_root_ranges(planner, orc):
    inst = synth.c2_instance(3)
    for lo, hi in [(0, 1), (100, 1500), (2990, 3000), (2999, 0xFFFFFFFF)]:
        for mode in (sge.RI, sge.RIDS_SI_FC):
            planner.check(orc, inst.pattern, inst.target, mode, True, root=(lo, hi))


def test_plan_serving_targets(planner, orc):
    targets = [synth.c5_target(t) for t in (0, 1)]
    for q in range(6):
        ti, P, _ = synth.c5_query(q, targets)
        _note(f"plan c5 query {q}: n={targets[ti].n} k={P.n}")
        planner.check(orc, P, targets[ti], sge.RIDS_SI_FC, True)


def test_plan_disconnected_pattern(planner, orc):
    # three components: three parentless positions, each with its own list
    T = G.petersen()
    P = G.from_edges(6, [(0, 1), (2, 3)])
    for mode in range(4):
        b = planner.check(orc, P, T, mode, False)
        assert (b["parent"] < 0).sum() == 4   # components {0,1}, {2,3}, {4}, {5}


@pytest.mark.parametrize("words", [4112, 8208])
def test_plan_wide_target_support_in_global_memory(planner, orc, words):
    # rows of 4112 words: the bit-row support sets live in LDS, one dirty
    # node per batch; more than 8192 words (the plan kernel's LDS budget):
    # they live in device memory
    g = np.random.default_rng(77)
    n = 64 * words - 24
    src = g.integers(0, n, size=3 * n)
    dst = g.integers(0, n, size=3 * n)
    keep = src != dst
    rp, col = synth.csr_from_edges(n, src[keep], dst[keep])
    T = synth.Graph(n, rp, col, g.integers(0, 3, size=n).astype(np.uint32))
    P = G.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [0, 1, 0, 2])
    _note(f"plan wide target: n={n}, {(n + 63) // 64} words per row")
    for mode in (sge.RIDS, sge.RIDS_SI_FC):
        planner.check(orc, P, T, mode, True)


def _many_label_instance(seed: int, n: int, nlab: int, k: int):
    # a contact-like target with `nlab` uniformly drawn labels and a
    # random-walk pattern on it, so that more pattern labels occur than the
    # plan kernel packs per target node (24 table columns)
    g = np.random.default_rng(seed)
    T = synth.contact_target(g, n)
    T = synth.Graph(T.n, T.row_ptr, T.col, g.integers(0, nlab, size=T.n).astype(np.uint32))
    P, _ = synth.induced_pattern(g, T, synth.walk_selection(g, T, k))
    return T, P


@pytest.mark.parametrize("n", [1500, 7000])
def test_plan_more_pattern_labels_than_packed_columns(planner, orc, n):
    # over 24 distinct labels among the pattern's nodes: the first
    # arc-consistency round cannot use the packed table bytes; on the
    # register path (n <= 6144) the rounds start from every node with a
    # neighbour, on the row path the table round reads column by column
    T, P = _many_label_instance(91 + n, n, 48, 56)
    distinct = len(set(P.labels.tolist()))
    _note(f"plan many labels: n={T.n} k={P.n} distinct pattern labels {distinct}")
    assert distinct > 24
    for mode in range(4):
        planner.check(orc, P, T, mode, True)


@pytest.mark.parametrize("n", [64 * 96, 64 * 96 + 1])
def test_plan_register_path_boundary(planner, orc, n):
    # 96 words (6144 nodes) is the widest target whose domain memberships the
    # plan kernel keeps in registers; one node more takes the support-row path
    g = np.random.default_rng(5000 + n)
    T = synth.contact_target(g, n)
    P, _ = synth.induced_pattern(g, T, synth.walk_selection(g, T, 40))
    _note(f"plan register boundary: n={T.n} k={P.n}")
    for mode in (sge.RIDS, sge.RIDS_SI_FC):
        planner.check(orc, P, T, mode, True)
        planner.check(orc, P, T, mode, False)
