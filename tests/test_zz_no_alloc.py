"""The allocation-free count (every device buffer in the library's static
scratch array) against sge_count through the C ABI: two calls in a row, the
second on a smaller input, then the dense kernel on a root shard, and the
size check that refuses an instance larger than the array."""
from __future__ import annotations

import json
import os
import sys

import pytest

import graphs as G
from paper_1705_09358_amd import sge, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = sge.Context(0)
    c.set_time_limit(60000)
    yield c
    c.close()


def both(ctx, th, ph, mode, labelled=True):
    ctx.set_mode(mode)
    ctx.set_labelled(labelled)
    want = ctx.count(th, ph)
    got = ctx.count_noalloc(th, ph)
    assert got.status == sge.OK
    assert (got.matches, got.states, got.alg_bytes) == (want.matches, want.states, want.alg_bytes)
    return got


def test_two_calls_second_smaller(ctx):
    targets = [synth.c5_target(t) for t in range(synth.C5_TARGETS)]
    q = next(q for q in range(200) if synth.c5_query(q, targets)[1].n >= 48)
    t, P, _ = synth.c5_query(q, targets)
    th, ph = ctx.load_target(targets[t]), ctx.load_pattern(P)
    _note(f"noalloc: serving query {q} (n={targets[t].n}, k={P.n}), then c1/0")
    big = both(ctx, th, ph, sge.RIDS_SI_FC)
    inst = synth.c1_instance(0)
    th2, ph2 = ctx.load_target(inst.target), ctx.load_pattern(inst.pattern)
    small = both(ctx, th2, ph2, sge.RI)
    assert big.states > 0 and small.matches > 0
    # and back to the larger one: nothing of the earlier calls leaks into it
    assert both(ctx, th, ph, sge.RIDS_SI_FC).states == big.states
    for h in (ph, ph2):
        ctx.unload_pattern(h)
    for h in (th, th2):
        ctx.unload_target(h)


def test_contact3000_and_dense_shard(ctx):
    man = json.load(open(os.path.join(GOLDEN, "c2.json")))
    r = man["instances"][28]
    inst = synth.c2_instance(r["j"], r["attempt"])
    th, ph = ctx.load_target(inst.target), ctx.load_pattern(inst.pattern)
    _note("noalloc: contact-3000 pattern 28")
    got = both(ctx, th, ph, sge.RI)
    assert (got.matches, got.states) == (r["matches"], r["states"])
    ctx.unload_pattern(ph)
    ctx.unload_target(th)
    w = json.load(open(os.path.join(GOLDEN, "c3.json")))["instances"][0]
    inst = synth.c3_instance(w["j"], 0)
    th, ph = ctx.load_target(inst.target), ctx.load_pattern(inst.pattern)
    ctx.set_root_range(w["root_lo"], w["root_hi"])
    try:
        _note("noalloc: dense pattern 0 on a root shard")
        got = both(ctx, th, ph, sge.RIDS_SI_FC)
        assert (got.matches, got.states) == (w["matches"], w["states"])
    finally:
        ctx.set_root_range()
        ctx.unload_pattern(ph)
        ctx.unload_target(th)


def test_too_large_for_the_array_is_refused(ctx):
    """A 64-component pattern on a 600,000-node target needs a candidate list
    of 64 x 600,000 ids: far beyond the array, refused before any launch."""
    T = synth.contact_target(synth.rng(99, 0, 1, 0), 600_000)
    P = G.edgeless(64)
    th, ph = ctx.load_target(T), ctx.load_pattern(P)
    try:
        ctx.set_mode(sge.RI)
        ctx.set_labelled(False)
        with pytest.raises(sge.SgeError) as e:
            ctx.count_noalloc(th, ph)
        assert e.value.code == sge.E_INVAL and "scratch" in str(e.value)
    finally:
        ctx.unload_pattern(ph)
        ctx.unload_target(th)
