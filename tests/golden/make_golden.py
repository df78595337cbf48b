"""Write the oracle's results for every workload instance to tests/golden/*.json.

Only the oracle and the seeded input generators are called here.  Each
instance is screened against the workload's deterministic states cap: an
instance whose search exceeds the cap is redrawn with the next `attempt`
(the counterpart of the paper's per-instance time limit), and the attempt
used is recorded.

    python tests/golden/make_golden.py c1 c2 c4 c3 c5 c2d [--procs 8]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, REPO)

import oracle  # noqa: E402
from paper_1705_09358_amd import synth  # noqa: E402

CAPS = {"c1": 10 ** 8, "c2": 10 ** 8, "c4": 10 ** 8, "c3": 0, "c5": 10 ** 7, "c2d": 10 ** 8}
C5_SAMPLE = 48   # serving queries checked against the oracle (the first of the arrival stream)
MAKERS = {"c1": synth.c1_instance, "c2": synth.c2_instance, "c4": synth.c4_instance, "c2d": synth.c2d_instance}
COUNTS = {"c1": synth.C1_COUNT, "c2": synth.C2_COUNT, "c4": synth.C4_COUNT, "c3": synth.C3_COUNT, "c5": C5_SAMPLE,
          "c2d": synth.C2D_COUNT}


def c3_shard(j):
    """Dense workload: the full search of a pattern is ~1e9 states, beyond the
    oracle; it is checked on a shard -- the first node of the order restricted
    to target ids [lo, lo + 2)."""
    inst = synth.c3_instance(j, 0)
    lo = (37 * j) % (inst.target.n - 2)
    t0 = time.perf_counter()
    r = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled, rows=True, cap_rows=1 << 20,
                   root_range=(lo, lo + 2))
    dt = time.perf_counter() - t0
    return dict(j=j, attempt=0, n=inst.target.n, k=inst.pattern.n, mode=inst.mode, labelled=inst.labelled,
                root_lo=lo, root_hi=lo + 2, matches=r["matches"], states=r["states"],
                candidates=r["candidates"], alg_bytes=r["alg_bytes"],
                sha256=oracle.rows_digest(r["rows"], inst.pattern.n), oracle_s=round(dt, 3))


_c5_targets = None


def c5_query(q):
    """Serving workload: query q of the arrival stream, state cap 1e7 (a query
    above it is reported as aborted, by the oracle and by the server alike)."""
    global _c5_targets
    if _c5_targets is None:
        _c5_targets = [synth.c5_target(t) for t in range(synth.C5_TARGETS)]
    t, P, planted = synth.c5_query(q, _c5_targets)
    T = _c5_targets[t]
    t0 = time.perf_counter()
    r = oracle.run(P, T, oracle.RIDS_SI_FC, True, state_cap=CAPS["c5"], rows=True, cap_rows=1 << 20)
    dt = time.perf_counter() - t0
    ok = r["status"] == oracle.OK
    return dict(j=q, attempt=0, target=t, n=T.n, k=P.n, mode=oracle.RIDS_SI_FC, labelled=True,
                status="ok" if ok else "aborted", matches=r["matches"] if ok else None,
                states=r["states"] if ok else None, candidates=r["candidates"], alg_bytes=r["alg_bytes"],
                sha256=oracle.rows_digest(r["rows"], P.n) if ok else None, oracle_s=round(dt, 3))


def one(args):
    cfg, j = args
    if cfg == "c3":
        return c3_shard(j)
    if cfg == "c5":
        return c5_query(j)
    cap = CAPS[cfg]
    for attempt in range(100):
        inst = MAKERS[cfg](j, attempt)
        t0 = time.perf_counter()
        r = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled, state_cap=cap, rows=True,
                       cap_rows=1 << 22)
        dt = time.perf_counter() - t0
        if r["status"] == oracle.OK:
            return dict(j=j, attempt=attempt, n=inst.target.n, k=inst.pattern.n, mode=inst.mode,
                        labelled=inst.labelled, matches=r["matches"], states=r["states"],
                        candidates=r["candidates"], alg_bytes=r["alg_bytes"],
                        sha256=oracle.rows_digest(r["rows"], inst.pattern.n), oracle_s=round(dt, 4))
    raise RuntimeError(f"{cfg}/{j}: no attempt under the cap")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    oracle.build()
    for cfg in a.configs:
        t0 = time.time()
        with mp.Pool(a.procs) as pool:
            rows = pool.map(one, [(cfg, j) for j in range(COUNTS[cfg])], chunksize=1 if cfg in ("c3", "c5") else 4)
        out = dict(config=cfg, state_cap=CAPS[cfg], instances=rows,
                   total_states=sum(r["states"] or 0 for r in rows),
                   total_matches=sum(r["matches"] or 0 for r in rows),
                   total_alg_bytes=sum(r["alg_bytes"] for r in rows))
        path = os.path.join(HERE, f"{cfg}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print(f"{cfg}: {len(rows)} instances, states {out['total_states']}, matches {out['total_matches']}, "
              f"redrawn {sum(r['attempt'] > 0 for r in rows)}, "
              f"aborted {sum(r.get('status') == 'aborted' for r in rows)}, {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
