"""Write the oracle's results for every workload instance to tests/golden/*.json.

Only the oracle and the seeded input generators are called here.  Each
instance is screened against the workload's deterministic states cap: an
instance whose search exceeds the cap is redrawn with the next `attempt`
(the counterpart of the paper's per-instance time limit), and the attempt
used is recorded.

    python tests/golden/make_golden.py c1 c2 c4 c3 c5 c2d c3full [--procs 8]

The byte counts stored (`alg_bytes`, `dense_bytes`) are the oracle's, for a
count-only search: an enumeration also writes 4k bytes per match.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, REPO)

import oracle  # noqa: E402
from paper_1705_09358_amd import synth  # noqa: E402

CAPS = {"c1": 10 ** 8, "c2": 10 ** 8, "c4": 10 ** 8, "c3": 0, "c5": 10 ** 7, "c2d": 10 ** 8}
C5_SECONDS = 60.0   # the serving run: every query of 60 s of arrivals is checked against the oracle
C3_FULL = (0, 1, 2, 3)   # dense patterns searched in full by the benchmark
C3_SHARD = 10            # root ids per task of a full dense search
ROW_CAP = 1 << 22        # rows kept per instance for the digest
MAKERS = {"c1": synth.c1_instance, "c2": synth.c2_instance, "c4": synth.c4_instance, "c2d": synth.c2d_instance}
COUNTS = {"c1": synth.C1_COUNT, "c2": synth.C2_COUNT, "c4": synth.C4_COUNT, "c3": synth.C3_COUNT,
          "c5": len(synth.c5_arrivals(C5_SECONDS)), "c2d": synth.C2D_COUNT}


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
                candidates=r["candidates"], alg_bytes=r["alg_bytes"], dense_bytes=r["dense_bytes"],
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
    return dict(j=q, target=t, n=T.n, k=P.n, status="ok" if ok else "aborted",
                matches=r["matches"] if ok else None, states=r["states"] if ok else None,
                alg_bytes=r["alg_bytes"] if ok else None,
                sha256=oracle.rows_digest(r["rows"], P.n) if ok else None, oracle_s=round(dt, 3))


def c3_full_shard(args):
    """One task of a full dense search: pattern j with the first node of the
    order restricted to target ids [lo, hi); rows kept for the digest."""
    j, lo, hi = args
    inst = synth.c3_instance(j, 0)
    t0 = time.perf_counter()
    r = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled, rows=True, cap_rows=1 << 22,
                   root_range=(lo, hi))
    if r["matches"] > (1 << 22):
        raise RuntimeError(f"c3/{j} [{lo},{hi}): more rows than the buffer")
    return dict(j=j, lo=lo, hi=hi, matches=r["matches"], states=r["states"], candidates=r["candidates"],
                alg_bytes=r["alg_bytes"], dense_bytes=r["dense_bytes"], rows=r["rows"].tolist(),
                oracle_s=time.perf_counter() - t0)


def c3_full(procs, log_path):
    """Full dense searches of the benchmark's patterns, split by root-id range
    over a process pool (disjoint ranges partition a search exactly); shard
    results are appended to log_path so that an interrupted run resumes."""
    import numpy as np
    n = synth.c3_target().n
    tasks = [(j, lo, min(lo + C3_SHARD, n)) for j in C3_FULL for lo in range(0, n, C3_SHARD)]
    done = {}
    if os.path.exists(log_path):
        for line in open(log_path):
            r = json.loads(line)
            done[(r["j"], r["lo"], r["hi"])] = r
    todo = [t for t in tasks if t not in done]
    print(f"c3full: {len(tasks)} shards, {len(todo)} to run", flush=True)
    with mp.Pool(procs) as pool, open(log_path, "a") as logf:
        for i, r in enumerate(pool.imap_unordered(c3_full_shard, todo, chunksize=1)):
            logf.write(json.dumps(r) + "\n")
            logf.flush()
            done[(r["j"], r["lo"], r["hi"])] = r
            if i % 20 == 0:
                print(f"c3full: {i + 1}/{len(todo)} shards", flush=True)
    out = []
    for j in C3_FULL:
        parts = [done[t] for t in tasks if t[0] == j]
        inst = synth.c3_instance(j, 0)
        rows = np.array([x for p in parts for x in p["rows"]], dtype=np.uint32).reshape(-1, inst.pattern.n)
        out.append(dict(j=j, attempt=0, n=n, k=inst.pattern.n, mode=inst.mode, labelled=inst.labelled,
                        matches=sum(p["matches"] for p in parts), states=sum(p["states"] for p in parts),
                        candidates=sum(p["candidates"] for p in parts),
                        alg_bytes=sum(p["alg_bytes"] for p in parts),
                        # the bitset model charges a search's root expansion (one
                        # domain row of W words) once; every shard is a search
                        # of its own and charges it again
                        dense_bytes=sum(p["dense_bytes"] for p in parts) - (len(parts) - 1) * 8 * ((n + 63) // 64),
                        sha256=oracle.rows_digest(rows, inst.pattern.n), shards=len(parts),
                        oracle_s=round(sum(p["oracle_s"] for p in parts), 1)))
    return out


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
                       cap_rows=ROW_CAP)
        dt = time.perf_counter() - t0
        if r["status"] == oracle.OK:
            return dict(j=j, attempt=attempt, n=inst.target.n, k=inst.pattern.n, mode=inst.mode,
                        labelled=inst.labelled, matches=r["matches"], states=r["states"],
                        candidates=r["candidates"], alg_bytes=r["alg_bytes"], dense_bytes=r["dense_bytes"],
                        sha256=(oracle.rows_digest(r["rows"], inst.pattern.n) if r["matches"] <= ROW_CAP
                                else None),   # more matches than the row buffer: no digest
                        oracle_s=round(dt, 4))
    raise RuntimeError(f"{cfg}/{j}: no attempt under the cap")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--c3-log", default=os.path.join(tempfile.gettempdir(), "sge_c3full_shards.jsonl"),
                    help="where full dense shard results accumulate (resumable)")
    a = ap.parse_args()
    oracle.build()
    for cfg in a.configs:
        t0 = time.time()
        if cfg == "c3full":
            rows = c3_full(a.procs, a.c3_log)
        else:
            with mp.Pool(a.procs) as pool:
                rows = pool.map(one, [(cfg, j) for j in range(COUNTS[cfg])],
                                chunksize=1 if cfg == "c3" else 4)
        out = dict(config=cfg, state_cap=CAPS.get(cfg, 0), instances=rows,
                   total_states=sum(r["states"] or 0 for r in rows),
                   total_matches=sum(r["matches"] or 0 for r in rows),
                   total_alg_bytes=sum(r["alg_bytes"] or 0 for r in rows),
                   total_dense_bytes=sum(r.get("dense_bytes") or 0 for r in rows))
        if cfg == "c5":
            out["seconds"] = C5_SECONDS
        path = os.path.join(HERE, f"{cfg}.json")
        with open(path, "w") as f:
            if cfg == "c5":   # one query per line: ~12k of them
                f.write(json.dumps({k: v for k, v in out.items() if k != "instances"})[:-1] + ', "instances": [\n')
                f.write(",\n".join(json.dumps(r) for r in rows) + "\n]}\n")
            else:
                json.dump(out, f, indent=0)
        print(f"{cfg}: {len(rows)} instances, states {out['total_states']}, matches {out['total_matches']}, "
              f"redrawn {sum(r.get('attempt', 0) > 0 for r in rows)}, "
              f"aborted {sum(r.get('status') == 'aborted' for r in rows)}, {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
