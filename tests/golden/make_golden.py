"""Write the oracle's results for every workload instance to tests/golden/*.json.

Only the oracle and the seeded input generators are called here.  Each
instance is screened against the workload's deterministic states cap: an
instance whose search exceeds the cap is redrawn with the next `attempt`
(the counterpart of the paper's per-instance time limit), and the attempt
used is recorded.

    python tests/golden/make_golden.py c1 c2 c4 [--procs 8]
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

CAPS = {"c1": 10 ** 8, "c2": 10 ** 8, "c4": 10 ** 8}
MAKERS = {"c1": synth.c1_instance, "c2": synth.c2_instance, "c4": synth.c4_instance}
COUNTS = {"c1": synth.C1_COUNT, "c2": synth.C2_COUNT, "c4": synth.C4_COUNT}


def one(args):
    cfg, j = args
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
            rows = pool.map(one, [(cfg, j) for j in range(COUNTS[cfg])], chunksize=4)
        out = dict(config=cfg, state_cap=CAPS[cfg], instances=rows,
                   total_states=sum(r["states"] for r in rows), total_matches=sum(r["matches"] for r in rows),
                   total_alg_bytes=sum(r["alg_bytes"] for r in rows))
        path = os.path.join(HERE, f"{cfg}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print(f"{cfg}: {len(rows)} instances, states {out['total_states']}, matches {out['total_matches']}, "
              f"redrawn {sum(r['attempt'] > 0 for r in rows)}, {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
