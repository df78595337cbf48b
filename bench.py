"""Benchmark: RI / RI-DS subgraph enumeration on one MI355X.

Workload (one step): the batching configuration -- 4096 (pattern, target)
pairs, each with its own protein-contact-like target (100-5000 nodes,
log-uniform) and a random-walk pattern of 8-64 nodes (log-uniform), mode RI
or RI-DS-SI-FC by a fair coin, labelled -- in one HIP-graph launch that
uploads the job descriptors, plans every instance on the device and runs the
persistent search of all of them.  Inputs are seeded and synthetic (the
paper's PDBSv1 / PPIS32 / GRAEMLIN32 collections are not available).  Every
step's state and match counts, and every instance's algorithmic bytes, are
checked against the oracle's stored values.

Also reported: the plain single-instance path (one sge_count per instance,
every result checked) on the same 4096 instances and `vs_plain`; the search
kernel's algorithmic bytes over its HIP-event time against the HBM peak; the
contact-3000 workload (with the four-mode variant study), C1, the dense C3
searches (checked against the oracle's full-size values) and the directed
edge-labelled workload, each batched and plain; the serving run (60 s of
Poisson arrivals, every result checked; p50/p99 latency) with host plans
and a shorter one with device plans; and three CPU baselines on this host
(baselines, not the target): the oracle single-threaded on one pinned core,
the paper's parallel scheduler on up to 16 threads, and a pool of up to 16
single-threaded oracle processes over one pass of the batching workload.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--extra c2,c1,c3,c2d]
                    [--serve-seconds 60] [--serve-device-seconds 20] [--no-variants]
                    [--no-plain] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

HBM_PEAK_GBS = 8000.0
METRIC = "search states/s + matches/s vs plain GPU search (exact); p99 query latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def load_manifest(cfg):
    with open(os.path.join(REPO, "tests", "golden", f"{cfg}.json")) as f:
        return json.load(f)


def instances(cfg, man):
    from paper_1705_09358_amd import synth
    make = {"c1": synth.c1_instance, "c2": synth.c2_instance, "c4": synth.c4_instance,
            "c2d": synth.c2d_instance}[cfg]
    return [make(r["j"], r["attempt"]) for r in man["instances"]]


def bytes_model(res_bytes, man):
    """Which byte model the launch counted (the CSR search counts the oracle's
    sparse model, the dense-bitset search its dense model) and the total; every
    instance must match the stored oracle value of that model."""
    got = [int(x) for x in res_bytes]
    for key, name in (("alg_bytes", "csr"), ("dense_bytes", "dense")):
        want = [r.get(key) for r in man["instances"]]
        if got == want:
            return name, sum(want)
    raise SystemExit("algorithmic bytes differ from the oracle's stored values")


def run_batch_workload(ctx, torch, insts, man, steps, warmup, label):
    """Load all targets and patterns, then time `steps` batched launches
    (every one checked against the oracle's stored counts and bytes)."""
    from paper_1705_09358_amd import sge
    tgt = {}
    jobs = []
    for inst in insts:
        key = id(inst.target)
        if key not in tgt:
            tgt[key] = ctx.load_target(inst.target)
        jobs.append((tgt[key], ctx.load_pattern(inst.pattern), inst.mode, inst.labelled))
    want_states = np.array([r["states"] for r in man["instances"]], dtype=np.uint64)
    want_matches = np.array([r["matches"] for r in man["instances"]], dtype=np.uint64)
    job_arr = sge.job_array(jobs)
    log(f"{label}: {len(jobs)} jobs loaded; warmup {warmup}")
    for _ in range(max(1, warmup)):
        st, res = ctx.batch_run(job_arr)
    model, alg_bytes = bytes_model(res.alg_bytes, man)
    torch.cuda.synchronize()
    ev_ms, dev_ms = [], []
    log(f"{label}: timing {steps} steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        st, res = ctx.batch_run(job_arr)
        ev_ms.append(ctx.last_kernel_ms())
        dev_ms.append(float(res.ms_search[0]))
        if not (np.array_equal(res.states, want_states) and np.array_equal(res.matches, want_matches)):
            raise SystemExit(f"{label}: counts differ from the oracle's stored values")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the last launch's search units and the share of their time spent holding
    # tasks (the shape the autotuner picked shows in the unit count)
    busy_ms, units = ctx.last_launch_occupancy()
    launch = dict(units=int(units),
                  busy_fraction=busy_ms / (units * ev_ms[-1]) if units and ev_ms[-1] > 0 else None)
    if int(res.alg_bytes.sum()) != alg_bytes:
        raise SystemExit(f"{label}: algorithmic bytes changed between launches")
    tot_states = int(want_states.sum()) * steps
    tot_matches = int(want_matches.sum()) * steps
    kernel_ms = sum(ev_ms) / len(ev_ms)
    if kernel_ms <= 0:
        raise SystemExit(f"{label}: the search kernel's events recorded nothing ({ctx.last_error()})")
    return dict(ms_per_step=1000 * el / steps, states_per_s=tot_states / el, matches_per_s=tot_matches / el,
                kernel_ms=kernel_ms, kernel_ms_device_clock=sum(dev_ms) / len(dev_ms),
                prep_ms=float(res.ms_prep[0]), launch=launch, jobs=jobs, tgt=tgt, model=model, alg_bytes=alg_bytes,
                roofline=dict(roofline(alg_bytes, kernel_ms), alg_bytes_per_state=alg_bytes / int(want_states.sum())),
                instances=len(jobs),
                states_per_step=int(want_states.sum()), matches_per_step=int(want_matches.sum()))


def roofline(alg_bytes, kernel_ms):
    """Algorithmic bytes of one launch over the search kernel's HIP-event time,
    against the HBM peak."""
    achieved = alg_bytes / (kernel_ms / 1000.0) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes, "kernel_ms": kernel_ms}


def run_plain(ctx, torch, jobs, man, reps=1):
    """One sge_count per instance, sequentially (the plain single-instance
    path), every result checked against the oracle's stored values."""
    want = man["instances"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = 0.0
    for _ in range(reps):
        for (t, p, mode, lab), w in zip(jobs, want):
            ctx.set_mode(mode)
            ctx.set_labelled(lab)
            r = ctx.count(t, p)
            kms += ctx.last_kernel_ms()
            if (r.states, r.matches) != (w["states"], w["matches"]):
                raise SystemExit("plain path: counts differ from the oracle's stored values")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    states = sum(w["states"] for w in want) * reps
    matches = sum(w["matches"] for w in want) * reps
    return dict(states_per_s=states / el, matches_per_s=matches / el, ms_per_pass=1000 * el / reps,
                kernel_ms_per_pass=kms / reps, searches=len(jobs) * reps)


MODE_NAMES = {0: "RI", 1: "RI-DS", 2: "RI-DS-SI", 3: "RI-DS-SI-FC"}


def run_variants(ctx, torch, jobs, steps):
    """The variant study on the contact-3000 workload: the same 100 patterns
    batched in each search mode (RI, RI-DS, RI-DS-SI, RI-DS-SI-FC).  The match
    set must not change with the mode; states and time show what the domains,
    the SI tie-break and forward checking save."""
    from paper_1705_09358_amd import sge
    out = {}
    ref_matches = None
    for mode in range(4):
        arr = sge.job_array([(t, p, mode, lab) for t, p, _, lab in jobs])
        st, res = ctx.batch_run(arr)   # first call of this batch size: autotune
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = []
        for _ in range(steps):
            st, res = ctx.batch_run(arr)
            kms.append(ctx.last_kernel_ms())
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        if ref_matches is None:
            ref_matches = res.matches.copy()
        elif not np.array_equal(res.matches, ref_matches):
            raise SystemExit(f"variants: matches of mode {MODE_NAMES[mode]} differ from RI")
        states = int(res.states.sum())
        out[MODE_NAMES[mode]] = dict(states_per_step=states, matches_per_step=int(res.matches.sum()),
                                     ms_per_step=1000 * el, kernel_ms=sum(kms) / len(kms),
                                     states_per_s=states / el, alg_bytes_per_step=int(res.alg_bytes.sum()))
    return out


# The dense workload's benchmark patterns (their full oracle values are stored)
C3_BENCH = 4
VALU_PEAK_GOPS = 256 * 64 * 2.4   # 256 CUs x 64 int32 lanes per clock (4 SIMD x 16) x 2.4 GHz


def run_dense(ctx, torch, steps):
    """Dense workload: the first four RI-DS-SI-FC patterns on G(1000, 0.3),
    full searches, batched (one launch) and plain (one sge_enumerate each),
    checked against the oracle's full-size values: matches, states, bytes and
    (plain path) the digest of the sorted rows."""
    import oracle
    from paper_1705_09358_amd import synth
    man = load_manifest("c3full")
    want = man["instances"][:C3_BENCH]
    T = synth.c3_target()
    th = ctx.load_target(T)
    insts = [synth.c3_instance(w["j"], 0) for w in want]
    jobs = [(th, ctx.load_pattern(i.pattern), i.mode, i.labelled) for i in insts]
    ctx.set_batch_policy(2)
    log(f"c3: {len(jobs)} dense patterns, warmup")
    st, res = ctx.batch_run(jobs)
    ref = [(int(r.matches), int(r.states), int(r.alg_bytes)) for r in res]
    if ref != [(w["matches"], w["states"], w["dense_bytes"]) for w in want]:
        raise SystemExit("c3: counts or bytes differ from the oracle's full-size values")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = []
    for _ in range(steps):
        st, res = ctx.batch_run(jobs)
        kms.append(ctx.last_kernel_ms())
        if [(int(r.matches), int(r.states), int(r.alg_bytes)) for r in res] != ref:
            raise SystemExit("c3: counts changed between runs")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    states = sum(s for _, s, _ in ref)
    alg = sum(b for _, _, b in ref)
    log("c3: plain path (sge_enumerate, rows checked)")
    ctx.set_mode(synth.MODE_RIDS_SI_FC)
    ctx.set_labelled(True)
    tp = time.perf_counter()
    for (t, p, _, _), inst, w in zip(jobs, insts, want):
        r, rows = ctx.enumerate(t, p, inst.pattern.n, cap_rows=max(1, w["matches"]))
        if (r.matches, r.states) != (w["matches"], w["states"]) or \
                oracle.rows_digest(rows, inst.pattern.n) != w["sha256"]:
            raise SystemExit("c3: the plain path differs from the oracle's full-size values")
    plain_el = time.perf_counter() - tp
    ctx.set_batch_policy(0)
    kernel_ms = sum(kms) / len(kms)
    # the integer-ALU ceiling: per expansion and candidate word, one 64-bit
    # AND per row read beyond the first, one AND-NOT with the used set and
    # one popcount, two 32-bit lane operations each; expansions per instance
    # = its states below the last position + 1 (the root)
    W = 16
    rows_read = alg // (8 * W)
    expansions = sum(s - m + 1 for m, s, _ in ref)
    valu_ops = 2 * W * (rows_read + expansions)
    return dict(instances=len(jobs), states_per_step=states, matches_per_step=sum(m for m, _, _ in ref),
                states_per_s=states * steps / el, ms_per_step=1000 * el / steps, kernel_ms=kernel_ms,
                plain_states_per_s=states / plain_el, vs_plain=(states * steps / el) / (states / plain_el),
                checked="matches, states, bytes and the sorted-row digest equal the oracle's full searches",
                roofline=roofline(alg, kernel_ms), model="dense",
                valu={"bound": "alu", "ops_per_launch_lower_bound": valu_ops,
                      "achieved_Gops": valu_ops / (kernel_ms / 1000.0) / 1e9, "peak_Gops": VALU_PEAK_GOPS,
                      "frac": valu_ops / (kernel_ms / 1000.0) / 1e9 / VALU_PEAK_GOPS})


def run_serve(torch, seconds, rate, plan_where=-1, plain=False):
    """Serving workload: resident contact targets (5k-20k nodes), queries of
    4-64 nodes arriving as a Poisson process; latency = result visible on the
    host - scheduled arrival.  Every result is checked against the oracle's
    stored value for its query (status, matches, states, bytes).  With
    `plain`, the same queries are then searched one at a time (sge_count, all
    CUs on each, host plans), every result checked again: the plain path on
    the same instance set, with its per-query time."""
    from paper_1705_09358_amd import sge, synth
    man = load_manifest("c5")
    log("serve: generating 50 resident targets")
    targets = [synth.c5_target(t) for t in range(synth.C5_TARGETS)]
    arrivals = synth.c5_arrivals(seconds, rate)
    if len(arrivals) > len(man["instances"]):
        raise SystemExit(f"serve: {len(arrivals)} arrivals but oracle values for {len(man['instances'])}")
    log(f"serve: generating {len(arrivals)} queries")
    queries = [synth.c5_query(q, targets) for q in range(len(arrivals))]
    ctx = sge.Context(0)
    ctx.set_time_limit(30000)
    ctx.set_state_cap(man["state_cap"])
    ctx.set_plan_location(plan_where)
    th = [ctx.load_target(T) for T in targets]
    ph = [ctx.load_pattern(P) for _, P, _ in queries]
    ctx.serve_start(256, 2 << 30)
    lat = np.zeros(len(arrivals))
    res = [None] * len(arrivals)
    tickets = {}
    busy = 0
    max_conc = 0
    log(f"serve: {seconds:.0f} s of arrivals at {rate:.0f}/s, plan location {plan_where}")
    t0 = time.perf_counter()
    nxt = 0
    last_print = t0
    while nxt < len(arrivals) or tickets:
        now = time.perf_counter() - t0
        while nxt < len(arrivals) and arrivals[nxt] <= now:
            t, _, _ = queries[nxt]
            tk = ctx.serve_submit(th[t], ph[nxt], sge.RIDS_SI_FC, True)
            if tk is None:
                busy += 1
                break                      # not admissible now: retried on the next pass
            tickets[tk] = nxt
            nxt += 1
        max_conc = max(max_conc, len(tickets))
        for tk in list(tickets):
            r = ctx.serve_poll(tk)
            if r is not None:
                q = tickets.pop(tk)
                lat[q] = (time.perf_counter() - t0) - arrivals[q]
                res[q] = r
        if time.perf_counter() - last_print > 5:
            last_print = time.perf_counter()
            log(f"serve: {nxt}/{len(arrivals)} submitted, {len(tickets)} in flight")
        time.sleep(0.0002)
    el = time.perf_counter() - t0
    ctx.serve_stop()

    def check(q, r, w, what):
        if w["j"] != q:
            raise SystemExit("serve: the stored oracle values are not in arrival order")
        if w["status"] == "ok":
            if r.status != sge.OK or (r.matches, r.states, r.alg_bytes) != (w["matches"], w["states"],
                                                                           w["alg_bytes"]):
                raise SystemExit(f"{what}: query {q} differs from the oracle's stored value")
        elif r.status != sge.E_ABORTED:
            raise SystemExit(f"{what}: query {q} should have been stopped at the state cap")

    for q, (r, w) in enumerate(zip(res, man["instances"])):
        check(q, r, w, "serve")
    plain_leg = None
    if plain:
        log(f"serve: the same {len(arrivals)} queries one at a time (plain path)")
        ctx.set_mode(sge.RIDS_SI_FC)
        ctx.set_labelled(True)
        per = np.zeros(len(arrivals))
        pst = 0
        tp = time.perf_counter()
        for q in range(len(arrivals)):
            a0 = time.perf_counter()
            r = ctx.count(th[queries[q][0]], ph[q], allow=(sge.OK, sge.E_ABORTED))
            per[q] = time.perf_counter() - a0
            check(q, r, man["instances"][q], "serve, plain path")
            if r.status == sge.OK:
                pst += r.states
        pel = time.perf_counter() - tp
        pms = per * 1000
        plain_leg = dict(queries=len(arrivals), checked=len(arrivals), seconds=pel, states_per_s=pst / pel,
                         p50_ms=float(np.percentile(pms, 50)), p99_ms=float(np.percentile(pms, 99)),
                         note="per-query time of sge_count back to back (no arrivals, no queueing)")
    ctx.close()
    ok = [r for r in res if r.status == sge.OK]
    states = sum(r.states for r in ok)
    ms = lat * 1000
    return dict(seconds=seconds, rate_qps=rate, queries=len(arrivals), checked=len(arrivals),
                plan_location="host" if plan_where <= 0 else "device",
                completed_qps=len(arrivals) / el, p50_ms=float(np.percentile(ms, 50)),
                p99_ms=float(np.percentile(ms, 99)), max_ms=float(ms.max()),
                mean_prep_ms=float(np.mean([r.ms_prep for r in res])),
                states_per_s=states / el, matches_per_s=sum(r.matches for r in ok) / el,
                alg_bytes_per_s=sum(r.alg_bytes for r in ok) / el,
                aborted=sum(r.status == sge.E_ABORTED for r in res), busy_retries=busy, max_in_flight=max_conc,
                plain=plain_leg)


def kernel_source_hash():
    import hashlib
    src = os.path.join(REPO, "paper_1705_09358_amd", "csrc", "sge_search.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of the search kernel on a workload, from the
    committed counter summary -- only while the kernel source is the one that
    was measured (else None)."""
    import re
    path = os.path.join(REPO, "profiles", f"search_kernel_hbm_traffic_{workload}.md")
    try:
        m = re.search(r"traffic_bytes_per_launch=([0-9.eE+]+) kernel_source_sha256=([0-9a-f]+)", open(path).read())
    except OSError:
        return None
    return float(m.group(1)) if m and m.group(2) == kernel_source_hash() else None


def host_cpu():
    """The host's processor model, its current clock as the kernel reports it
    (first core, MHz) and the cores this process may use."""
    model = mhz = None
    try:
        for line in open("/proc/cpuinfo"):
            if model is None and line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
            elif mhz is None and line.startswith("cpu MHz"):
                mhz = float(line.split(":", 1)[1])
            if model is not None and mhz is not None:
                break
    except (OSError, ValueError):
        pass
    return dict(cpu_model=model, cpu_mhz=mhz, host_cores=len(os.sched_getaffinity(0)))


def measured_l2(workload, kernel_ms):
    """L2 hit rate and request rate of the search kernel on a workload, from
    the committed counter summary, only while the kernel source is the one
    that was measured (else None)."""
    import re
    path = os.path.join(REPO, "profiles", f"search_kernel_l2_{workload}.md")
    try:
        m = re.search(r"l2_hit_rate=([0-9.]+) l2_requests_per_launch=([0-9.eE+]+) kernel_source_sha256=([0-9a-f]+)",
                      open(path).read())
    except OSError:
        return None
    if not m or m.group(3) != kernel_source_hash():
        return None
    req = float(m.group(2))
    return dict(hit_rate=float(m.group(1)), requests_per_launch=req,
                requests_per_s=req / (kernel_ms / 1000.0), source=os.path.relpath(path, REPO))


def cpu_baseline(insts, variant_insts, budget_s=12.0, variant_sample=34):
    """The oracle, single-threaded, with the calling thread pinned to one core
    (restored afterwards, before the multi-threaded legs)."""
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})
    try:
        r = _cpu_baseline(insts, variant_insts, budget_s, variant_sample)
    finally:
        os.sched_setaffinity(0, allowed)
    r["pinned_core"] = core
    return r


def _cpu_baseline(insts, variant_insts, budget_s, variant_sample):
    import oracle
    oracle.lib()
    # the variant study's oracle leg: every third contact-3000 pattern in each mode
    variants = {}
    sample = variant_insts[::3][:variant_sample]
    for mode in range(4):
        t0 = time.process_time()
        st = 0
        for inst in sample:
            st += oracle.run(inst.pattern, inst.target, mode, inst.labelled)["states"]
        el = time.process_time() - t0
        variants[MODE_NAMES[mode]] = dict(states=st, seconds=el, states_per_s=st / el if el > 0 else None)
    t0 = time.process_time()
    states = matches = 0
    n = 0
    passes = 0
    while time.process_time() - t0 < budget_s:
        for inst in insts:
            r = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled)
            states += r["states"]
            matches += r["matches"]
            n += 1
            if time.process_time() - t0 >= budget_s and passes >= 1:
                break
        passes += 1
    el = time.process_time() - t0
    return dict(value=states / el, unit="states/s", cores=1, kind="oracle",
                matches_per_s=matches / el,
                sample=f"{n} searches of the batching workload's instances in their order ({passes} pass(es) "
                       f"started), single thread, {el:.1f} s CPU",
                variants=dict(sample=f"{len(sample)} of the 100 contact-3000 patterns (every third), each mode",
                              **variants))


def _pool_init(root):
    sys.path.insert(0, root)
    import oracle
    oracle.lib()


def _pool_run(inst):
    import oracle
    r = oracle.run(inst.pattern, inst.target, inst.mode, inst.labelled)
    return r["states"], r["matches"]


def cpu_pool(insts, procs=16):
    """A pool of single-threaded oracle processes, one instance per task, over
    one pass of a many-instance workload (wall time from the first task to the
    last result; the pool is started and warm before the clock starts)."""
    import multiprocessing as mp
    procs = max(1, min(procs, len(os.sched_getaffinity(0))))
    with mp.get_context("spawn").Pool(procs, initializer=_pool_init, initargs=(REPO,)) as pool:
        pool.map(_pool_run, insts[:procs], chunksize=1)   # warm: every worker has loaded the oracle
        t0 = time.perf_counter()
        res = pool.map(_pool_run, insts, chunksize=1)
        el = time.perf_counter() - t0
    states = sum(r[0] for r in res)
    matches = sum(r[1] for r in res)
    return dict(value=states / el, unit="states/s", cores=procs, kind="oracle pool",
                matches_per_s=matches / el, states=states, seconds=el,
                sample=f"one pass over the {len(insts)} instances, one instance per task, {procs} single-threaded "
                       f"oracle processes, wall time")


def cpu_parallel(insts, budget_s=6.0, group=4):
    """The paper's own parallel CPU search (private deques, stealing, task
    groups, token ring) on the host cores, over the same workload."""
    from paper_1705_09358_amd import cpu_baseline as cb
    threads = max(1, min(16, os.cpu_count() or 1))
    states = matches = 0
    search_s = 0.0
    passes = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s or passes == 0:
        for inst in insts:
            r = cb.count(inst.pattern, inst.target, inst.mode, inst.labelled, threads, group)
            states += r["states"]
            matches += r["matches"]
            search_s += r["seconds"]
        passes += 1
    return dict(value=states / search_s, unit="states/s", threads=threads, kind="paper scheduler (Section 3)",
                matches_per_s=matches / search_s, task_group=group,
                sample=f"{passes} pass(es) over the {len(insts)} patterns, search time only (host plans excluded)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--extra", default="c2,c1,c3,c2d",
                    help="comma list of extra workloads: c2 (contact-3000, with the variant study), c1, c3 "
                         "(dense), c2d (directed, edge labels); '' for none")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy a buffer of this many MiB (calibrates the HBM byte counters; prints the copy rate)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-device-seconds", type=float, default=20.0,
                    help="a second serving run with every query planned by the plan kernel")
    ap.add_argument("--no-variants", action="store_true", help="skip the four-mode variant study")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of "
                                   "this build (the search shards by root candidates, see the design notes)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_1705_09358_amd import sge
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if a.copy_probe:
        # a plain device copy: calibrates the HBM byte counters (five copies)
        # and measures the streaming rate (read + write bytes / copy time,
        # median of 20 timed copies after the five)
        n = a.copy_probe << 18        # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        ms = []
        for _ in range(20):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        ms.sort()
        med = ms[len(ms) // 2]
        print(json.dumps({"copy_probe_MiB": a.copy_probe, "copies": 25, "ms_per_copy": med,
                          "GBps_read_plus_write": 2 * n * 4 / (med / 1000.0) / 1e9}))
        return
    stream = torch.cuda.Stream()
    man = load_manifest("c4")
    log("generating the batching workload (4096 pairs)")
    insts = instances("c4", man)
    extras = {}
    variants = None
    c2_insts = None
    with torch.cuda.stream(stream):
        ctx = sge.Context(0, stream=stream)
        b = run_batch_workload(ctx, torch, insts, man, a.steps, a.warmup, "c4")
        plain = None
        if not a.no_plain:
            log("c4: plain single-instance path (4096 searches)")
            plain = run_plain(ctx, torch, b["jobs"], man)
        ctx.close()
        for cfg in [x for x in a.extra.split(",") if x]:
            if cfg == "c3":
                ctx3 = sge.Context(0, stream=stream)
                extras["c3"] = run_dense(ctx3, torch, max(1, a.steps // 10))
                ctx3.close()
                continue
            m2 = load_manifest(cfg)
            log(f"generating the {cfg} workload")
            i2 = instances(cfg, m2)
            ctx2 = sge.Context(0, stream=stream)
            e = run_batch_workload(ctx2, torch, i2, m2, max(5, a.steps // 4), 2, cfg)
            extras[cfg] = {k: e[k] for k in ("states_per_s", "matches_per_s", "ms_per_step", "kernel_ms",
                                             "kernel_ms_device_clock", "instances", "states_per_step",
                                             "matches_per_step", "model", "roofline")}
            if not a.no_plain:
                p2 = run_plain(ctx2, torch, e["jobs"], m2, reps=2 if cfg == "c2" else 1)
                extras[cfg]["plain_states_per_s"] = p2["states_per_s"]
                extras[cfg]["vs_plain"] = e["states_per_s"] / p2["states_per_s"]
            if cfg == "c2":
                c2_insts = i2
                tr = measured_traffic("contact3000")
                extras[cfg]["roofline"]["traffic"] = tr
                extras[cfg]["l2"] = measured_l2("contact3000", e["kernel_ms"])
                if not a.no_variants:
                    log("c2: variant study (four modes)")
                    variants = run_variants(ctx2, torch, e["jobs"], max(3, a.steps // 4))
            ctx2.close()
    serve = run_serve(torch, a.serve_seconds, 200.0, -1, plain=not a.no_plain) if a.serve_seconds > 0 else None
    serve_dev = run_serve(torch, a.serve_device_seconds, 200.0, 1) if a.serve_device_seconds > 0 else None
    rl = dict(b["roofline"])
    rl["traffic"] = measured_traffic("c4")
    res = {
        "metric": METRIC,
        "value": b["states_per_s"],
        "unit": "states/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generators standing in for the paper's biochemical collections)",
        "config": {"workload": "batching: 4096 (pattern, target) pairs, contact-like targets of 100-5000 nodes "
                               "(log-uniform), random-walk patterns of 8-64 nodes (log-uniform), RI or "
                               "RI-DS-SI-FC by a fair coin, labelled; one persistent search launch in a HIP graph",
                   "instances": b["instances"], "states_per_step": b["states_per_step"],
                   "matches_per_step": b["matches_per_step"]},
        "matches_per_s": b["matches_per_s"],
        "kernel_ms_per_step": b["kernel_ms"],
        "kernel_ms_device_clock": b["kernel_ms_device_clock"],
        "search_launch": b["launch"],
        "prep_ms_per_step": b["prep_ms"],
        "plain": plain,
        "vs_plain": None if plain is None else b["states_per_s"] / plain["states_per_s"],
        "roofline": rl,
        "l2": measured_l2("c4", b["kernel_ms"]),
        "p99_ms": None if serve is None else serve["p99_ms"],
        "serve": serve,
        "serve_device_plan": serve_dev,
        "variants": variants,
        "extra": extras,
    }
    if not a.no_cpu:
        log("cpu baseline (oracle)")
        if c2_insts is None:
            c2_insts = instances("c2", load_manifest("c2"))
        res["cpu_baseline"] = cpu_baseline(insts, c2_insts)
        res["cpu_baseline"].update(host_cpu())
        log("cpu baseline (the paper's parallel scheduler)")
        res["cpu_parallel"] = cpu_parallel(c2_insts)
        log("cpu baseline: oracle process pool over the batching workload")
        res["cpu_pool_c4"] = cpu_pool(insts)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
