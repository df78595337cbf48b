"""The benchmark's host-side contract, on the CPU: the one-GPU guard, the
readers of the committed counter summaries, the host description and the
oracle process pool (which must reproduce the oracle's stored counts)."""
import json
import os
import subprocess
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, REPO)

import bench  # noqa: E402
from paper_1705_09358_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    # the guard runs before anything touches a GPU
    r = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_counter_summaries_are_read_or_withheld():
    # figures from the committed summaries are used only while the kernel
    # source hash matches; either way the result is well formed
    for w in ("c4", "contact3000"):
        t = bench.measured_traffic(w)
        assert t is None or t > 0
    assert bench.measured_traffic("no-such-workload") is None
    l2 = bench.measured_l2("c4", 2.0)
    if l2 is not None:
        assert 0.0 < l2["hit_rate"] <= 1.0
        assert l2["requests_per_launch"] > 0
        assert l2["requests_per_s"] == pytest.approx(l2["requests_per_launch"] / 2e-3)


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["host_cores"] >= 1
    assert h["cpu_model"] is None or isinstance(h["cpu_model"], str)
    assert h["cpu_mhz"] is None or h["cpu_mhz"] > 0


def test_oracle_pool_reproduces_stored_counts():
    man = json.load(open(os.path.join(REPO, "tests", "golden", "c1.json")))
    rows = man["instances"][:6]
    insts = [synth.c1_instance(r["j"], r["attempt"]) for r in rows]
    r = bench.cpu_pool(insts, procs=2)
    assert r["states"] == sum(x["states"] for x in rows)
    assert r["cores"] == min(2, len(os.sched_getaffinity(0)))
    assert r["kind"] == "oracle pool" and r["value"] > 0


def test_pinned_oracle_leg_restores_affinity():
    before = os.sched_getaffinity(0)
    man = json.load(open(os.path.join(REPO, "tests", "golden", "c1.json")))
    insts = [synth.c1_instance(r["j"], r["attempt"]) for r in man["instances"][:3]]
    r = bench.cpu_baseline(insts, insts, budget_s=0.2, variant_sample=1)
    assert os.sched_getaffinity(0) == before
    assert r["pinned_core"] in before and r["cores"] == 1 and r["value"] > 0


def test_roofline_object():
    r = bench.roofline(8_000_000_000, 1000.0)   # 8 GB in one second
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(8.0) and r["frac"] == pytest.approx(1e-3)


def test_bytes_model_picks_the_kernel_variant():
    man = {"instances": [{"alg_bytes": 10, "dense_bytes": 40}, {"alg_bytes": 7, "dense_bytes": 16}]}
    assert bench.bytes_model([10, 7], man) == ("csr", 17)
    assert bench.bytes_model([40, 16], man) == ("dense", 56)
    with pytest.raises(SystemExit):
        bench.bytes_model([10, 16], man)
