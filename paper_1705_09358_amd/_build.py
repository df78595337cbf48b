"""In-tree build of the native parts: the HIP library (gfx950) and the C input generator."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
INCLUDE = os.path.join(REPO, "include")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SGE_SO = os.path.join(LIBDIR, "libsge.so")
SYNTH_SO = os.path.join(LIBDIR, "libsynth_walk.so")

# Host sources (plain C++) and device sources (HIP) of the search library.
HOST_SRCS = ["sge_graph.cpp", "sge_plan.cpp", "sge_api.cpp", "sge_launch.cpp", "sge_batch.cpp", "sge_serve.cpp"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__"]
HIP_SRCS = ["sge_search.hip", "sge_plan_dev.hip", "sge_noalloc.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions are kept out of every device object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def _atomic_link(cmd_out: list[str], out: str) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    _run(cmd_out + ["-o", tmp])
    os.replace(tmp, out)


def build_synth() -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    src = os.path.join(CSRC, "synth_walk.c")
    _atomic_link(["gcc", "-O2", "-shared", "-fPIC", src, "-lm"], SYNTH_SO)
    return SYNTH_SO


def build_sge() -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    inc = ["-I", INCLUDE, "-I", CSRC, "-I", os.path.join(ROCM, "include")]
    procs = []
    for s in HOST_SRCS + HIP_SRCS:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, s + ".o")
        if s.endswith(".cpp"):
            cmd = ["g++", *HOST_FLAGS, *inc, "-c", src, "-o", obj]
        else:
            cmd = [os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, *inc, "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for cmd, p in procs:
        outp, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + outp)
    _atomic_link([os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
                  "-lpthread", "-Wl,-rpath," + os.path.join(ROCM, "lib")], SGE_SO)
    return SGE_SO


CPU_WS_SO = os.path.join(LIBDIR, "libsge_cpuws.so")


def build_cpu_baseline() -> str:
    """The paper's parallel CPU search (a measurement baseline, host code only)."""
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = [os.path.join(HERE, "cpu", "sge_cpu_ws.cpp"), os.path.join(CSRC, "sge_plan.cpp"),
            os.path.join(CSRC, "sge_graph.cpp")]
    inc = ["-I", INCLUDE, "-I", CSRC, "-I", os.path.join(ROCM, "include")]
    _atomic_link(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-D__HIP_PLATFORM_AMD__", *inc, *srcs,
                  "-lpthread"], CPU_WS_SO)
    return CPU_WS_SO


def build_all() -> None:
    build_synth()
    build_sge()
    build_cpu_baseline()
