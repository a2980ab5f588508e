"""Build libcrbm.so (all HIP sources of the package) for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcrbm.so")
SOURCES = ["crbm_abi.cpp", "init.hip", "sweep_generic.hip", "sweep_ising.hip", "ops.hip", "tempering.hip", "autocorr.hip",
           # the bit-packed Ising kernel, one unit per compiled (K, Lw) pair so that they build in parallel
           "sweep_ising_k8l5.hip", "sweep_ising_k8l3.hip", "sweep_ising_k4l3.hip", "sweep_ising_k2l2.hip",
           "sweep_ising_kxl1.hip", "sweep_ising_kxl2.hip", "sweep_ising_kxl3.hip", "sweep_ising_kxl4.hip",
           "sweep_ising_kxl5.hip", "sweep_ising_kxl6.hip"]
ARCH = os.environ.get("CRBM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in _build/ and link libcrbm.so in-tree."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out)
        raise RuntimeError(f"hipcc failed on {src}")
    if out.strip():
        sys.stderr.write(out)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
