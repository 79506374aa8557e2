"""Build libising.so (the C-ABI library) in-tree with hipcc for gfx950.

    python -m paper_1110_2561_amd.build

It also builds microbench/lds_atomic, the microbenchmark of the LDS-atomic
and integer-VALU rates the benchmark's roofline is reported against.

The library is plain hipcc output: HIP kernels for gfx950 plus host C++,
linked against the HIP runtime only.  Every HIP source is compiled with
packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libising.so")
SOURCES = ["plan.cpp", "bond_plan.cpp", "enumerate.hip", "thermo.hip", "batch.hip", "bond.hip"]
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(out_dir, src + ".o")
        flags = HIP_FLAGS + ["-x", "hip"] if src.endswith(".hip") else CXX_FLAGS
        cmd = [hipcc, *flags, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        noise = [ln for ln in (r.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n" + "\n".join(noise))
        if verbose and noise:
            print("\n".join(noise))
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    # the LDS-atomic / integer-VALU microbenchmark behind the roofline peaks
    mb_src = os.path.join(HERE, "microbench", "lds_atomic.hip")
    mb_exe = os.path.join(HERE, "microbench", "lds_atomic")
    cmd = [hipcc, *HIP_FLAGS, "-x", "hip", mb_src, "-o", mb_exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"microbenchmark build failed: {' '.join(cmd)}\n{r.stderr}")
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
