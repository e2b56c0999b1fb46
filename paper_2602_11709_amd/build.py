"""Build libxrd.so (gfx950) in-tree with hipcc.

    python -m paper_2602_11709_amd.build

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (plain float code is still emitted as scalar or VOPD-free
vector ops).  The library lands next to this file, where the Python binding
looks for it.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxrd.so")
RATES = os.path.join(HERE, "xrd_rates")  # instruction-rate microbenchmark program
SOURCES = ["api.cpp", "scan.hip", "enumerate.hip", "sf.hip", "sortmerge.hip", "broaden.hip", "augment.hip", "family.hip",
           "noalloc.hip", "sfrec.hip", "lines.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object (in parallel), link libxrd.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr)
        elif verbose and text:
            print(text)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the instruction-rate microbenchmark (a standalone program)
    tmp = RATES + ".tmp"
    cmd = [hipcc(), *[f for f in flags() if f != "-fPIC"], "-x", "hip", os.path.join(CSRC, "rates.hip"), "-o", tmp]
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode != 0:
        print(out.stdout, file=sys.stderr)
        raise RuntimeError("hipcc failed for rates.hip")
    os.replace(tmp, RATES)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
