"""Build libnsmi.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2509_04336_amd.build [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnsmi.so")

SOURCES = ["nsmi_kernels.hip", "nsmi_walk.hip", "nsmi_hrss.hip", "nsmi_mlp.hip", "nsmi_host.cpp"]
HEADERS = ["nsmi_device.h", "nsmi_kernels.h", "nsmi_mlp.h", "nsmi_hrss.h"]

# Packed FP32 instructions stay off (they are formed by the compiler from
# scalar code otherwise); contraction is off so the explicit fma() calls are
# the only fused operations, as in the per-step parity definition.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-x", "hip", *srcs,
           "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libnsmi.so")
    if verbose and r.stderr.strip():
        sys.stderr.write("\n".join(l for l in r.stderr.splitlines()
                                   if "packed-fp32-ops" not in l) + "\n")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    deps.append(os.path.join(ROOT, "include", "nsmi.h"))
    return any(os.path.getmtime(p) > t for p in deps)


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
