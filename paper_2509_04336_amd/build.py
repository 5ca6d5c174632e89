"""Build libnsmi.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2509_04336_amd.build [--verbose]

Each source is compiled to its own object (in parallel), then linked.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnsmi.so")
OBJ = os.path.join(ROOT, "_build")

SOURCES = ["nsmi_kernels.hip", "nsmi_walk.hip", "nsmi_hrss.hip", "nsmi_mlp.hip", "nsmi_host.cpp"]
HEADERS = ["nsmi_device.h", "nsmi_kernels.h", "nsmi_mlp.h", "nsmi_hrss.h"]

# Packed FP32 instructions stay off (they are formed by the compiler from
# scalar code otherwise); contraction is off so the explicit fma() calls are
# the only fused operations, as in the per-step parity definition.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    if verbose and r.stderr.strip():
        sys.stderr.write("\n".join(l for l in r.stderr.splitlines()
                                   if "packed-fp32-ops" not in l) + "\n")


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for s in SOURCES:
        o = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        cmds.append([cc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-x", "hip", "-c",
                     os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
        for f in [pool.submit(_run, c, verbose) for c in cmds]:
            f.result()
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"], verbose)
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
