"""Build the HIP library in-tree for gfx950 (hipcc cross-compiles without a GPU).

Every source is compiled to an object of its own in parallel (device code is
not relocatable: each translation unit launches only its own kernels), then
the objects are linked into liblt.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblt.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["mg.hip", "mg_fused.hip", "krylov.hip", "unet.hip", "api.hip", "plan.cpp", "batch.cpp",
           "tune.hip", "noalloc.hip", "exact.hip", "geostat.hip", "block.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-pthread", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _jobs():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(s):
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")
        cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return s, obj, r

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(compile_one, srcs))
    failed = False
    for s, _, r in results:
        # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if msg.strip() and (verbose or r.returncode):
            print(f"--- {s}\n{msg}", flush=True)
        failed = failed or r.returncode != 0
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *[o for _, o, _ in results], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
