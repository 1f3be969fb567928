"""Build the SPFM HIP library for gfx950 in-tree: paper_1910_05180_amd/libspfm.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["step_kernels.hip", "step_local_tiled.hip", "step_local_batched.hip", "step_global.hip",
           "step_cf.hip", "resident.hip", "force.hip", "temporal.hip", "walls.hip", "volume.hip", "reduce.hip", "init.hip",
           "host_math.cpp", "api.cpp"]
LIB = os.path.join(HERE, "libspfm.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions (v_pk_*_f32) anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only where the source writes fma(): every inlined
    # copy of the point update then rounds alike, so results do not depend on
    # the tiling or on which loop of a sweep computes a plane
    "-ffp-contract=off",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, one hipcc per source) and link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, src + ".o") for src in SOURCES]

    def compile_one(src_obj):
        src, obj = src_obj
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
