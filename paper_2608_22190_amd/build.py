"""Build libhpsmc.so (gfx950) in-tree with hipcc.

    python -m paper_2608_22190_amd.build

Packed FP32 instructions are disabled (-packed-fp32-ops) for every HIP
translation unit.  The units compile in parallel (one process each, at most
one per CPU and at most 16).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhpsmc.so")
SOURCES = ["hpsmc_kern_valu_f32.hip", "hpsmc_kern_valu_f64.hip", "hpsmc_kern_mma.hip", "hpsmc_kern_mma5.hip",
           "hpsmc_kern_adjoint.hip", "hpsmc_kern_frac.hip", "hpsmc_kern_1d.hip", "hpsmc_kernels.hip",
           "hpsmc_host.cpp"]
HEADERS = ["hpsmc_internal.h", "hpsmc_device.h", "hpsmc_round.h", "hpsmc_lobatto_eigs.h"]
# per-unit extra flags: in the vector-unit round kernels machine LICM hoists
# every loop-invariant constant of the walk (series coefficients, source and
# nonlinearity parameters) into registers held across the step loop, which
# costs occupancy (FP64, one path per lane: the windowed 1-D kernel 150 -> 77
# VGPRs without it, the general 2-D kernel 225 -> 153)
_NO_MLICM = ["-mllvm", "-disable-machine-licm"]
UNIT_FLAGS = {"hpsmc_kern_1d.hip": _NO_MLICM, "hpsmc_kern_valu_f64.hip": _NO_MLICM,
              "hpsmc_kern_valu_f32.hip": _NO_MLICM}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True skips objects newer than their
    source and the shared headers)."""
    headers = [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "hpsmc.h")]
    jobs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        objs.append(obj)
        deps = [os.path.join(CSRC, src)] + headers
        if incremental and os.path.exists(obj) and all(os.path.getmtime(obj) > os.path.getmtime(d) for d in deps):
            continue
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        jobs.append([HIPCC] + FLAGS + UNIT_FLAGS.get(src, []) + lang + ["-c", os.path.join(CSRC, src), "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(run, c) for c in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
