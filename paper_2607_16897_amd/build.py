"""Build step: compile the HIP sources for gfx950 into libdptrack.so (in-tree)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdptrack.so")
SOURCES = ["dpt_kernels.hip", "dpt_select.hip", "dpt_coop.hip", "dpt_cnn.hip", "dpt_probe.hip", "dpt_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",  # every FMA is explicit (fmaf)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",  # no packed FP32 instructions
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


LIB_CYCLES = os.path.join(HERE, "libdptrack_cycles.so")


def build(verbose: bool = False, cycles: bool = False) -> str:
    """cycles=True: the instrumented library (libdptrack_cycles.so, -DDPT_CYCLE_PROFILE)
    whose track kernels record the per-phase cycle split (dpt_cycle_profile)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = LIB_CYCLES if cycles else LIB
    tag = ".cyc" if cycles else ""
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", f"{tag}.o"))
        cmd = [hipcc, *HIPCC_FLAGS, *(["-DDPT_CYCLE_PROFILE"] if cycles else []),
               "-I", os.path.join(os.path.dirname(HERE), "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the sources compile independently: a few at a time
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1, 8)) as ex:
        for _ in ex.map(subprocess.check_call, cmds):
            pass
    tmp = lib + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, cycles="--cycles" in sys.argv))
