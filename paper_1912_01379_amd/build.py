"""Build libasm.so (HIP, gfx950) in the package directory with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libasm.so")
# the on-chip microbenchmarks of bench.py --micro, in a library of their own
MICRO_SRC, MICRO_OUT = "micro.hip", os.path.join(HERE, "libasm_micro.so")
SOURCES = ["api.hip", "setup.hip", "sample.hip", "linalg.hip", "sample32.hip", "sample32p_l16.hip", "sample32_l4.hip",
           "sample32_l8.hip", "sample32_l16.hip", "sample32_l32.hip", "sample32_l64.hip", "sample32w_l8.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 arithmetic stays off: the scalar float code is what the samplers use
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs, so loop-carried sums are not copied between
    # register files every iteration
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for s in SOURCES:
        obj = os.path.join(bdir, s.replace(".hip", ".o"))
        cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(SRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    tmp = MICRO_OUT + ".tmp"
    cmd = [hipcc] + FLAGS + [os.path.join(SRC, MICRO_SRC), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, MICRO_OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
