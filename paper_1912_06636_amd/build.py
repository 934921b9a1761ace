"""Build libnao.so (HIP for gfx950 + host C++) in place, next to this file.

    python -m paper_1912_06636_amd.build

The planning code (plan.cpp) is plain C++ built by g++ with -ffp-contract=off (the
relevance test must be evaluated unfused); the runtime (runtime.cpp) is host C++ against
the HIP runtime API; the kernels (kernels.hip) are built by hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnao.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # keep the compiler from forming packed FP32 instructions by itself
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall",
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include")]
    objs = []
    for src in ("plan.cpp", "runtime.cpp", "scheduler.cpp", "server.cpp"):
        o = os.path.join(OBJ, src + ".o")
        _run(["g++"] + CXX_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    for src in ("kernels.hip",):
        o = os.path.join(OBJ, src + ".o")
        _run([os.path.join(ROCM, "bin", "hipcc")] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", o],
             verbose)
        objs.append(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([os.path.join(ROCM, "bin", "hipcc"), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
         + ["-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
