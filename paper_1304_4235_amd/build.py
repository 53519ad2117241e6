"""Build librrt.so (the HIP library) in place with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["rrt.hip", "workspace.hip", "tree.hip", "trace.hip", "rate.hip", "adjoint.hip", "transpose.hip",
           "tiles.hip", "noalloc.hip"]
LIB = os.path.join(HERE, "librrt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = "/opt/rocm/lib"
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the leaf predicate must round operation by operation: honour the
    # fp contract pragmas in the sources, never contract across them
    "-ffp-contract=fast-honor-pragmas",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    # roctx ranges around the library's calls (the rocprofiler-sdk marker library)
    libs = ["-L", ROCM_LIB, "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *srcs, *libs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
