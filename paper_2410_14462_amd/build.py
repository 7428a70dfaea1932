"""Build the gfx950 shared library liblv.so next to this file with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["geometry.hip", "sort.hip", "blend.hip", "codec.hip", "diffuse.hip", "prune.hip", "graph.hip",
           "api.hip", "serve.hip"]
LIB = os.path.join(HERE, "liblv.so")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # exact FP32: no contraction, IEEE denormals, correctly rounded div/sqrt
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # roctx ranges around the phases of a call (rocprofv3 --marker-trace)
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-o", out] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
