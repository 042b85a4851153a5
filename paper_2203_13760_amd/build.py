"""Build libcfd.so (the HIP kernels and the C ABI) in-tree for gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcfd.so")
SRC = os.path.join(HERE, "csrc", "cfd.hip")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950",
    # packed FP32 instructions stay off (the kernels are FP64; this keeps the
    # compiler from forming them anywhere in the library)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fPIC", "-shared",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
