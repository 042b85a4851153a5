"""Build the GPU check programs under tests/native for gfx950 (hipcc), next
to their sources; __graft_entry__.build() calls this with the library build,
so the GPU tests only run what is already built."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CHECKS = ["arith_check"]
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> None:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    for name in CHECKS:
        out = os.path.join(HERE, name)
        cmd = [hipcc, *FLAGS, "-o", out + ".tmp", os.path.join(HERE, name + ".hip")]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
