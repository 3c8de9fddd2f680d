"""Build libgf (HIP, gfx950) in-tree: paper_1209_4008_amd/libgf.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("GF_OFFLOAD_ARCH", "gfx950")
SOURCES = [os.path.join(HERE, "csrc", "gf_api.hip")]


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    cmd = [
        HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-shared",
        # packed FP32 instructions are kept out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"),
    ]
    if resource_usage:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    cmd += SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv)
    sys.exit(0)
