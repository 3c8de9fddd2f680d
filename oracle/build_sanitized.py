"""Build the oracle with AddressSanitizer and UndefinedBehaviorSanitizer into
oracle/liboracle_san.so (test infrastructure: a CPU test runs the oracle's
pins against the sanitized library, see tests/test_oracle_sanitized.py). Host code only;
plain gcc, the same flags as oracle/build.py plus the sanitizers."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_san.so")


def runtime_libs():
    """the sanitizer runtimes a host process must preload to load the build"""
    out = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                           check=True).stdout.strip()
        out.append(os.path.realpath(p))
    return out


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-fno-omit-frame-pointer",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
        os.path.join(HERE, "oracle.c"), "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
