"""Build libgf (HIP, gfx950) in-tree: paper_1209_4008_amd/libgf.so.

Each translation unit under csrc/ is compiled to an object file in parallel
(the kernels an entry point instantiates are compiled in its own unit), then
the objects are linked into the shared library.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgf.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("GF_OFFLOAD_ARCH", "gfx950")
CSRC = os.path.join(HERE, "csrc")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _flags(resource_usage=False):
    f = [
        f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
        # packed FP32 instructions are kept out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"),
    ]
    if resource_usage:
        f += ["-Rpass-analysis=kernel-resource-usage"]
    return f


def _newest_input():
    deps = glob.glob(os.path.join(CSRC, "*.hpp")) + [os.path.join(ROOT, "include", "gf.h")]
    return max(os.path.getmtime(p) for p in deps)


def build(verbose: bool = False, resource_usage: bool = False, incremental: bool = False,
          jobs: int = 0) -> str:
    """Compile every unit (incremental=True: only units older than their
    source or a header) and link libgf.so."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    hdr_time = _newest_input()
    todo = []
    objs = []
    for s in srcs:
        o = os.path.join(OBJ, os.path.basename(s)[:-4] + ".o")
        objs.append(o)
        if (not incremental or not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(s)
                or os.path.getmtime(o) < hdr_time):
            todo.append((s, o))
    flags = _flags(resource_usage)

    def compile_one(so):
        s, o = so
        cmd = [HIPCC] + flags + ["-c", s, "-o", o + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {os.path.basename(s)} failed:\n{r.stderr}")
        os.replace(o + ".tmp", o)
        return r.stderr

    n = jobs or min(len(todo), os.cpu_count() or 4, 16) or 1
    with concurrent.futures.ThreadPoolExecutor(max_workers=n) as ex:
        for err in ex.map(compile_one, todo):
            if resource_usage and err:
                print(err, flush=True)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv, incremental="--incremental" in sys.argv)
    sys.exit(0)
