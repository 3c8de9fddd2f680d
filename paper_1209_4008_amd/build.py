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
# the debug library: the site-update kernels with every link-element access
# counted (checks of the RED/BLACK decomposition); not part of libgf
DEBUG_LIB = os.path.join(HERE, "libgf_debug.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("GF_OFFLOAD_ARCH", "gfx950")
CSRC = os.path.join(HERE, "csrc")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def debug_sources():
    return sorted(glob.glob(os.path.join(CSRC, "debug", "*.hip")))


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
    deps = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return max(os.path.getmtime(p) for p in deps)


def build(verbose: bool = False, resource_usage: bool = False, incremental: bool = False,
          jobs: int = 0) -> str:
    """Compile every unit (incremental=True: only units older than their
    source or a header) and link libgf.so and the debug library."""
    os.makedirs(OBJ, exist_ok=True)
    hdr_time = _newest_input()
    targets = [(LIB, sources(), []), (DEBUG_LIB, debug_sources(), ["-DGF_ACCESS_COUNT"])]
    todo = []
    for lib, srcs, defs in targets:
        for s in srcs:
            o = os.path.join(OBJ, os.path.basename(s)[:-4] + ".o")
            if (not incremental or not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(s)
                    or os.path.getmtime(o) < hdr_time):
                todo.append((s, o, defs))
    flags = _flags(resource_usage)

    def compile_one(job):
        s, o, defs = job
        cmd = [HIPCC] + flags + defs + ["-c", s, "-o", o + ".tmp"]
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
    for lib, srcs, _ in targets:
        objs = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in srcs]
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", lib + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv, incremental="--incremental" in sys.argv)
    sys.exit(0)
