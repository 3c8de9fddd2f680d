"""The oracle's pins (tests/test_oracle_*.py, tests/test_inputs.py) run again
against a build of oracle.c with AddressSanitizer and
UndefinedBehaviorSanitizer: no out-of-bounds access, use after free or
undefined behaviour anywhere the pins reach. Host code only, in a child
process that preloads the sanitizer runtimes."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_oracle_pins_under_address_and_ub_sanitizers():
    sys.path.insert(0, ROOT)
    from oracle import build_sanitized as bs
    lib = bs.build()
    env = dict(os.environ)
    env["GF_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = ":".join(bs.runtime_libs())
    # Python's own allocations are not the subject; halt on the first report
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    files = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_oracle_annealing.py", "test_oracle_mag.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow"] + files,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
    assert " passed" in r.stdout, tail
