"""The host side of the library (argument validation, workspace carving, error and state
handling) under the host address and undefined-behaviour sanitizers: the CPU ABI tests run in
a child interpreter against libspg_san.so (GPU code built as usual, host runtime recompiled
with -fsanitize=address,undefined), with the sanitizer runtime preloaded.  Any sanitizer
report fails the run (UBSan is built not to recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_abi_tests_under_host_sanitizers():
    from paper_1905_13408_amd import build

    lib = build.build_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = build.sanitizer_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"  # the interpreter itself keeps memory
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    env["SPG_LIB_PATH"] = lib
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=540)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out
    assert " passed" in out
