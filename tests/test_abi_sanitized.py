"""The host-side ABI checks again, against a build of the library whose host
code carries AddressSanitizer and UndefinedBehaviorSanitizer: argument
validation, table layout and workspace planning all run on the CPU, so the
sanitizers see every path these checks exercise (device code is compiled as
usual and never launched here)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_checks_under_asan_and_ubsan():
    from paper_2511_03298_amd.build import asan_runtime, build
    try:
        runtime = asan_runtime()
    except RuntimeError:
        pytest.skip("the clang ASan runtime is not installed")
    lib = build(sanitize=True)
    undefined = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True,
                               text=True).stdout
    assert "__asan_report" in undefined and "__ubsan_handle" in undefined, "not instrumented"
    env = dict(os.environ, LD_PRELOAD=runtime, IVFPQ_LIB=lib, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout and "failed" not in r.stdout
