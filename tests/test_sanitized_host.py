"""The host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

The analysis (R-tree, levels, transfer tables, Galerkin patterns), the matrix-free set-up and the C ABI are
rebuilt with both sanitizers on their host side (paper_2607_28235_amd.build.build_sanitized) and the host
test-suite (tests/test_library_host.py, tests/test_error_paths.py; the full-size analysis excepted) runs
against that build in a child process with the sanitizer runtime preloaded.  Any out-of-bounds access, use
after free or undefined behaviour aborts the child, which fails this test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_2607_28235_amd import build as B
    lib = B.build_sanitized()
    out = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in out and "__ubsan_handle" in out      # the sanitizers are compiled in
    env = dict(os.environ)
    env.update(LD_PRELOAD=B.sanitizer_runtime(), R3MG_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_library_host.py", "tests/test_error_paths.py",
                        "-q", "-x", "-p", "no:cacheprovider", "-m", "not slow and not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout
