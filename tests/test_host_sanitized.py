"""The library's host logic under AddressSanitizer and
UndefinedBehaviorSanitizer, with no GPU: tests/host_checks.py (spec
validation, argument checks of the entry points, store-file parsing of
damaged and fuzzed files) runs in a child process against the
host-sanitized variant librbfl_san.so with the clang ASan runtime
preloaded.  A sanitizer report aborts the child."""
import os
import subprocess
import sys

import pytest

from paper_2508_04172_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(os.path.join(build.CSRC, f)) > t for f in os.listdir(build.CSRC))


def test_host_logic_under_asan_and_ubsan():
    rt = build.asan_runtime()
    if not os.path.exists(rt):
        pytest.skip("clang ASan runtime not found")
    if _stale(build.LIB_SAN):
        build.build(sanitize=True)
    # the variant is instrumented: its host code calls the ASan runtime
    with open(build.LIB_SAN, "rb") as f:
        assert b"__asan_report_load8" in f.read()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_checks.py"), build.LIB_SAN], env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host checks:" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
