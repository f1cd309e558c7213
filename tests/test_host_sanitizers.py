"""The host code of libhlb (argument checks, planner, tuning table, workspace and batch
bookkeeping) under AddressSanitizer and UndefinedBehaviorSanitizer: the library is rebuilt
with both sanitizers on its host compilation only, and the CPU ABI tests run against that
build in a child process with the shared ASan runtime preloaded.  Any sanitizer report ends
the child with an error."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_clean_under_host_asan_and_ubsan():
    from paper_2503_16080_amd import _sanitize
    try:
        runtime = _sanitize.asan_runtime()
    except FileNotFoundError:
        pytest.skip("no shared ASan runtime next to hipcc")
    lib = _sanitize.build()
    # the build is instrumented (it imports the ASan entry points)
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_init" in syms and "__ubsan_handle" in syms
    env = dict(os.environ, LD_PRELOAD=runtime, HLB_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:alloc_dealloc_mismatch=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = ("import paper_2503_16080_amd as h; h.load(); print(h.library_path())")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == lib, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi_cpu.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
