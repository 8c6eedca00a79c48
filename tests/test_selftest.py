"""The C ABI's host logic under AddressSanitizer and
UndefinedBehaviorSanitizer: paper_1903_00548_amd/qtx_selftest is the
self-test built by __graft_entry__.build() with the host code sanitized
(device code as in the library).  Here its host-only part runs (layout
self-check, version, error paths without a context, the charge helper);
tests/test_gpu_selftest.py runs the device part."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1903_00548_amd", "qtx_selftest")


def run_selftest(*args, timeout=120):
    if not os.path.exists(EXE):
        pytest.skip("qtx_selftest is not built (run __graft_entry__.build())")
    env = dict(os.environ)
    # the HIP runtime's own allocations live until exit: leak reports off;
    # any other report aborts with a non-zero status
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    p = subprocess.run([EXE, *args], capture_output=True, text=True, timeout=timeout, env=env)
    print(p.stdout[-2000:], p.stderr[-4000:])
    return p


def test_host_logic_under_sanitizers():
    p = run_selftest()
    assert p.returncode == 0, p.stderr[-4000:]
    assert "selftest: ok (host only)" in p.stdout
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr
