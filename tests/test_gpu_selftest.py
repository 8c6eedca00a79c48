"""The C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (host
code) on the GPU: every entry point on small synthetic problems (argument
errors, host and device solves, the no-allocation solve, self-energies,
charge, bands, density-matrix blocks, autotuning, a batch of three
problems replayed from its graph, the mode-space method, kernel timing),
with the checks that hold whatever the numbers (status codes, finite
outputs, bit-equal results where the entry points promise them).  The
self-test is a child process; a sanitizer report fails it."""
import pytest

from test_selftest import run_selftest

pytestmark = pytest.mark.gpu


def test_device_paths_under_sanitizers(gpu_lib):
    p = run_selftest("--gpu", timeout=240)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "selftest: ok (host and device)" in p.stdout
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr
