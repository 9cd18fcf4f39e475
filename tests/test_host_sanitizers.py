"""The runtime's host code under AddressSanitizer and UBSan.

build.py links a second copy of the library whose host code is instrumented
(device code is not: every -fsanitize= applies to the host pass only) and two
C programs against it.  The host-only paths run here without a GPU; the C
ABI program (setup, solve, error paths, destroy) runs on the GPU.  Any
sanitizer report fails the run (halt_on_error)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_PATHS = os.path.join(ROOT, "tests", "c", "ori_host_paths_asan")
SMOKE = os.path.join(ROOT, "tests", "c", "ori_abi_smoke_asan")


def _run(path, leaks):
    if not os.path.exists(path):
        pytest.skip("sanitized build not present (the compiler has no ASan runtime)")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={int(leaks)}:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    p = subprocess.run([path], env=env, capture_output=True, text=True, timeout=300)
    report = p.stdout[-2000:] + p.stderr[-4000:]
    assert p.returncode == 0, report
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, report
    return p.stdout


def test_host_paths_clean_under_asan_ubsan():
    # argument checks, sizes, failed creates and the out-of-memory refusal,
    # with leak detection (no device involved)
    assert "OK 0" in _run(HOST_PATHS, leaks=True)


@pytest.mark.gpu
def test_c_abi_program_clean_under_asan_ubsan():
    # the whole C ABI path with device work; the HIP runtime keeps its own
    # allocations until exit, so leaks are not checked here
    assert _run(SMOKE, leaks=False).startswith("OK")
