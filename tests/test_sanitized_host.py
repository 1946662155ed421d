"""The C-ABI tests against a host-sanitized build of the runtime
(AddressSanitizer and UndefinedBehaviorSanitizer on the host code; kernel
launchers stubbed): argument checks, planning, allocator bookkeeping and
error paths run without a memory error or undefined behaviour."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_under_host_sanitizers():
    from paper_1812_01502_amd import build_sanitized as BS
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no HIP toolchain")
    if BS.asan_runtime() is None:
        pytest.skip("no AddressSanitizer runtime in the toolchain")
    BS.build(verbose=False)
    env = dict(os.environ, PF_LIBRARY=BS.LIB, LD_PRELOAD=BS.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
