"""Host-sanitizer build of the C-ABI runtime (AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only).

Builds ``build_san/libpf_san.so`` from the host-side translation units
(``pf_runtime.hip``, ``pf_batch.hip``, ``pf_noalloc.hip``) with the host
pass instrumented (``-Xarch_host -fsanitize=...``; device code is not
instrumented) and with the kernel launchers replaced by stubs that report
``hipErrorNoDevice``: it exercises argument checking, planning, allocation
bookkeeping, checkpoint parsing and error paths, not the kernels. Run the
C-ABI tests against it with the sanitizer runtime preloaded, e.g.

    python -m paper_1812_01502_amd.build_sanitized --run tests/test_abi.py
"""
from __future__ import annotations

import argparse
import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "build_san")
LIB = os.path.join(OUT, "libpf_san.so")
HOST_UNITS = ["pf_runtime.hip", "pf_batch.hip", "pf_noalloc.hip"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
STUBS = """#include "pf_launch.h"
namespace pfk {
hipError_t launch_f32(const LaunchReq&, const void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_bf16(const LaunchReq&, const void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_f64(const LaunchReq&, const void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch(const BatchReq&, const BatchArgs&, hipStream_t) { return hipErrorNoDevice; }
}  // namespace pfk
"""


def asan_runtime() -> str | None:
    """The clang AddressSanitizer runtime of the ROCm toolchain (to preload
    into a Python process that loads the sanitized library)."""
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build(verbose: bool = True) -> str:
    from paper_1812_01502_amd.build import ARCH, _hipcc
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-Wno-unused-command-line-argument", *SAN]
    os.makedirs(OUT, exist_ok=True)
    tmp = tempfile.mkdtemp(prefix="pf_san_")
    try:
        stub = os.path.join(tmp, "launch_stubs.hip")
        with open(stub, "w") as f:
            f.write(STUBS)
        srcs = [os.path.join(CSRC, u) for u in HOST_UNITS if os.path.exists(os.path.join(CSRC, u))] + [stub]
        procs = []
        objs = []
        for s in srcs:
            o = os.path.join(tmp, os.path.basename(s) + ".o")
            objs.append(o)
            procs.append((s, subprocess.Popen([_hipcc(), *flags, "-c", s, "-o", o], stdout=subprocess.PIPE,
                                              stderr=subprocess.PIPE, text=True)))
        for s, p in procs:
            _, err = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed for {os.path.basename(s)}:\n{err[-4000:]}")
        r = subprocess.run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN[:4], "-o", LIB, *objs],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


def run_tests(paths, extra=()) -> int:
    """pytest on ``paths`` in a child process that loads the sanitized
    library (PF_LIBRARY) with the sanitizer runtime preloaded."""
    rt = asan_runtime()
    if rt is None:
        raise RuntimeError("no AddressSanitizer runtime found under /opt/rocm/lib/llvm")
    env = dict(os.environ, PF_LIBRARY=LIB, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *paths, *extra],
                          cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", nargs="*", default=None, help="test files to run against the sanitized library")
    a = ap.parse_args()
    build()
    if a.run is not None:
        sys.exit(run_tests(a.run or ["tests/test_abi.py"]))
