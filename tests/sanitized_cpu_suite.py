"""Runs the CPU test suite (-m "not gpu") against sanitized builds.

Builds the HIP library's host code only (``paper_0912_1379_amd/build.py
--sanitize``: argument checks, planner, ragged descriptor classification,
tune-line parser) and the oracle, both under AddressSanitizer and
UndefinedBehaviorSanitizer with the ROCm clang, then runs pytest in a child
process that preloads clang's sanitizer runtime and loads those two libraries
in place of the normal ones (LCT_LIBRARY, LCT_ORACLE_LIBRARY).  Any report
ends the run with a non-zero status.  Not collected by pytest (no test_ prefix):

    python tests/sanitized_cpu_suite.py [extra pytest arguments]
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import build as oracle_build  # noqa: E402
from paper_0912_1379_amd import build as lib_build  # noqa: E402


def runtime() -> str:
    r = subprocess.run([oracle_build.CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True, check=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang's ASan runtime not found")
    return path


def stale(lib: str) -> bool:
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(lib_build.CSRC, f) for f in os.listdir(lib_build.CSRC)]
    srcs += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return any(os.path.getmtime(f) > t for f in srcs)


def main(extra: list) -> int:
    lib = lib_build.SAN_LIB
    if stale(lib):
        lib = lib_build.build_sanitized()  # about two minutes: the device code is compiled as usual
    olib = oracle_build.build_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime(),
        # the interpreter and torch are not instrumented: their allocations at exit are not ours
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "LCT_LIBRARY": lib,
        "LCT_ORACLE_LIBRARY": olib,
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x", "-q",
           "-p", "no:cacheprovider", *extra]
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
