"""Build the oracle's shared library with gcc (CPU only).

Test infrastructure: the oracle is compiled here, next to its source, and is
loaded only by the tests, the smoke check and the CPU-baseline leg of the
benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lct_oracle.c")
LIB = os.path.join(HERE, "liblct_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# The same source under AddressSanitizer and UndefinedBehaviorSanitizer, built
# with the ROCm clang so that one sanitizer runtime serves it and the HIP
# library's host-only sanitized build in the same process.
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_LIB = os.path.join(os.path.dirname(HERE), "_build", "san", "liblct_oracle_san.so")


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    omp = os.path.join(os.path.dirname(os.path.dirname(CLANG)), "lib")
    cmd = [CLANG, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-shared-libsan", "-Wall", "-Wextra",
           f"-Wl,-rpath,{omp}", "-o", SAN_LIB, SRC, "-lm", "-latomic"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        print(build_sanitized(verbose=True))
        sys.exit(0)
    print(build(verbose=True))
    sys.exit(0)
