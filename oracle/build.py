"""Build the FP64 oracle shared library (test infrastructure only).

build(): plain gcc -O2, no architecture-specific flags, so the library built here also runs
on the host of the GPU machine (the tests and the smoke check load it).

build_timing(path): the same source with -O3 -march=native, for timing the oracle as the CPU
baseline. It is built on the machine that runs it (native instructions of that host), into a
path the caller names, and only the benchmark's CPU-baseline leg loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgrid_oracle.so")
SRC = os.path.join(HERE, "grid_oracle.c")
TIMING_FLAGS = ["-O3", "-march=native"]


def _compile(opt, out, verbose):
    cmd = ["gcc", "-std=gnu11", *opt, "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-Wno-unused-function", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(out + ".tmp", out)
    return cmd


def build(verbose: bool = False) -> str:
    _compile(["-O2"], LIB, verbose)
    return LIB


def build_sanitized(path: str, verbose: bool = False) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer, at `path` (for the
    CPU tests under the sanitizers)."""
    return " ".join(_compile(["-O1", "-g", "-fsanitize=address,undefined",
                              "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
                             path, verbose))


def build_timing(path: str, verbose: bool = False) -> str:
    """The timing build at `path`; returns the gcc command line it used."""
    return " ".join(_compile(TIMING_FLAGS, path, verbose))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
