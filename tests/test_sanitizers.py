"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two sanitized builds of the same sources: libgrid.so's host code (hipcc, each -fsanitize=
behind -Xarch_host, so the device code is built as usual) and the oracle (gcc). A process can
hold one ASan runtime, and the two builds come from two compilers, so each runs in a
subprocess of its own with its compiler's runtime preloaded: the library with the CPU tests of
the C ABI (code generation, argument checks, the server's and the mixed module's refusals
without a device), the oracle with its pins. Leak checking is off (the Python interpreter
keeps its own allocations to the end); any other report aborts the subprocess.

Each runtime is first shown to catch a planted heap overflow in a small test-only library
built the same way, so that a green run is not a run in which the sanitizer never looked.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_COMMON = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

PLANTED = r'''
#include <stdlib.h>
#ifdef __cplusplus
extern "C"
#endif
int planted_overflow(int n)
{
    int* a = (int*)malloc(sizeof(int) * n);
    for (int i = 0; i <= n; ++i)     /* one past the end */
        a[i] = i;
    int s = a[0];
    free(a);
    return s;
}
'''


def _gcc_runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _clang_runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
                  + glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _run(cmd, runtime, extra_env, timeout=900):
    env = dict(os.environ)
    env.update(ENV_COMMON)
    env.update(extra_env)
    env["LD_PRELOAD"] = runtime
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


def _planted_is_caught(lib_path, runtime):
    code = ("import ctypes, sys; l = ctypes.CDLL(sys.argv[1]); "
            "l.planted_overflow(8); print('not caught')")
    r = _run([sys.executable, "-c", code, lib_path], runtime, {}, timeout=120)
    return r.returncode != 0 and "heap-buffer-overflow" in r.stderr


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitized")
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    from paper_2109_06976_amd import build as lib_build
    out = {"grid": str(d / "libgrid_san.so"), "oracle": str(d / "liboracle_san.so"),
           "planted_gcc": str(d / "planted_gcc.so"), "planted_clang": str(d / "planted_clang.so")}
    lib_build.build_library(out=out["grid"], sanitize=True)
    oracle_build.build_sanitized(out["oracle"])
    src_c = d / "planted.c"
    src_c.write_text(PLANTED)
    src_cpp = d / "planted.cpp"
    src_cpp.write_text(PLANTED)
    subprocess.run(["gcc", "-shared", "-fPIC", "-O1", "-fsanitize=address,undefined",
                    "-o", out["planted_gcc"], str(src_c)], check=True)
    subprocess.run([lib_build.HIPCC, "-shared", "-fPIC", "-O1", *lib_build.HOST_SANITIZE,
                    "-o", out["planted_clang"], str(src_cpp)], check=True)
    return out


def test_oracle_pins_under_sanitizers(builds):
    rt = _gcc_runtime()
    assert rt, "gcc's ASan runtime not found"
    assert _planted_is_caught(builds["planted_gcc"], rt)
    r = _run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
              "tests/test_oracle_pins.py", "tests/test_oracle_vjp.py", "tests/test_oracle_dt.py"],
             rt, {"GRID_ORACLE_LIB": builds["oracle"]})
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]


def test_library_host_code_under_sanitizers(builds):
    rt = _clang_runtime()
    assert rt, "clang's ASan runtime not found"
    assert _planted_is_caught(builds["planted_clang"], rt)
    r = _run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
              "tests/test_abi.py", "tests/test_fixed_joints.py"],
             rt, {"GRID_LIB": builds["grid"]})
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
