"""Build libgrid.so (hipcc, gfx950) in-tree and fill its kernel cache.

Steps:
  1. embed the device sources csrc/grid_device.hip, grid_fused.hip, grid_serial.hip and
     grid_ops.hip into generated includes (_build/<name>_src.inc);
  2. compile the host runtime (csrc/*.cpp) with hipcc into libgrid.so;
  3. compile the device source with hipcc for gfx950 behind a generated chain prelude
     (a full offline compile check; -save-temps keeps the ISA under _build/);
  4. run the library's own code generator + hiprtc for every topology the tests,
     benchmark and smoke check use, so no kernel is compiled inside a GPU run.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgrid.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# no packed FP32 instructions in any HIP code of this project
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the pipe kernel module's scheduling strategy (the library passes the same to hiprtc)
KERNEL_SCHED = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def embed_device_source() -> None:
    """Device sources as byte arrays for the library's code generator."""
    os.makedirs(BUILD, exist_ok=True)
    for name in ("grid_device", "grid_fused", "grid_serial", "grid_ops"):
        src = open(os.path.join(CSRC, f"{name}.hip"), "rb").read()
        body = ",".join(str(b) for b in src)
        inc = os.path.join(BUILD, f"{name}_src.inc")
        text = (f"// generated from csrc/{name}.hip by build.py\n"
                f"static const char {name}_src[] = {{{body},0}};\n")
        if not os.path.exists(inc) or open(inc).read() != text:
            with open(inc, "w") as f:
                f.write(text)


# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (each -fsanitize=
# behind -Xarch_host: the device code is built as usual)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build_library(verbose=False, out=None, sanitize=False) -> str:
    """libgrid.so in-tree; with sanitize=True a build of the same sources whose host code
    carries ASan and UBSan, at `out` (for the CPU tests under the sanitizers)."""
    embed_device_source()
    target = out or LIB
    opt = ["-O1", "-g", *HOST_SANITIZE] if sanitize else ["-O2"]
    cmd = [HIPCC, "-std=c++17", *opt, "-fPIC", "-shared", "-Wall", "-Wextra",
           "--offload-arch=gfx950", *NO_PACKED_FP32,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", BUILD,
           os.path.join(CSRC, "grid_runtime.cpp"), os.path.join(CSRC, "grid_codegen.cpp"),
           os.path.join(CSRC, "grid_vjp.hip"), os.path.join(CSRC, "grid_server.cpp"),
           os.path.join(CSRC, "grid_batch.cpp"), os.path.join(CSRC, "grid_noalloc.hip"),
           os.path.join(CSRC, "grid_io.hip"),
           "-lhiprtc", "-lpthread", "-o", target + ".tmp"]
    _run(cmd, verbose)
    os.replace(target + ".tmp", target)
    return target


def standard_models():
    """Every robot model the tests, the benchmark and the smoke check instantiate."""
    import numpy as np
    from paper_2109_06976_amd import synth
    models = [synth.chain7(), synth.quad12(), synth.humanoid30(),
              synth.humanoid30(variant="literal")]
    # small trees of the GPU tests: (parent, seed)
    for parent, seed in [([-1], 40), ([-1, 0], 41), ([-1, 0, 1], 42), ([-1, 0, 0], 43),
                         ([-1, -1, 1], 44), ([-1, 0, 0, 1, 1, 2, 2], 45)]:
        models.append(synth.random_model(np.array(parent, np.int32), seed))
    # joints about random axes
    models.append(synth.random_model(synth.chain_parent(7), 0, axes="random"))
    models.append(synth.random_model(np.array([-1, 0, 0, 1, -1], np.int32), 6, axes="random"))
    # fixed joints
    models.append(synth.with_fixed_joints(synth.chain7(), [2, 5]))
    models.append(synth.with_fixed_joints(
        synth.random_model(np.array([-1, 0, 0, 1, 3, -1, 5], np.int32), 77), [1, 3, 6]))
    models.append(synth.with_fixed_joints(
        synth.random_model(synth.chain_parent(7), 0, axes="random"), [0, 4]))
    # prismatic joints (with revolute ones; random axes; on a branch beyond 16 bodies;
    # with fixed joints, one welded to a prismatic owner)
    models.extend(prismatic_models().values())
    # the largest robot the library accepts (32 bodies), and 32 bodies each on the base
    models.append(max_size_model())
    models.append(star_model())
    return models


def star_model():
    """32 bodies, each on its own joint to the fixed base: 32 branches of one body, M
    diagonal (the degenerate tree)."""
    import numpy as np
    from paper_2109_06976_amd import synth
    return synth.random_model(np.full(32, -1, np.int32), 48, "star32")


def max_size_model():
    """32 bodies (the library's maximum): the humanoid with a hand on each arm, so the
    torso tree is one branch of 20 bodies."""
    import numpy as np
    from paper_2109_06976_amd import synth
    parent = np.concatenate([synth.humanoid_parent(), np.array([22, 29], np.int32)])
    return synth.random_model(parent.astype(np.int32), 47, "humanoid32")


def prismatic_models():
    """The robots with prismatic joints that the tests run, by name."""
    import numpy as np
    from paper_2109_06976_amd import synth
    tree5 = synth.random_model(np.array([-1, 0, 0, 1, -1], np.int32), 6, "tree5-axes",
                               axes="random")
    tree7 = synth.random_model(np.array([-1, 0, 0, 1, 3, -1, 5], np.int32), 77, "tree7")
    return {
        "chain7-prism": synth.with_prismatic_joints(synth.chain7(), [1, 4]),
        "tree5-axes-prism": synth.with_prismatic_joints(tree5, [0, 3, 4]),
        "humanoid30-prism": synth.with_prismatic_joints(synth.humanoid30(), [1, 9, 20, 29]),
        "tree7-fixed-prism": synth.with_prismatic_joints(
            synth.with_fixed_joints(tree7, [1, 3, 6]), [0, 4]),
    }


def mixed_sets():
    """The robot lists of the mixed modules (one launch, several robots) that the tests and
    the benchmark create."""
    from paper_2109_06976_amd import synth
    prism = prismatic_models()
    return [
        [synth.quad12(), synth.chain7()],
        [synth.chain7(), synth.quad12(), synth.humanoid30(), prism["tree5-axes-prism"],
         prism["tree7-fixed-prism"], star_model()],
    ]


def offline_compile_check(verbose=False):
    """hipcc --genco of the generated sources (both modules) for the three workload robots,
    with the options the library gives hiprtc for each."""
    from paper_2109_06976_amd import grid, synth
    for robot in (synth.chain7(), synth.quad12(), synth.humanoid30()):
        name = robot.name.split("-")[0]
        for suffix, flags, extra in (("", 0, []),
                                     ("_pipe", grid.GRID_CODEGEN_PIPE_MODULE, KERNEL_SCHED)):
            src = "#include <hip/hip_runtime.h>\n" + grid.codegen_source(robot, flags)
            path = os.path.join(BUILD, f"{name}{suffix}.hip")
            with open(path, "w") as f:
                f.write(src)
            out = os.path.join(BUILD, f"{name}{suffix}.hsaco")
            _run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", *NO_PACKED_FP32, *extra,
                  "--genco", "-save-temps=obj", "-o", out, path], verbose)


def _precompile_one(robot):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_2109_06976_amd import grid
    grid.codegen_precompile(robot)
    return robot.name


def _precompile_mixed(k):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_2109_06976_amd import grid
    robots = mixed_sets()[k]
    grid.mixed_precompile(robots)
    return "+".join(r.name for r in robots)


def precompile(verbose=False, workers=None):
    """Compile every standard model's kernels and the mixed modules into the cache, several
    at a time (one process each: a compile is single-threaded), the largest first."""
    import concurrent.futures
    import multiprocessing
    robots = sorted(standard_models(), key=lambda r: -r.n)
    workers = workers or max(1, min(8, os.cpu_count() or 1))
    ctx = multiprocessing.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as pool:
        jobs = [pool.submit(_precompile_mixed, k) for k in range(len(mixed_sets()))]
        jobs += [pool.submit(_precompile_one, r) for r in robots]
        for job in jobs:
            name = job.result()
            if verbose:
                print(f"cached kernels for {name}", flush=True)


def build(verbose=False):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    build_library(verbose)
    offline_compile_check(verbose)
    precompile(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
