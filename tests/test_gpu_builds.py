"""Every build of the fused kernel against the FP64 oracle, through the C ABI, on an MI355X.

Builds (grid_tune_apply pins one): 0 quad layout, 1-3 lane layout at 1, 2, 4 wavefronts per
SIMD, 4 quad layout in three roles, 5 one lane per knot, 6 four lanes per knot. Knot counts 1 and 37 leave ragged workgroups for every
packing; the tolerances are those of the parity tests (normwise per knot: qdd 1e-4, the
matrices 1e-3), and M^-1 must come out exactly symmetric.
"""
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth
from paper_2109_06976_amd.build import max_size_model, prismatic_models, star_model

pytestmark = pytest.mark.gpu

TOL = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}

ROBOTS = {
    "chain7": synth.chain7,
    "quad12": synth.quad12,
    "humanoid30": synth.humanoid30,
    "chain1": lambda: synth.random_model(synth.chain_parent(1), 40, "chain1"),
    "chain2": lambda: synth.random_model(synth.chain_parent(2), 41, "chain2"),
    "tree3": lambda: synth.random_model(np.array([-1, 0, 0], np.int32), 43, "tree3"),
    "fork3": lambda: synth.random_model(np.array([-1, -1, 1], np.int32), 44, "fork3"),
    "binary7": lambda: synth.random_model(np.array([-1, 0, 0, 1, 1, 2, 2], np.int32), 45,
                                          "binary7"),
    # joints about random unit axes (the library rotates body frames to make them z)
    "chain7-axes": lambda: synth.random_model(synth.chain_parent(7), 0, "chain7-axes",
                                              axes="random"),
    "tree5-axes": lambda: synth.random_model(np.array([-1, 0, 0, 1, -1], np.int32), 6,
                                             "tree5-axes", axes="random"),
    # prismatic joints among revolute ones (z axes, random axes, a 30-body branch set)
    "chain7-prism": lambda: prismatic_models()["chain7-prism"],
    "tree5-axes-prism": lambda: prismatic_models()["tree5-axes-prism"],
    "humanoid30-prism": lambda: prismatic_models()["humanoid30-prism"],
    # the largest robot the library accepts: 32 bodies, one branch of 20
    "humanoid32": max_size_model,
    # 32 bodies each on the base: 32 one-body branches, M diagonal
    "star32": star_model,
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(ROBOTS))
def test_every_build_matches_oracle(orc, name):
    import torch
    robot = ROBOTS[name]()
    m = grid.Model(robot)
    try:
        for build in range(len(grid.BUILD_KERNELS)):
            grid.tune_apply(m, {1 << 22: build})
            assert grid.build_for(m, 5) == build
            for N in (1, 37, 130):
                say(f"[gpu] {name}: build {build}, N={N}")
                kn = synth.random_knots(robot.n, N, 300 + N)
                out = grid.fd_grad_torch(m, *(torch.from_numpy(a).cuda()
                                              for a in (kn.q, kn.qd, kn.tau)))
                torch.cuda.synchronize()
                ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
                errs = {}
                for k, b in TOL.items():
                    y = out[k].cpu().numpy().astype(np.float64).reshape(N, -1)
                    r = ref[k].reshape(N, -1)
                    # normwise per knot; a knot whose reference is exactly zero (dqdd/dqd of a
                    # single joint) is held to the same bound in absolute terms
                    scale = np.abs(r).max(1)
                    errs[k] = float((np.abs(y - r).max(1) / np.where(scale > 0, scale, 1.0)).max())
                say("  " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()))
                for k, b in TOL.items():
                    assert errs[k] <= b, (name, build, N, k)
                Mi = out["Minv"].cpu().numpy()
                np.testing.assert_array_equal(Mi, np.swapaxes(Mi, 1, 2))
    finally:
        m.close()


def test_tune_apply_rejects_bad_tables():
    m = grid.Model(synth.chain7())
    try:
        for Ns, builds, status in (([64, 32], [0, 0], grid.GRID_EINVAL),
                                   ([0], [0], grid.GRID_EINVAL),
                                   ([64], [len(grid.BUILD_KERNELS)], grid.GRID_EUNSUPPORTED),
                                   ([64], [-1], grid.GRID_EUNSUPPORTED)):
            n = np.array(Ns, np.int32)
            b = np.array(builds, np.int32)
            rc = grid.lib().grid_tune_apply(m.handle, n.ctypes.data_as(grid._i32p),
                                            b.ctypes.data_as(grid._i32p), len(Ns))
            assert rc == status, (Ns, builds, rc)
        grid.tune_apply(m, {})
    finally:
        m.close()


@pytest.mark.parametrize("build", [grid.BUILD_SERIAL, grid.BUILD_SERIAL4, grid.BUILD_SERIAL2])
@pytest.mark.parametrize("name", ["chain7", "chain2", "chain7-prism", "quad12", "tree3", "star32"])
def test_serial_build_unaligned_outputs(name, build):
    """Builds 5, 6 and 7 stage the outputs of single-branch robots in LDS and write them with
    16-byte stores when the output arrays are 16-byte aligned, else one float at a time: outputs
    at an offset of one float from an aligned base equal the aligned run bit for bit (N = 100:
    full and partial wavefronts). A branched robot's smaller branches have their rows staged
    and written row by row, zeros in the other branches' columns included (builds 6 and 7 only
    when every branch fits, as on quad12, tree3 and star32): on arrays
    filled with NaN beforehand every element comes out finite, and nothing outside them is
    written."""
    import torch
    robot = ROBOTS[name]()
    m = grid.Model(robot)
    try:
        grid.tune_apply(m, {1 << 22: build})
        n, N = robot.n, 100
        kn = synth.random_knots(n, N, 808)
        ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
        say(f"[gpu] build {build} aligned vs unaligned outputs: {name} N={N}")
        sizes = (N * n, N * n * n, N * n * n, N * n * n)
        runs = []
        for off in (0, 1):
            bufs = [torch.full((s + 4,), float("nan"), device="cuda") for s in sizes]
            outs = [b[off:off + s] for b, s in zip(bufs, sizes)]
            m.fd_grad(*ins, *outs, N=N)
            torch.cuda.synchronize()
            runs.append([o.cpu().numpy() for o in outs])
            # nothing written outside the arrays
            for b, s in zip(bufs, sizes):
                head = b[:off].cpu().numpy()
                tail = b[off + s:].cpu().numpy()
                assert np.all(np.isnan(head)) and np.all(np.isnan(tail))
        for a, b in zip(*runs):
            assert np.all(np.isfinite(a))
            np.testing.assert_array_equal(b, a)
    finally:
        grid.tune_apply(m, {})
        m.close()


def test_untuned_build_choice():
    """The build an untuned model runs per batch size: the three-role kernel while its
    wavefronts fit one per SIMD, then the lane layout, build 6 from 64 knots per compute unit
    and build 5 from 128 (16384 and 32768 knots on the MI355X's 256); a robot with a branch of
    more than 8 bodies keeps the three-role kernel up to 4096 knots and takes build 6 beyond
    (the choices the tuner makes for these robots on an MI355X)."""
    import torch
    assert torch.cuda.is_available()
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    cases = {"chain7": {128: grid.BUILD_PIPE, 512: grid.BUILD_PIPE, 4096: grid.BUILD_LANE,
                        64 * cu - 1: grid.BUILD_LANE, 64 * cu: grid.BUILD_SERIAL4,
                        128 * cu - 1: grid.BUILD_SERIAL4, 128 * cu: grid.BUILD_SERIAL,
                        65536: grid.BUILD_SERIAL},
             "quad12": {64 * cu: grid.BUILD_SERIAL4, 128 * cu: grid.BUILD_SERIAL},
             "humanoid30": {128: grid.BUILD_PIPE, 1024: grid.BUILD_PIPE, 4096: grid.BUILD_PIPE,
                            8192: grid.BUILD_SERIAL4, 65536: grid.BUILD_SERIAL4}}
    for name, want in cases.items():
        m = grid.Model(synth.model_by_name(name))
        try:
            for N, build in want.items():
                assert grid.build_for(m, N) == build, (name, N, grid.build_for(m, N))
        finally:
            m.close()
