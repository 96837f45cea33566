"""Parity of the HIP path with the FP64 oracle, through the C ABI, on an MI355X.

Tolerance (normwise per knot and per output, the reading of the stated relative
errors): e = max_ij |Y - Y_ref| / max_ij |Y_ref|; qdd <= 1e-4, and M^-1, dqdd/dq,
dqdd/dqd <= 1e-3. The oracle consumes the same float32 inputs promoted to float64.
"""
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth
from paper_2109_06976_amd.build import prismatic_models

pytestmark = pytest.mark.gpu

TOL = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}
OUTS = ("qdd", "Minv", "dqdd_dq", "dqdd_dqd")

ROBOTS = {
    "chain7": synth.chain7,
    "quad12": synth.quad12,
    "humanoid30": synth.humanoid30,
    "humanoid30-literal": lambda: synth.humanoid30(variant="literal"),
    "chain1": lambda: synth.random_model(synth.chain_parent(1), 40, "chain1"),
    "chain2": lambda: synth.random_model(synth.chain_parent(2), 41, "chain2"),
    "chain3": lambda: synth.random_model(synth.chain_parent(3), 42, "chain3"),
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
}

_models = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def get_model(name, flags=0):
    key = (name, flags)
    if key not in _models:
        _models[key] = (ROBOTS[name](), grid.Model(ROBOTS[name](), device=0, flags=flags))
    return _models[key]


def run_device(torch, model, kn):
    q = torch.from_numpy(kn.q).cuda()
    qd = torch.from_numpy(kn.qd).cuda()
    tau = torch.from_numpy(kn.tau).cuda()
    out = grid.fd_grad_torch(model, q, qd, tau)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def normwise(y, ref):
    N = ref.shape[0]
    d = np.abs(y.astype(np.float64) - ref).reshape(N, -1).max(axis=1)
    s = np.abs(ref).reshape(N, -1).max(axis=1)
    return d / np.maximum(s, 1e-300)


def check(orc, robot, kn, got, tol=TOL, label=""):
    ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
    worst = {}
    for k in OUTS:
        assert np.all(np.isfinite(got[k])), f"{label} {k} has non-finite values"
        e = normwise(got[k], ref[k])
        worst[k] = float(e.max())
    say(f"  {label} worst normwise error: " +
        ", ".join(f"{k}={v:.2e}" for k, v in worst.items()))
    for k in OUTS:
        assert worst[k] <= tol[k], f"{label} {k}: {worst[k]:.3e} > {tol[k]:.1e}"
    # M^-1 is returned exactly symmetric
    np.testing.assert_array_equal(got["Minv"], np.swapaxes(got["Minv"], 1, 2))
    return worst


@pytest.mark.parametrize("name,N,seed", [
    ("chain7", 16, 101),          # the 7-dof correctness configuration
    ("chain7", 37, 5),            # ragged tail: not a multiple of the knots per wavefront
    ("chain7", 128, 102),         # the benchmark's launch
    ("chain7", 1024, 102),
    ("quad12", 64, 103),
    ("quad12", 33, 6),
    ("quad12", 1024, 103),
    ("humanoid30", 128, 104),
    ("humanoid30-literal", 19, 7),
    ("chain1", 65, 8),
    ("chain2", 40, 9),
    ("chain3", 21, 10),
    ("tree3", 17, 11),
    ("fork3", 9, 12),
    ("binary7", 13, 13),
    ("chain7-axes", 128, 14),
    ("tree5-axes", 41, 15),
    ("chain7-prism", 128, 16),
    ("tree5-axes-prism", 41, 17),
    ("humanoid30-prism", 37, 18),
])
def test_fd_grad_matches_oracle(torch_cuda, orc, name, N, seed):
    robot, model = get_model(name)
    say(f"[gpu] fd_grad {name} N={N} seed={seed} lanes/knot={model.lanes_per_knot}")
    kn = synth.random_knots(robot.n, N, seed)
    got = run_device(torch_cuda, model, kn)
    check(orc, robot, kn, got, label=f"{name} N={N}")


def test_single_knot_and_empty(torch_cuda, orc):
    robot, model = get_model("chain7")
    say("[gpu] fd_grad chain7 N=1 and N=0")
    kn = synth.random_knots(robot.n, 1, 77)
    got = run_device(torch_cuda, model, kn)
    check(orc, robot, kn, got, label="chain7 N=1")
    t = torch_cuda.empty(0, device="cuda")
    model.fd_grad(t, t, t, t, t, t, t, N=0)     # no-op
    torch_cuda.cuda.synchronize()


def test_results_do_not_depend_on_batch_position(torch_cuda):
    """A knot gives bitwise the same outputs alone and inside a larger batch."""
    robot, model = get_model("quad12")
    say("[gpu] batch-position independence quad12")
    kn = synth.random_knots(robot.n, 50, 21)
    full = run_device(torch_cuda, model, kn)
    for k in (0, 13, 49):
        one = synth.Knots(kn.q[k:k + 1], kn.qd[k:k + 1], kn.tau[k:k + 1])
        alone = run_device(torch_cuda, model, one)
        for key in OUTS:
            np.testing.assert_array_equal(alone[key][0], full[key][k])


def test_host_pointer_path_matches_device_path(torch_cuda):
    robot, model = get_model("chain7")
    say("[gpu] host-pointer path chain7 N=100")
    kn = synth.random_knots(robot.n, 100, 31)
    dev = run_device(torch_cuda, model, kn)
    ws = grid.Workspace(model, 128)
    host, timing = ws.fd_grad_host(kn.q, kn.qd, kn.tau)
    ws.close()
    for key in OUTS:
        np.testing.assert_array_equal(host[key], dev[key])
    assert timing["kernel_ms"] > 0 and timing["total_ms"] >= timing["kernel_ms"]
    with pytest.raises(grid.GridError):
        ws2 = grid.Workspace(model, 8)
        ws2.fd_grad_host(kn.q, kn.qd, kn.tau)     # N > max_knots


def test_pinned_path_matches_device_path(torch_cuda):
    """The pinned-buffer call (inputs written in place, no pageable copies), in one piece and
    split into overlapping pieces, gives bitwise the device path's outputs (each piece runs the
    build picked for its own knot count, so the model is pinned to one build here)."""
    robot, model = get_model("chain7")
    N = 300
    kn = synth.random_knots(robot.n, N, 35)
    ws = grid.Workspace(model, 512)
    try:
        for build in (grid.BUILD_PIPE, grid.BUILD_LANE):
            grid.tune_apply(model, {1 << 22: build})
            dev = run_device(torch_cuda, model, kn)
            for pieces in (1, 2, 3, 7):
                say(f"[gpu] pinned path chain7 N={N} build {build} pieces={pieces}")
                ins, outs = ws.host_buffers(N)
                ins["q"][:], ins["qd"][:], ins["tau"][:] = kn.q, kn.qd, kn.tau
                for o in outs.values():
                    o.fill(np.nan)
                t = ws.fd_grad_pinned(N, pieces)
                assert t["total_ms"] > 0
                if pieces == 1:
                    assert t["kernel_ms"] > 0 and t["h2d_ms"] > 0 and t["d2h_ms"] > 0
                for key in OUTS:
                    np.testing.assert_array_equal(outs[key], dev[key])
        with pytest.raises(grid.GridError) as e:
            ws.fd_grad_pinned(N, 0)
        assert e.value.status == grid.GRID_EINVAL
        with pytest.raises(grid.GridError) as e:
            ws.fd_grad_pinned(513, 1)
        assert e.value.status == grid.GRID_EINVAL
    finally:
        grid.tune_apply(model, {})
        ws.close()


@pytest.mark.parametrize("name,N", [("chain7", 301), ("humanoid30", 37), ("quad12", 1)])
def test_mapped_path_matches_device_path(torch_cuda, name, N):
    """The mapped call (the fused kernel reads the pinned inputs through the device mapping;
    the outputs reach the pinned buffer through a copy kernel or straight from the fused
    kernel's stores) gives bitwise the device path's outputs, for a size whose packed outputs
    leave a tail of floats after the 16-byte copies."""
    robot, model = get_model(name)
    kn = synth.random_knots(robot.n, N, 36)
    dev = run_device(torch_cuda, model, kn)
    ws = grid.Workspace(model, N + 3)
    try:
        for mode in (grid.IO_COPY_KERNEL, grid.IO_DIRECT):
            say(f"[gpu] mapped path {name} N={N} mode {mode}")
            ins, outs = ws.host_buffers(N)
            ins["q"][:], ins["qd"][:], ins["tau"][:] = kn.q, kn.qd, kn.tau
            for o in outs.values():
                o.fill(np.nan)
            t = ws.fd_grad_mapped(N, mode)
            assert t["total_ms"] > 0 and t["kernel_ms"] > 0 and t["h2d_ms"] == 0
            for key in OUTS:
                np.testing.assert_array_equal(outs[key], dev[key], err_msg=f"{key} mode {mode}")
        with pytest.raises(grid.GridError) as e:
            ws.fd_grad_mapped(N, 2)
        assert e.value.status == grid.GRID_EINVAL
        with pytest.raises(grid.GridError) as e:
            ws.fd_grad_mapped(N + 4, 0)
        assert e.value.status == grid.GRID_EINVAL
    finally:
        ws.close()


def test_invalid_launch_arguments(torch_cuda):
    robot, model = get_model("chain7")
    t = torch_cuda.zeros((4, 7), device="cuda")
    with pytest.raises(grid.GridError) as e:
        model.fd_grad(t, t, t, t, t, t, t, N=-1)
    assert e.value.status == grid.GRID_EINVAL
    with pytest.raises(grid.GridError) as e:
        model.fd_grad(t, None, t, t, t, t, t, N=4)
    assert e.value.status == grid.GRID_EINVAL


def test_bound_call_matches_plain_call(torch_cuda):
    """fd_grad_call (arguments converted once, called repeatedly) gives bitwise the outputs of
    fd_grad on the same buffers."""
    robot, model = get_model("chain7")
    say("[gpu] bound call chain7 N=77")
    kn = synth.random_knots(robot.n, 77, 41)
    ins = [torch_cuda.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
    n = robot.n
    outs = [torch_cuda.empty((77, n), device="cuda")] + \
        [torch_cuda.empty((77, n, n), device="cuda") for _ in range(3)]
    ref = run_device(torch_cuda, model, kn)
    call = model.fd_grad_call(*ins, *outs)
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        call()
        torch_cuda.cuda.synchronize()
        for key, o in zip(OUTS, outs):
            np.testing.assert_array_equal(o.cpu().numpy(), ref[key])
