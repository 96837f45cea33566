"""grid_fd_grad_staged_noalloc (the staged pipeline on the library's static scratch array)
against grid_fd_grad_staged (the same five kernels on a workspace the library allocates):
bit for bit, on two calls in a row whose second is smaller, on robots with different per-knot
scratch strides one after the other, and at the largest N the array holds; the limit is
rejected with EINVAL. The small calls are also held to the oracle's tolerances."""
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth

pytestmark = pytest.mark.gpu

OUTS = ("qdd", "Minv", "dqdd_dq", "dqdd_dqd")
TOL = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _buffers(torch, n, N, seed):
    kn = synth.random_knots(n, N, seed)
    ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
    return kn, ins


def _outs(torch, n, N):
    outs = [torch.empty(N, n, device="cuda"), torch.empty(N, n, n, device="cuda"),
            torch.empty(N, n, n, device="cuda"), torch.empty(N, n, n, device="cuda")]
    for t in outs:
        t.fill_(float("nan"))
    return outs


def _max_knots(model):
    """Knots of this model the static array holds (the entry point's limit)."""
    with pytest.raises(grid.GridError) as e:
        model.fd_grad_staged_noalloc(*([0] * 7), N=grid.GRID_MAX_KNOTS)
    assert e.value.status == grid.GRID_EINVAL
    msg = str(e.value)
    return int(msg.split("(at most ")[1].split(" knots")[0])


def _run_pair(torch, name, model, ws, N, seed):
    n = model.n
    kn, ins = _buffers(torch, n, N, seed)
    a = _outs(torch, n, N)
    b = _outs(torch, n, N)
    ws.fd_grad_staged(*ins, *a)
    model.fd_grad_staged_noalloc(*ins, *b)
    torch.cuda.synchronize()
    a = [t.cpu().numpy() for t in a]
    b = [t.cpu().numpy() for t in b]
    for k, x, y in zip(OUTS, a, b):
        assert np.all(np.isfinite(y)), f"{name} N={N} {k}: non-finite outputs"
        np.testing.assert_array_equal(y, x, err_msg=f"{name} N={N} {k}")
    return kn, dict(zip(OUTS, b))


def _oracle_check(orc, robot, kn, got, N):
    ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
    for k in OUTS:
        y = got[k].astype(np.float64).reshape(N, -1)
        w = ref[k].reshape(N, -1)
        err = (np.abs(y - w).max(1) / np.abs(w).max(1)).max()
        assert err <= TOL[k], (robot.name, N, k, err)


def test_noalloc_equals_staged_two_calls(orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    robots = [synth.chain7(), synth.humanoid30(), synth.quad12()]
    plans = [(300, 37), (200, 19), (129, 5)]
    models = [grid.Model(r, device=0) for r in robots]
    try:
        for robot, model, (big, small) in zip(robots, models, plans):
            ws = grid.Workspace(model, big)
            try:
                say(f"[gpu] noalloc vs staged: {robot.name} N={big} then N={small}")
                _run_pair(torch, robot.name, model, ws, big, 500 + big)
                kn, got = _run_pair(torch, robot.name, model, ws, small, 600 + small)
                _oracle_check(orc, robot, kn, got, small)
            finally:
                ws.close()
    finally:
        for m in models:
            m.close()


def test_noalloc_limit():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    robot = synth.humanoid30()
    model = grid.Model(robot, device=0)
    try:
        cap = _max_knots(model)
        say(f"[gpu] noalloc limit: humanoid30 holds {cap} knots")
        assert cap >= 1000
        n = model.n
        kn, ins = _buffers(torch, n, cap + 1, 700)
        outs = _outs(torch, n, cap + 1)
        with pytest.raises(grid.GridError) as e:
            model.fd_grad_staged_noalloc(*ins, *outs)
        assert e.value.status == grid.GRID_EINVAL
        # the largest N the array holds, then a much smaller call, each equal to the staged call
        ws = grid.Workspace(model, cap)
        try:
            say(f"[gpu] noalloc at the limit: N={cap} then N=3")
            _run_pair(torch, robot.name, model, ws, cap, 701)
            _run_pair(torch, robot.name, model, ws, 3, 702)
        finally:
            ws.close()
        # an empty call does nothing and succeeds
        model.fd_grad_staged_noalloc(*ins, *outs, N=0)
    finally:
        model.close()
