"""The paper's other algorithms (ID, FD, M^-1, dID) through the C ABI on an MI355X, against
the FP64 oracle's own RNEA, Cholesky M^-1, FD and analytic dRNEA.

Tolerances are those of the dFD parity tests (normwise per knot: vectors 1e-4, matrices
1e-3). qdd inputs for ID and dID are drawn like tau: N(0, 5^2). Knot counts 1, 37, 130 leave
ragged workgroups for every packing; dID outputs rows of other branches as exact zeros.
"""
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth
from paper_2109_06976_amd.build import max_size_model, prismatic_models

pytestmark = pytest.mark.gpu

ROBOTS = {
    "chain7": synth.chain7,
    "quad12": synth.quad12,
    "humanoid30": synth.humanoid30,
    "chain1": lambda: synth.random_model(synth.chain_parent(1), 40, "chain1"),
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
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _roots(parent):
    root = np.zeros(len(parent), np.int64)
    for i, p in enumerate(parent):
        root[i] = i if p < 0 else root[p]
    return root


def normwise(y, ref):
    N = ref.shape[0]
    d = np.abs(y.astype(np.float64) - ref).reshape(N, -1).max(axis=1)
    s = np.abs(ref).reshape(N, -1).max(axis=1)
    return d / np.where(s > 0, s, 1.0)


@pytest.mark.parametrize("name", list(ROBOTS))
def test_ops_match_oracle(orc, name):
    import torch
    robot = ROBOTS[name]()
    n = robot.n
    m = grid.Model(robot)
    try:
        for N in (1, 37, 130):
            kn = synth.random_knots(n, N, 700 + N)
            qdd_in = synth.random_knots(n, N, 800 + N).tau
            dev = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau, qdd_in)]
            q, qd, tau, qdd = dev
            out_tau = torch.full((N, n), float("nan"), device="cuda")
            out_qdd = torch.full((N, n), float("nan"), device="cuda")
            out_mi = torch.full((N, n, n), float("nan"), device="cuda")
            out_dq = torch.full((N, n, n), float("nan"), device="cuda")
            out_dqd = torch.full((N, n, n), float("nan"), device="cuda")
            say(f"[gpu] {name}: ID, FD, M^-1, dID at N={N}")
            m.id(q, qd, qdd, out_tau)
            m.fd(q, qd, tau, out_qdd)
            m.minv(q, out_mi)
            m.id_grad(q, qd, qdd, out_dq, out_dqd)
            torch.cuda.synchronize()
            r_tau = np.stack([orc.rnea(robot, kn.q[k], kn.qd[k], qdd_in[k]) for k in range(N)])
            r_qdd = np.stack([orc.fd(robot, kn.q[k], kn.qd[k], kn.tau[k]) for k in range(N)])
            r_mi = np.stack([orc.minv_cholesky(robot, kn.q[k]) for k in range(N)])
            grads = [orc.rnea_grad(robot, kn.q[k], kn.qd[k], qdd_in[k]) for k in range(N)]
            r_dq = np.stack([g[0] for g in grads])
            r_dqd = np.stack([g[1] for g in grads])
            errs = {"tau": normwise(out_tau.cpu().numpy(), r_tau).max(),
                    "qdd": normwise(out_qdd.cpu().numpy(), r_qdd).max(),
                    "Minv": normwise(out_mi.cpu().numpy(), r_mi).max(),
                    "dtau_dq": normwise(out_dq.cpu().numpy(), r_dq).max(),
                    "dtau_dqd": normwise(out_dqd.cpu().numpy(), r_dqd).max()}
            say("  " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()))
            for k, tol in (("tau", 1e-4), ("qdd", 1e-4), ("Minv", 1e-3), ("dtau_dq", 1e-3),
                           ("dtau_dqd", 1e-3)):
                assert errs[k] <= tol, (name, N, k)
            mi = out_mi.cpu().numpy()
            np.testing.assert_array_equal(mi, np.swapaxes(mi, 1, 2))
            # entries coupling different base branches are exact zeros (other zeros of the
            # oracle, such as d tau_leaf / d qd_leaf, vanish by cancellation, not structure)
            root = _roots(robot.parent)
            cross = root[:, None] != root[None, :]
            for got in (mi, out_dq.cpu().numpy(), out_dqd.cpu().numpy()):
                assert np.all(got[:, cross] == 0.0)
    finally:
        m.close()


@pytest.mark.parametrize("name", list(ROBOTS))
def test_minv_routes_match_oracle(orc, name):
    """grid_minv_route: the one-lane-per-knot routes (composite bodies with the L^T L factor,
    and the paper's direct articulated-body inverse) against the oracle's Cholesky M^-1 and
    its direct recursion, at knot counts that leave ragged 64-knot workgroups; the quad route
    is grid_minv itself (bit for bit); all three exactly symmetric with exact zeros between
    base branches."""
    import torch
    robot = ROBOTS[name]()
    n = robot.n
    m = grid.Model(robot)
    root = _roots(robot.parent)
    cross = root[:, None] != root[None, :]
    try:
        for N in (1, 65, 130):
            kn = synth.random_knots(n, N, 900 + N)
            q = torch.from_numpy(kn.q).cuda()
            r_chol = np.stack([orc.minv_cholesky(robot, kn.q[k]) for k in range(N)])
            r_dir = np.stack([orc.minv_direct(robot, kn.q[k]) for k in range(N)])
            say(f"[gpu] {name}: M^-1 routes at N={N}")
            plain = torch.full((N, n, n), float("nan"), device="cuda")
            m.minv(q, plain)
            for route in (grid.MINV_QUAD, grid.MINV_LANE_LTL, grid.MINV_LANE_DIRECT):
                out = torch.full((N, n, n), float("nan"), device="cuda")
                m.minv_route(q, out, route)
                torch.cuda.synchronize()
                got = out.cpu().numpy()
                e1 = normwise(got, r_chol).max()
                e2 = normwise(got, r_dir).max()
                say(f"  route {route}: vs Cholesky {e1:.1e}, vs direct {e2:.1e}")
                assert e1 <= 1e-3 and e2 <= 1e-3, (name, N, route)
                np.testing.assert_array_equal(got, np.swapaxes(got, 1, 2))
                assert np.all(got[:, cross] == 0.0)
                if route == grid.MINV_QUAD:
                    np.testing.assert_array_equal(got, plain.cpu().numpy())
        with pytest.raises(grid.GridError) as e:
            m.minv_route(q, plain, 3)
        assert e.value.status == grid.GRID_EINVAL
        m.minv_route(q, plain, grid.MINV_LANE_DIRECT, N=0)   # N = 0 is a no-op
    finally:
        m.close()


@pytest.mark.parametrize("name", ["chain7", "quad12", "humanoid30"])
def test_minv_routes_at_bench_sizes(orc, name):
    """The M^-1 routes at the largest knot count the benchmark times them at (65536): a seeded
    sample of knots, the first and last included, against the oracle's Cholesky inverse; every
    knot exactly symmetric."""
    import torch
    robot = ROBOTS[name]()
    n = robot.n
    N = 65536
    m = grid.Model(robot)
    try:
        kn = synth.random_knots(n, N, 950)
        q = torch.from_numpy(kn.q).cuda()
        pick = np.unique(np.concatenate([[0, N - 1], np.random.default_rng(951).integers(0, N, 62)]))
        ref = np.stack([orc.minv_cholesky(robot, kn.q[k]) for k in pick])
        for route in (grid.MINV_QUAD, grid.MINV_LANE_LTL, grid.MINV_LANE_DIRECT):
            say(f"[gpu] {name}: M^-1 route {route} at N={N}")
            out = torch.full((N, n, n), float("nan"), device="cuda")
            m.minv_route(q, out, route)
            torch.cuda.synchronize()
            assert bool(torch.equal(out, out.transpose(1, 2)))
            got = out[torch.from_numpy(pick).cuda()].cpu().numpy()
            assert normwise(got, ref).max() <= 1e-3, (name, route)
            del out
    finally:
        m.close()


def test_ops_reject_bad_arguments():
    import torch
    m = grid.Model(synth.chain7())
    t = torch.zeros((4, 7), device="cuda")
    try:
        with pytest.raises(grid.GridError) as e:
            m.id(t, None, t, t, N=4)
        assert e.value.status == grid.GRID_EINVAL
        with pytest.raises(grid.GridError) as e:
            m.fd(t, t, t, t, N=-1)
        assert e.value.status == grid.GRID_EINVAL
        m.minv(t, t, N=0)     # N = 0 is a no-op
    finally:
        m.close()


@pytest.mark.parametrize("name", ["chain7", "humanoid30", "tree5-axes"])
def test_dt_jacobians_match_central_differences_of_the_oracle_step(orc, name):
    # A, B of one semi-implicit Euler step from the GPU's dFD, against central differences
    # of the step computed with the oracle's forward dynamics (FP64)
    import torch
    robot = ROBOTS[name]()
    n = robot.n
    N, dt, h = 5, 0.02, 1e-6
    m = grid.Model(robot)
    try:
        kn = synth.random_knots(n, N, 901)
        out = grid.fd_grad_torch(m, *(torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)))
        A = torch.full((N, 2 * n, 2 * n), float("nan"), device="cuda")
        B = torch.full((N, 2 * n, n), float("nan"), device="cuda")
        say(f"[gpu] {name}: discrete-time Jacobians, N={N}, dt={dt}")
        grid.dt_jacobians(m, dt, out["dqdd_dq"], out["dqdd_dqd"], out["Minv"], A, B)
        torch.cuda.synchronize()
        A, B = A.cpu().numpy().astype(np.float64), B.cpu().numpy().astype(np.float64)

        def step(q, qd, tau):
            qd1 = qd + dt * orc.fd(robot, q, qd, tau)
            return np.concatenate([q + dt * qd1, qd1])

        for k in range(N):
            q, qd, tau = (a[k].astype(float) for a in (kn.q, kn.qd, kn.tau))
            x = np.concatenate([q, qd])
            Afd = np.stack([(step(*np.split(x + h * e, 2), tau) - step(*np.split(x - h * e, 2), tau))
                            / (2 * h) for e in np.eye(2 * n)], axis=1)
            Bfd = np.stack([(step(q, qd, tau + h * e) - step(q, qd, tau - h * e)) / (2 * h)
                            for e in np.eye(n)], axis=1)
            # the step's Jacobians are 1 + O(dt): compare their dynamic parts normwise
            eA = np.abs(A[k] - Afd).max() / np.abs(Afd - np.eye(2 * n)).max()
            eB = np.abs(B[k] - Bfd).max() / np.abs(Bfd).max()
            assert eA <= 1e-3 and eB <= 1e-3, (name, k, eA, eB)
        with pytest.raises(grid.GridError) as e:
            grid.dt_jacobians(m, 0.0, out["dqdd_dq"], out["dqdd_dqd"], out["Minv"], A=None, B=None,
                              N=N)
        assert e.value.status == grid.GRID_EINVAL
    finally:
        m.close()


@pytest.mark.parametrize("name", list(ROBOTS))
def test_vjp_adjoint_matches_oracle(orc, name):
    # the reverse-sweep VJP from (q, qd, qdd) against the oracle's dense dFD products
    import torch
    robot = ROBOTS[name]()
    n, N = robot.n, 37
    m = grid.Model(robot)
    try:
        kn = synth.random_knots(n, N, 950)
        gbar = np.random.default_rng(951).standard_normal((N, n)).astype(np.float32)
        ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
        q, qd, qdd, g = (torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
                         for a in (kn.q, kn.qd, ref["qdd"], gbar))
        outs = [torch.full((N, n), float("nan"), device="cuda") for _ in range(3)]
        say(f"[gpu] {name}: adjoint VJP, N={N}")
        grid.fd_vjp_adjoint(m, q, qd, qdd, g, *outs)
        torch.cuda.synchronize()
        want = {"q": np.einsum("kij,ki->kj", ref["dqdd_dq"], gbar),
                "qd": np.einsum("kij,ki->kj", ref["dqdd_dqd"], gbar),
                "tau": np.einsum("kij,ki->kj", ref["Minv"], gbar)}
        for k, got in zip(("q", "qd", "tau"), outs):
            e = normwise(got.cpu().numpy(), want[k]).max()
            say(f"  {k}bar {e:.1e}")
            assert e <= 1e-3, (name, k, e)
    finally:
        m.close()
