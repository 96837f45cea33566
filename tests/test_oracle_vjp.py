"""The reverse-mode product of forward dynamics, pinned on the CPU.

For L = sum_k ||qdd_k||^2 with qdd_k = FD(q_k, qd_k, tau_k), the gradient with respect to
each knot's inputs is (dqdd/du)^T (2 qdd) for u = q, qd and M^-1 (2 qdd) for tau. The
oracle's Jacobians, transposed this way, must equal central differences (h = 1e-6, FP64)
of the oracle's own FD through L.
"""
import numpy as np

from paper_2109_06976_amd import synth


def _loss(orc, robot, q, qd, tau):
    return float(sum(np.sum(orc.fd(robot, q[k], qd[k], tau[k]) ** 2) for k in range(q.shape[0])))


def test_vjp_matches_central_differences(orc):
    robot = synth.humanoid30()
    kn = synth.random_knots(robot.n, 2, 104)
    q, qd, tau = (a.astype(np.float64) for a in (kn.q, kn.qd, kn.tau))
    out = orc.fd_grad_batch(robot, q, qd, tau)
    g = 2.0 * out["qdd"]
    qbar = np.einsum("kij,ki->kj", out["dqdd_dq"], g)
    qdbar = np.einsum("kij,ki->kj", out["dqdd_dqd"], g)
    taubar = np.einsum("kij,ki->kj", out["Minv"], g)
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(8):
        k, j = int(rng.integers(2)), int(rng.integers(robot.n))
        for arr, bar in ((q, qbar), (qd, qdbar), (tau, taubar)):
            plus, minus = arr.copy(), arr.copy()
            plus[k, j] += h
            minus[k, j] -= h
            args_p = [plus if a is arr else a for a in (q, qd, tau)]
            args_m = [minus if a is arr else a for a in (q, qd, tau)]
            cd = (_loss(orc, robot, *args_p) - _loss(orc, robot, *args_m)) / (2 * h)
            assert abs(cd - bar[k, j]) <= 1e-6 * max(1.0, np.abs(bar).max())
