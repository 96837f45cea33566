"""Robots with fixed joints through the C ABI on an MI355X, every build, against the FP64
oracle. Reference: the oracle's full model with each fixed joint held at q = qd = qdd = 0 (a
fixed joint is a joint that cannot move): M_r = M[r, r], c_r = RNEA(q, qd, 0)[r],
qdd_r = M_r^-1 (tau_r - c_r), dqdd_r/du_r = -M_r^-1 dtau[r, r]/du_r with dtau from the
oracle's dRNEA at qdd = (qdd_r, 0); r the movable joints. Tolerances as for dFD.
"""
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth
from paper_2109_06976_amd.build import prismatic_models

pytestmark = pytest.mark.gpu

CASES = {
    "chain7-fixed25": lambda: synth.with_fixed_joints(synth.chain7(), [2, 5]),
    "tree7-fixed136": lambda: synth.with_fixed_joints(
        synth.random_model(np.array([-1, 0, 0, 1, 3, -1, 5], np.int32), 77, "tree7"), [1, 3, 6]),
    "chain7-axes-fixed04": lambda: synth.with_fixed_joints(
        synth.random_model(synth.chain_parent(7), 0, "chain7-axes", axes="random"), [0, 4]),
    # prismatic joints 0 and 4, fixed bodies 1 and 3 welded to the prismatic body 0
    "tree7-fixed-prism": lambda: prismatic_models()["tree7-fixed-prism"],
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def locked_reference(orc, robot, q_r, qd_r, tau_r):
    n = robot.n
    r = np.flatnonzero(robot.joint_type != grid.JOINT_FIXED)
    out = {"qdd": [], "Minv": [], "dqdd_dq": [], "dqdd_dqd": []}
    for k in range(q_r.shape[0]):
        q = np.zeros(n)
        qd = np.zeros(n)
        q[r], qd[r] = q_r[k], qd_r[k]
        M = orc.crba(robot, q)[np.ix_(r, r)]
        c = orc.rnea(robot, q, qd, np.zeros(n))[r]
        qdd_r = np.linalg.solve(M, tau_r[k] - c)
        qdd = np.zeros(n)
        qdd[r] = qdd_r
        dq, dqd = orc.rnea_grad(robot, q, qd, qdd)
        Minv = np.linalg.inv(M)
        out["qdd"].append(qdd_r)
        out["Minv"].append(Minv)
        out["dqdd_dq"].append(-Minv @ dq[np.ix_(r, r)])
        out["dqdd_dqd"].append(-Minv @ dqd[np.ix_(r, r)])
    return {k: np.stack(v) for k, v in out.items()}


@pytest.mark.parametrize("name", list(CASES))
def test_fixed_joint_robots_match_locked_oracle(orc, name):
    import torch
    robot = CASES[name]()
    nd = int((robot.joint_type != grid.JOINT_FIXED).sum())
    m = grid.Model(robot)
    try:
        assert m.n == nd
        N = 37
        kn = synth.random_knots(nd, N, 610)
        ref = locked_reference(orc, robot, kn.q.astype(float), kn.qd.astype(float),
                               kn.tau.astype(float))
        for build in range(len(grid.BUILD_KERNELS)):
            grid.tune_apply(m, {1 << 22: build})
            say(f"[gpu] {name} (n_dof={nd}): build {build}, N={N}")
            out = grid.fd_grad_torch(m, *(torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)))
            torch.cuda.synchronize()
            errs = {}
            for k, tol in (("qdd", 1e-4), ("Minv", 1e-3), ("dqdd_dq", 1e-3), ("dqdd_dqd", 1e-3)):
                y = out[k].cpu().numpy().astype(np.float64).reshape(N, -1)
                r = ref[k].reshape(N, -1)
                s = np.abs(r).max(1)
                errs[k] = float((np.abs(y - r).max(1) / np.where(s > 0, s, 1.0)).max())
                assert errs[k] <= tol, (name, build, k, errs[k])
            say("  " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    finally:
        m.close()
