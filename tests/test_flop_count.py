"""The instrumented FLOP count of the oracle's formulation (oracle/flop_count.py), on the CPU.

The count replays the oracle's steps on a counting scalar; it is the oracle's formulation
only if the replay computes the oracle's outputs, so that is checked first (bit for bit: same
operations in the same order). Then the counting rules on primitives whose cost is known by
hand, and the stored per-knot counts that the benchmark's roofline reads.
"""
import json
import os

import numpy as np
import pytest

from oracle import flop_count as fc
from paper_2109_06976_amd import synth
from paper_2109_06976_amd.build import prismatic_models

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name", ["chain7", "quad12", "tree5-axes-prism", "chain2"])
def test_replay_computes_the_oracle_outputs(orc, name):
    robot = {"chain7": synth.chain7, "quad12": synth.quad12,
             "tree5-axes-prism": lambda: prismatic_models()["tree5-axes-prism"],
             "chain2": lambda: synth.random_model(synth.chain_parent(2), 41, "chain2")}[name]()
    kn = synth.random_knots(robot.n, 1, 78)
    got, steps = fc.fd_grad_counted(robot, kn.q[0], kn.qd[0], kn.tau[0])
    ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
    for k in ("qdd", "Minv", "dqdd_dq", "dqdd_dqd"):
        np.testing.assert_array_equal(got[k], ref[k][0], err_msg=k)
    assert set(steps) == set(fc.STEPS) and all(v >= 0 for v in steps.values())


def test_counting_rules_on_known_primitives():
    fc._C = fc.Counter()
    fc._C.step = "drnea"
    rng = np.random.default_rng(5)
    A = [fc.Num(x) for x in rng.standard_normal(36)]
    x = [fc.Num(v) for v in rng.standard_normal(6)]
    fc.mv6(A, x)
    assert fc._C.by_step["drnea"] == 66                 # 36 multiplications + 30 additions
    fc._C.by_step["drnea"] = 0
    fc.crm_apply(x, [fc.Num(v) for v in rng.standard_normal(6)])
    assert fc._C.by_step["drnea"] == 30                 # 18 products + 12 sums (Eq. 2's zeros)
    fc._C.by_step["drnea"] = 0
    S = [fc.Num(0.0, True)] * 2 + [fc.Num(1.0, True)] + [fc.Num(0.0, True)] * 3
    fc.crm_apply(x, S)                                  # x cross e_z: selections only
    assert fc._C.by_step["drnea"] == 0
    c1, c2 = fc.Num(2.0, True), fc.Num(3.0, True)
    _ = c1 * c2 + c1                                    # model constants only: precomputable
    assert fc._C.by_step["drnea"] == 0
    _ = x[0] * x[1] + x[2] - x[3] / x[4]
    assert fc._C.by_step["drnea"] == 4


def test_stored_counts_are_reproducible():
    doc = json.load(open(os.path.join(ROOT, "profiles", "flops_per_knot.json")))
    assert doc["robots"] == fc.workload_counts()
    tot = {k: v["total"] for k, v in doc["robots"].items()}
    # the quadruped's legs are decoupled: far less per joint than the coupled chain
    assert tot["quad12"] / 12 < tot["chain7"] / 7 < tot["humanoid30"] / 30
