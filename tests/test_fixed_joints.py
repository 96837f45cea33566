"""Fixed joints: the library merges each body on a fixed joint into its nearest ancestor on a
revolute joint. The generated constants of the reduced robot are checked here against
compositions of the oracle's own 6x6 joint transforms and spatial inertias (a fixed joint is
a revolute joint held at q = 0, whose transform is X_T): the merged body's spatial inertia
is I_o + sum over its fixed descendants of X^T I X, and a child's transform from its new
parent is its own X_T times the fixed chain's. CPU only (code generation, no device).
"""
import re

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth


def _consts(src):
    """Per generated branch: robot bodies and their 24 floats (E_T, r, Ibar, h, m)."""
    out = {}
    for m in re.finditer(r"struct Inst<(\d+)> \{\s*using S = Shape<\d+>;\s*"
                         r"static constexpr int N = \d+;\s*"
                         r"static constexpr int body\[S::B\] = \{([^}]*)\};", src):
        k = int(m.group(1))
        bodies = [int(x) for x in m.group(2).split(",")]
        c = re.search(r"grid_const_%d\[\d+\] = \{([^}]*)\}" % k, src)
        vals = np.array([float.fromhex(x.strip().rstrip("f")) for x in c.group(1).split(",")])
        for b, i in enumerate(bodies):
            out[i] = vals[24 * b:24 * b + 24]
    return out


def _spatial(v):
    """Spatial inertia about the body origin from (Ibar, h, m)."""
    Ib = np.array([[v[12], v[15], v[16]], [v[15], v[13], v[17]], [v[16], v[17], v[14]]])
    h = v[18:21]
    hx = np.array([[0, -h[2], h[1]], [h[2], 0, -h[0]], [-h[1], h[0], 0]])
    return np.block([[Ib, hx], [hx.T, v[21] * np.eye(3)]])


def _xt(v):
    E = v[0:9].reshape(3, 3)
    r = v[9:12]
    rx = np.array([[0, -r[2], r[1]], [r[2], 0, -r[0]], [-r[1], r[0], 0]])
    return np.block([[E, np.zeros((3, 3))], [-E @ rx, E]])


@pytest.mark.parametrize("parent,fixed", [
    ([-1, 0, 1, 2, 3, 4, 5], [2, 5]),          # chain with two welded links
    ([-1, 0, 1, 2, 3, 4, 5], [0]),             # first link welded to the base
    ([-1, 0, 0, 1, 3, -1, 5], [1, 3, 6]),      # welded chain of two, a welded leaf, a second root
])
def test_reduced_constants_match_oracle_compositions(orc, parent, fixed):
    robot = synth.with_fixed_joints(
        synth.random_model(np.array(parent, np.int32), 77, "t"), fixed)
    n = robot.n
    movable = [i for i in range(n) if i not in fixed]
    src = grid.codegen_source(robot)
    assert f"static constexpr int N = {len(movable)};\n" in src
    consts = _consts(src)
    assert sorted(consts) == list(range(len(movable)))
    X0 = [orc.joint_transform(robot, i, 0.0) for i in range(n)]   # X_T: fixed joints at 0
    Ibody = [orc.spatial_inertia(robot, i) for i in range(n)]
    owner, chain = {}, {}                      # chain[i]: owner frame -> body frame i
    for i in range(n):
        p = parent[i]
        up = np.eye(6) if p < 0 else chain[p]
        if i in fixed:
            owner[i] = -1 if p < 0 else owner[p]
            chain[i] = X0[i] @ up
        else:
            owner[i] = i
            chain[i] = np.eye(6)
            k = movable.index(i)
            # this joint's X_T from the new parent's frame: X_T,i composed with the chain
            np.testing.assert_allclose(_xt(consts[k]), X0[i] @ up, rtol=2e-6, atol=2e-6)
    for i in movable:
        want = Ibody[i].copy()
        for f in fixed:
            if owner[f] == i:
                want += chain[f].T @ Ibody[f] @ chain[f]
        np.testing.assert_allclose(_spatial(consts[movable.index(i)]), want, rtol=2e-6,
                                   atol=2e-6)


def test_joint_type_errors():
    robot = synth.chain7()
    with pytest.raises(grid.GridError) as e:
        grid.codegen_source(synth.with_fixed_joints(robot, range(7)))
    assert e.value.status == grid.GRID_EINVAL
    bad = robot.copy()
    bad.joint_type = np.full(7, 9, np.int32)
    with pytest.raises(grid.GridError) as e:
        grid.codegen_source(bad)
    assert e.value.status == grid.GRID_EINVAL


def test_prismatic_joints_marked_per_branch():
    """The generated kernel marks each branch's prismatic bodies in local numbering: tree7
    reduces to branches (0, 2, 4) and (5) of the original bodies; 0 and 4 slide."""
    from paper_2109_06976_amd.build import prismatic_models
    robot = prismatic_models()["tree7-fixed-prism"]
    assert list(robot.joint_type) == [1, 2, 0, 2, 1, 0, 2]
    src = grid.codegen_source(robot)
    assert "static constexpr unsigned long long prism = 5ull;" in src      # local 0 and 2
    assert "static constexpr unsigned long long prism = 0ull;" in src
    m = grid.codegen_source(prismatic_models()["chain7-prism"])
    assert "static constexpr unsigned long long prism = 18ull;" in m       # joints 1 and 4
    assert "prism = 0ull;" in grid.codegen_source(synth.chain7())
