"""Seeded synthetic robot models and knot-point inputs.

This module only draws random numbers and arranges them into arrays. It holds none
of the dynamics arithmetic: no transforms, inertias, recursions or derivatives. Both
the HIP library and the FP64 oracle consume what it returns, so neither has to
reproduce the other's random stream.

Robots are stand-ins for the paper's three workloads (Sec. V-A: a 7-dof serial
manipulator, a 12-dof quadruped, a 30-dof humanoid), whose model files are not
available. Unless asked otherwise, every joint is revolute about its own z axis
(Sec. III-B: S_i is the joint's motion subspace); random unit axes, prismatic joints
(sliding along the axis, q in metres) and fixed joints are options. Per-body parameters:

* parent index lambda_i < i, -1 for the fixed base (Sec. III-B numbering);
* tree rotation E_T (Haar-uniform, from a normalised Gaussian quaternion) and
  joint origin r ~ U[0, 0.4]^3 m, both expressed in the parent frame;
* mass ~ U[0.5, 5] kg, centre of mass c ~ U[-0.1, 0.1]^3 m in the body frame;
* rotational inertia about the centre of mass R diag(d) R^T with R Haar and
  d ~ U[0.01, 0.1]^3 kg m^2, stored as (xx, yy, zz, xy, xz, yz).

Knot inputs: q ~ U[-pi, pi], qd ~ N(0, 1), tau ~ N(0, 5^2) (standard deviation 5).

All model parameters are rounded to float32 and returned as float64, so the FP32
GPU path and the FP64 oracle see bit-identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GRAVITY = (0.0, 0.0, -9.81)

# model seeds and knot seeds used by the workloads
SEED_CHAIN7 = 0
SEED_QUAD12 = 1
SEED_HUMANOID30 = 2

# Batch sizes of the measured workloads (the tests run parity at each of them):
# the paper's multiple-computation sweep (Sec. V-B, Fig. 4) on each of the three robots
SWEEP_KNOTS = (32, 64, 128, 256, 1024)
# larger batches of the 7-dof chain, where the throughput builds take over
THROUGHPUT_KNOTS = (1024, 16384, 32768, 65536)
# larger batches of the quadruped and the humanoid, each on its own tuned build
ROBOT_THROUGHPUT_KNOTS = {"quad12": (16384, 65536), "humanoid30": (4096, 16384)}
# quadruped + 7-dof chain mixes at uneven knot counts in one step
MIXED_PLANS = ((64, 37), (256, 181), (1024, 613))


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class RobotModel:
    name: str
    parent: np.ndarray          # int32 [n]
    E_T: np.ndarray             # float64 [n, 3, 3]
    r: np.ndarray               # float64 [n, 3]
    mass: np.ndarray            # float64 [n]
    com: np.ndarray             # float64 [n, 3]
    Ic: np.ndarray              # float64 [n, 6]  (xx, yy, zz, xy, xz, yz)
    gravity: np.ndarray = field(default_factory=lambda: np.array(GRAVITY))
    base_mass: float | None = None   # mass of a fixed base link (cannot affect outputs)
    axis: np.ndarray | None = None   # float64 [n, 3] unit joint axes (None: every joint +z)
    joint_type: np.ndarray | None = None   # int32 [n]: 0 revolute, 1 prismatic, 2 fixed
                                            # (None: all revolute)

    @property
    def n(self) -> int:
        return int(self.parent.shape[0])

    def copy(self) -> "RobotModel":
        return RobotModel(self.name, self.parent.copy(), self.E_T.copy(), self.r.copy(),
                          self.mass.copy(), self.com.copy(), self.Ic.copy(),
                          self.gravity.copy(), self.base_mass,
                          None if self.axis is None else self.axis.copy(),
                          None if self.joint_type is None else self.joint_type.copy())


# ---------------------------------------------------------------- topologies

def chain_parent(n: int) -> np.ndarray:
    """Serial chain: body i hangs off body i-1, body 0 off the base."""
    return np.arange(-1, n - 1, dtype=np.int32)


def quadruped_parent(legs: int = 4, per_leg: int = 3) -> np.ndarray:
    """Legs of `per_leg` joints, each attached to the fixed torso, numbered leg by leg."""
    p = []
    for leg in range(legs):
        base = leg * per_leg
        p.append(-1)
        p.extend(range(base, base + per_leg - 1))
    return np.asarray(p, dtype=np.int32)


def humanoid_parent(variant: str = "anatomical") -> np.ndarray:
    """30-joint humanoid: torso 2, two legs of 6, head 2, two arms of 7.

    anatomical: torso chain and both legs on the fixed pelvis; head and both arms
    on the second torso link (longest path 9 joints).
    literal: arms, legs and torso on the pelvis; head on the second torso link
    (longest path 7 joints).
    """
    parent: list[int] = []

    def limb(attach: int, length: int) -> int:
        first = len(parent)
        parent.append(attach)
        for k in range(1, length):
            parent.append(first + k - 1)
        return first + length - 1

    torso_end = limb(-1, 2)
    limb(-1, 6)
    limb(-1, 6)
    limb(torso_end, 2)
    arm_attach = torso_end if variant == "anatomical" else -1
    if variant not in ("anatomical", "literal"):
        raise ValueError(variant)
    limb(arm_attach, 7)
    limb(arm_attach, 7)
    assert len(parent) == 30
    return np.asarray(parent, dtype=np.int32)


# ---------------------------------------------------------------- random draws

def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion (Shoemake)."""
    w, x, y, z = rng.standard_normal(4)
    s = np.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / s, x / s, y / s, z / s
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_model(parent, seed: int, name: str = "robot", base_mass: float | None = None,
                 gravity=GRAVITY, axes: str = "z") -> RobotModel:
    """Draw per-body parameters in a fixed order: r, E_T, mass, com, inertia.

    axes: "z" (every joint about its own +z) or "random" (unit axes drawn uniformly on the
    sphere from a second stream seeded by (seed, 1), so the other parameters are the same
    as with "z")."""
    parent = np.asarray(parent, dtype=np.int32)
    n = parent.shape[0]
    for i, p in enumerate(parent):
        if not (-1 <= p < i):
            raise ValueError(f"parent[{i}]={p} must satisfy -1 <= parent[i] < i")
    rng = np.random.default_rng(seed)
    E_T = np.zeros((n, 3, 3))
    r = np.zeros((n, 3))
    mass = np.zeros(n)
    com = np.zeros((n, 3))
    Ic = np.zeros((n, 6))
    for i in range(n):
        r[i] = rng.uniform(0.0, 0.4, 3)
        E_T[i] = _haar_rotation(rng)
        mass[i] = rng.uniform(0.5, 5.0)
        com[i] = rng.uniform(-0.1, 0.1, 3)
        R = _haar_rotation(rng)
        d = rng.uniform(0.01, 0.1, 3)
        J = R @ np.diag(d) @ R.T
        Ic[i] = [J[0, 0], J[1, 1], J[2, 2], J[0, 1], J[0, 2], J[1, 2]]
    axis = None
    if axes == "random":
        arng = np.random.default_rng([seed, 1])
        a = arng.standard_normal((n, 3))
        axis = _f32(a / np.linalg.norm(a, axis=1, keepdims=True))
    elif axes != "z":
        raise ValueError(axes)
    return RobotModel(name, parent, _f32(E_T), _f32(r), _f32(mass), _f32(com), _f32(Ic),
                      _f32(np.asarray(gravity, dtype=np.float64)), base_mass, axis)


def chain7(seed: int = SEED_CHAIN7) -> RobotModel:
    return random_model(chain_parent(7), seed, "chain7")


def quad12(seed: int = SEED_QUAD12) -> RobotModel:
    return random_model(quadruped_parent(), seed, "quad12", base_mass=10.0)


def humanoid30(seed: int = SEED_HUMANOID30, variant: str = "anatomical") -> RobotModel:
    return random_model(humanoid_parent(variant), seed, f"humanoid30-{variant}")


def with_fixed_joints(model: RobotModel, fixed) -> RobotModel:
    """The same bodies with the listed joints fixed (welded to their parents)."""
    m = model.copy()
    jt = np.zeros(m.n, np.int32)
    jt[list(fixed)] = 2
    m.joint_type = jt
    m.name = f"{model.name}-fixed{''.join(str(i) for i in fixed)}"
    return m


def with_prismatic_joints(model: RobotModel, prismatic) -> RobotModel:
    """The same bodies with the listed joints prismatic (sliding along their axes); the
    other joints keep their types."""
    m = model.copy()
    jt = np.zeros(m.n, np.int32) if m.joint_type is None else m.joint_type.copy()
    jt[list(prismatic)] = 1
    m.joint_type = jt
    m.name = f"{model.name}-prism{''.join(str(i) for i in prismatic)}"
    return m


def model_by_name(name: str) -> RobotModel:
    table = {
        "chain7": chain7,
        "quad12": quad12,
        "humanoid30": humanoid30,
        "humanoid30-literal": lambda: humanoid30(variant="literal"),
    }
    return table[name]()


@dataclass
class Knots:
    q: np.ndarray      # float32 [N, n]
    qd: np.ndarray     # float32 [N, n]
    tau: np.ndarray    # float32 [N, n]

    @property
    def N(self) -> int:
        return int(self.q.shape[0])


def random_knots(n: int, N: int, seed: int) -> Knots:
    """q ~ U[-pi, pi], qd ~ N(0, 1), tau ~ N(0, 25); drawn as whole arrays in that order."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(-np.pi, np.pi, (N, n)).astype(np.float32)
    qd = rng.standard_normal((N, n)).astype(np.float32)
    tau = (5.0 * rng.standard_normal((N, n))).astype(np.float32)
    return Knots(q, qd, tau)
