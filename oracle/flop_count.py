"""Instrumented FLOP count of the oracle's formulation (test infrastructure only).

The algorithmic work per knot used for roofline fractions is counted on the oracle's own
formulation, not on a kernel's. This module replays the oracle's steps for one knot --
transforms X_i(q_i) (Sec. III-B), RNEA for c = RNEA(q, qd, 0) (Sec. IV-B), CRBA for M,
Cholesky M = L L^T, qdd = M^-1 (tau - c) and the n columns of M^-1 by triangular solves,
RNEA at qdd, the analytic dRNEA of Algorithm 1 with its backward pass, and
dqdd/du = -M^-1 dtau/du (Sec. IV-B) -- with the same dense 6x6 primitives and loop order as
oracle/rbd_generic.inc and oracle/grid_oracle.c, on a scalar that counts its arithmetic:

* a multiplication costs 1 unless an operand is exactly 0 or +-1 (a structural zero, or the
  revolute-z selection of S_i, whose products are free);
* an addition or subtraction costs 1 unless an operand is exactly 0;
* a division costs 1 unless the numerator is 0 or the denominator +-1;
* operations whose operands all derive from model constants only (E_T, r, inertias, axes,
  gravity) are free: they can be precomputed once per robot;
* sin, cos and sqrt are not counted (transcendentals), negation is free.

So a fused multiply-add counts 2, and exact zeros that the robot's structure produces (zero
blocks of X, non-ancestor columns of dRNEA, the block-diagonal M^-1 of a tree) cost nothing.
Each quantity is computed once per knot (the C oracle rebuilds X in every routine and
factors M twice; those repeats are not the algorithm's work).

The replay's outputs are checked against the C oracle in tests/test_flop_count.py, so the
count belongs to the oracle's formulation. `python -m oracle.flop_count --write PATH` writes
the per-knot counts of the three workload robots as JSON.
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np

STEPS = ("transforms", "rnea_bias", "crba", "factor_and_minv", "qdd", "rnea_at_qdd", "drnea",
         "product")


class Counter:
    def __init__(self):
        self.by_step = {k: 0 for k in STEPS}
        self.step = None

    def tick(self, k=1):
        self.by_step[self.step] += k


_C = Counter()


class Num:
    """A float that counts the arithmetic done on it (see the module docstring)."""
    __slots__ = ("v", "c")

    def __init__(self, v, const=False):
        self.v = float(v)
        self.c = const

    @staticmethod
    def of(x):
        return x if isinstance(x, Num) else Num(x, True)

    def __add__(self, o):
        o = Num.of(o)
        if not (self.c and o.c) and self.v != 0.0 and o.v != 0.0:
            _C.tick()
        return Num(self.v + o.v, self.c and o.c)

    __radd__ = __add__

    def __sub__(self, o):
        o = Num.of(o)
        if not (self.c and o.c) and self.v != 0.0 and o.v != 0.0:
            _C.tick()
        return Num(self.v - o.v, self.c and o.c)

    def __rsub__(self, o):
        return Num.of(o) - self

    def __mul__(self, o):
        o = Num.of(o)
        if not (self.c and o.c) and abs(self.v) not in (0.0, 1.0) and abs(o.v) not in (0.0, 1.0):
            _C.tick()
        return Num(self.v * o.v, self.c and o.c)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = Num.of(o)
        if not (self.c and o.c) and self.v != 0.0 and abs(o.v) != 1.0:
            _C.tick()
        return Num(self.v / o.v, self.c and o.c)

    def __neg__(self):
        return Num(-self.v, self.c)

    def __float__(self):
        return self.v


def nsin(x):
    x = Num.of(x)
    return Num(math.sin(x.v), x.c)


def ncos(x):
    x = Num.of(x)
    return Num(math.cos(x.v), x.c)


def nsqrt(x):
    x = Num.of(x)
    return Num(math.sqrt(x.v), x.c)


def Z():
    return Num(0.0, True)


# ------------------------------------------------------------------ primitives (as the oracle)

def mv6(A, x):
    out = []
    for r in range(6):
        s = Z()
        for c in range(6):
            s = s + A[r * 6 + c] * x[c]
        out.append(s)
    return out


def mtv6(A, x):
    out = []
    for c in range(6):
        s = Z()
        for r in range(6):
            s = s + A[r * 6 + c] * x[r]
        out.append(s)
    return out


def mm6(A, B):
    C = []
    for r in range(6):
        for c in range(6):
            s = Z()
            for k in range(6):
                s = s + A[r * 6 + k] * B[k * 6 + c]
            C.append(s)
    return C


def crm(v):
    m = [Z() for _ in range(36)]
    m[0 * 6 + 1] = -v[2]; m[0 * 6 + 2] = v[1]
    m[1 * 6 + 0] = v[2]; m[1 * 6 + 2] = -v[0]
    m[2 * 6 + 0] = -v[1]; m[2 * 6 + 1] = v[0]
    m[3 * 6 + 1] = -v[5]; m[3 * 6 + 2] = v[4]; m[3 * 6 + 4] = -v[2]; m[3 * 6 + 5] = v[1]
    m[4 * 6 + 0] = v[5]; m[4 * 6 + 2] = -v[3]; m[4 * 6 + 3] = v[2]; m[4 * 6 + 5] = -v[0]
    m[5 * 6 + 0] = -v[4]; m[5 * 6 + 1] = v[3]; m[5 * 6 + 3] = -v[1]; m[5 * 6 + 4] = v[0]
    return m


def crf(v):
    c = crm(v)
    return [-c[k * 6 + r] for r in range(6) for k in range(6)]


def crm_apply(v, w):
    return mv6(crm(v), w)


def crf_apply(v, w):
    return mv6(crf(v), w)


def skew3(x):
    return [Z(), -x[2], x[1], x[2], Z(), -x[0], -x[1], x[0], Z()]


# ------------------------------------------------------------------ model pieces

def joint_axis(model, i):
    ax = getattr(model, "axis", None)
    if ax is None:
        return [0.0, 0.0, 1.0]
    a = np.asarray(ax, np.float64).reshape(-1, 3)[i]
    return list(a / np.linalg.norm(a))


def is_prismatic(model, i):
    jt = getattr(model, "joint_type", None)
    return jt is not None and int(np.asarray(jt)[i]) == 1


def joint_S(model, i):
    ax = joint_axis(model, i)
    lin = 3 if is_prismatic(model, i) else 0
    S = [Z() for _ in range(6)]
    for k in range(3):
        S[lin + k] = Num(ax[k], True)
    return S


def xform(model, i, q):
    ET = [Num(x, True) for x in np.asarray(model.E_T, np.float64).reshape(-1, 9)[i]]
    rv = [Num(x, True) for x in np.asarray(model.r, np.float64).reshape(-1, 3)[i]]
    ax = joint_axis(model, i)
    if is_prismatic(model, i):
        d = [q * ax[0], q * ax[1], q * ax[2]]
        rx, dx = skew3(rv), skew3(d)
        XT = [Z() for _ in range(36)]
        XJ = [Z() for _ in range(36)]
        for a in range(3):
            XJ[a * 6 + a] = Num(1.0, True)
            XJ[(a + 3) * 6 + (a + 3)] = Num(1.0, True)
            for b in range(3):
                XJ[(a + 3) * 6 + b] = -dx[a * 3 + b]
                XT[a * 6 + b] = ET[a * 3 + b]
                XT[(a + 3) * 6 + (b + 3)] = ET[a * 3 + b]
                acc = Z()
                for k in range(3):
                    acc = acc + ET[a * 3 + k] * rx[k * 3 + b]
                XT[(a + 3) * 6 + b] = -acc
        return mm6(XJ, XT)
    c, s = ncos(q), nsin(q)
    ak = skew3([Num(x, True) for x in ax])
    EJ = []
    for a in range(3):
        for b in range(3):
            EJ.append((c if a == b else Z()) - s * ak[a * 3 + b]
                      + (1 - c) * Num(ax[a], True) * Num(ax[b], True))
    E = []
    for a in range(3):
        for b in range(3):
            acc = Z()
            for k in range(3):
                acc = acc + EJ[a * 3 + k] * ET[k * 3 + b]
            E.append(acc)
    rx = skew3(rv)
    X = [Z() for _ in range(36)]
    for a in range(3):
        for b in range(3):
            X[a * 6 + b] = E[a * 3 + b]
            X[(a + 3) * 6 + (b + 3)] = E[a * 3 + b]
            acc = Z()
            for k in range(3):
                acc = acc + E[a * 3 + k] * rx[k * 3 + b]
            X[(a + 3) * 6 + b] = -acc
    return X


def inertia(model, i):
    ic = np.asarray(model.Ic, np.float64).reshape(-1, 6)[i]
    cv = np.asarray(model.com, np.float64).reshape(-1, 3)[i]
    mass = Num(np.asarray(model.mass, np.float64).reshape(-1)[i], True)
    cx = skew3([Num(x, True) for x in cv])
    J = [Num(x, True) for x in (ic[0], ic[3], ic[4], ic[3], ic[1], ic[5], ic[4], ic[5], ic[2])]
    Ib = [Z() for _ in range(36)]
    for a in range(3):
        for b in range(3):
            ccT = Z()
            for k in range(3):
                ccT = ccT + cx[a * 3 + k] * cx[b * 3 + k]
            Ib[a * 6 + b] = J[a * 3 + b] + mass * ccT
            Ib[a * 6 + (b + 3)] = mass * cx[a * 3 + b]
            Ib[(a + 3) * 6 + b] = mass * cx[b * 3 + a]
            Ib[(a + 3) * 6 + (b + 3)] = mass if a == b else Z()
    return Ib


# ------------------------------------------------------------------ the oracle's steps

def rnea(model, X, Ib, S, qd, qdd, gravity_on=True):
    """tau, v, a, f (f accumulated), as the oracle's RNEA."""
    n = len(X)
    g = np.asarray(model.gravity, np.float64).reshape(3)
    a0 = [Z(), Z(), Z()] + [Num(-g[k], True) for k in range(3)] if gravity_on \
        else [Z() for _ in range(6)]
    zero6 = [Z() for _ in range(6)]
    v, a, f = [None] * n, [None] * n, [None] * n
    for i in range(n):
        p = int(model.parent[i])
        vp = zero6 if p < 0 else v[p]
        ap = a0 if p < 0 else a[p]
        v[i] = [x + S[i][k] * qd[i] for k, x in enumerate(mv6(X[i], vp))]
        t = mv6(X[i], ap)
        vxS = crm_apply(v[i], S[i])
        a[i] = [t[k] + S[i][k] * qdd[i] + vxS[k] * qd[i] for k in range(6)]
        t = mv6(Ib[i], a[i])
        w = crf_apply(v[i], mv6(Ib[i], v[i]))
        f[i] = [t[k] + w[k] for k in range(6)]
    tau = [None] * n
    for i in range(n - 1, -1, -1):
        p = int(model.parent[i])
        s = Z()
        for k in range(6):
            s = s + S[i][k] * f[i][k]
        tau[i] = s
        if p >= 0:
            t = mtv6(X[i], f[i])
            f[p] = [f[p][k] + t[k] for k in range(6)]
    return tau, v, a, f


def crba(model, X, Ib, S):
    n = len(X)
    IC = [list(x) for x in Ib]
    for i in range(n - 1, -1, -1):
        p = int(model.parent[i])
        if p >= 0:
            t = mm6(IC[i], X[i])
            u = []                                  # X^T t, as the oracle's mtm6
            for r in range(6):
                for c in range(6):
                    s = Z()
                    for k in range(6):
                        s = s + X[i][k * 6 + r] * t[k * 6 + c]
                    u.append(s)
            IC[p] = [IC[p][k] + u[k] for k in range(36)]
    M = [[Z() for _ in range(n)] for _ in range(n)]
    for i in range(n):
        F = mv6(IC[i], S[i])
        d = Z()
        for k in range(6):
            d = d + S[i][k] * F[k]
        M[i][i] = d
        j = i
        while int(model.parent[j]) >= 0:
            F = mtv6(X[j], F)
            j = int(model.parent[j])
            e = Z()
            for k in range(6):
                e = e + S[j][k] * F[k]
            M[i][j] = e
            M[j][i] = e
    return M


def cholesky(M):
    n = len(M)
    L = [[Z() for _ in range(n)] for _ in range(n)]
    for j in range(n):
        s = M[j][j]
        for k in range(j):
            s = s - L[j][k] * L[j][k]
        L[j][j] = nsqrt(s)
        for i in range(j + 1, n):
            t = M[i][j]
            for k in range(j):
                t = t - L[i][k] * L[j][k]
            L[i][j] = t / L[j][j]
    return L


def chol_solve(L, b):
    n = len(L)
    x = [None] * n
    for i in range(n):
        s = b[i]
        for k in range(i):
            s = s - L[i][k] * x[k]
        x[i] = s / L[i][i]
    for i in range(n - 1, -1, -1):
        s = x[i]
        for k in range(i + 1, n):
            s = s - L[k][i] * x[k]
        x[i] = s / L[i][i]
    return x


def rnea_grad(model, X, Ib, S, qd, v, a, f):
    n = len(X)
    g = np.asarray(model.gravity, np.float64).reshape(3)
    a0 = [Z(), Z(), Z()] + [Num(-g[k], True) for k in range(3)]
    zero6 = [Z() for _ in range(6)]
    out = []
    for u in range(2):
        D = [[None] * n for _ in range(n)]
        for j in range(n):
            dv, da, df = [None] * n, [None] * n, [None] * n
            for i in range(n):
                p = int(model.parent[i])
                dvp = zero6 if p < 0 else dv[p]
                dap = zero6 if p < 0 else da[p]
                vp = zero6 if p < 0 else v[p]
                ap = a0 if p < 0 else a[p]
                dv[i] = mv6(X[i], dvp)
                if i == j:
                    s = crm_apply(mv6(X[i], vp), S[i]) if u == 0 else list(S[i])
                    dv[i] = [dv[i][k] + s[k] for k in range(6)]
                da[i] = mv6(X[i], dap)
                s = crm_apply(dv[i], S[i])
                da[i] = [da[i][k] + s[k] * qd[i] for k in range(6)]
                if i == j:
                    s = crm_apply(mv6(X[i], ap), S[i]) if u == 0 else crm_apply(v[i], S[i])
                    da[i] = [da[i][k] + s[k] for k in range(6)]
                df[i] = mv6(Ib[i], da[i])
                w = crf_apply(dv[i], mv6(Ib[i], v[i]))
                df[i] = [df[i][k] + w[k] for k in range(6)]
                w = crf_apply(v[i], mv6(Ib[i], dv[i]))
                df[i] = [df[i][k] + w[k] for k in range(6)]
            for i in range(n - 1, -1, -1):
                p = int(model.parent[i])
                s_ = Z()
                for k in range(6):
                    s_ = s_ + S[i][k] * df[i][k]
                D[i][j] = s_
                if p >= 0:
                    t = mtv6(X[i], df[i])
                    df[p] = [df[p][k] + t[k] for k in range(6)]
                    if u == 0 and i == j:
                        t = mtv6(X[i], crf_apply(S[i], f[i]))
                        df[p] = [df[p][k] + t[k] for k in range(6)]
        out.append(D)
    return out


def fd_grad_counted(model, q, qd, tau):
    """One knot of the path on counting scalars: (outputs as float arrays, FLOPs by step)."""
    global _C
    _C = Counter()
    n = len(model.parent)
    q = [Num(x) for x in np.asarray(q, np.float64)]
    qd = [Num(x) for x in np.asarray(qd, np.float64)]
    tau = [Num(x) for x in np.asarray(tau, np.float64)]
    _C.step = "transforms"
    X = [xform(model, i, q[i]) for i in range(n)]
    Ib = [inertia(model, i) for i in range(n)]        # model constants: free
    S = [joint_S(model, i) for i in range(n)]
    _C.step = "rnea_bias"
    c, _, _, _ = rnea(model, X, Ib, S, qd, [Z() for _ in range(n)])
    _C.step = "crba"
    M = crba(model, X, Ib, S)
    _C.step = "factor_and_minv"
    L = cholesky(M)
    cols = []
    for k in range(n):
        e = [Num(1.0 if i == k else 0.0, True) for i in range(n)]
        cols.append(chol_solve(L, e))
    Minv = [[cols[j][i] for j in range(n)] for i in range(n)]
    _C.step = "qdd"
    qdd = chol_solve(L, [tau[i] - c[i] for i in range(n)])
    _C.step = "rnea_at_qdd"
    _, v, a, f = rnea(model, X, Ib, S, qd, qdd)
    _C.step = "drnea"
    Dq, Dqd = rnea_grad(model, X, Ib, S, qd, v, a, f)
    _C.step = "product"
    outs = []
    for D in (Dq, Dqd):
        R = [[None] * n for _ in range(n)]
        for i in range(n):
            for j in range(n):
                s = Z()
                for k in range(n):
                    s = s + Minv[i][k] * D[k][j]
                R[i][j] = -s
        outs.append(R)
    f64 = lambda m: np.array([[float(x) for x in row] for row in m])
    result = {"qdd": np.array([float(x) for x in qdd]), "Minv": f64(Minv),
              "dqdd_dq": f64(outs[0]), "dqdd_dqd": f64(outs[1])}
    return result, dict(_C.by_step)


def workload_counts():
    """Per-knot FLOPs of the three workload robots (one seeded knot each)."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from paper_2109_06976_amd import synth
    out = {}
    for name in ("chain7", "quad12", "humanoid30"):
        robot = synth.model_by_name(name)
        kn = synth.random_knots(robot.n, 1, 77)
        _, steps = fd_grad_counted(robot, kn.q[0], kn.qd[0], kn.tau[0])
        out[name] = {"total": sum(steps.values()), "by_step": steps,
                     "io_bytes": 4 * (4 * robot.n + 3 * robot.n * robot.n)}
    return out


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--write":
        counts = workload_counts()
        doc = {"what": "FLOPs per knot of the gradient of forward dynamics, counted on the "
                       "oracle's formulation (oracle/flop_count.py: zero and +-1 operands and "
                       "model-constant arithmetic free, FMA = 2, transcendentals not counted)",
               "command": "python -m oracle.flop_count --write profiles/flops_per_knot.json",
               "robots": counts}
        with open(sys.argv[2], "w") as fh:
            json.dump(doc, fh, indent=1)
            fh.write("\n")
        print(json.dumps({k: v["total"] for k, v in counts.items()}))
    else:
        print(json.dumps(workload_counts(), indent=1))
