"""Algorithmic work per knot of the batched gradient of forward dynamics.

A structure-aware operation count (one FMA = 2 FLOP) of the formulation the kernel
implements, with every structurally zero block skipped and nothing counted twice:
derivative columns touch only the bodies they can reach, M^-1 is block diagonal over
the branches attached to the fixed base, and the final product multiplies only those
blocks. Transcendentals (one sincos per joint) are not counted.

Per-primitive costs (FLOP):
  X m (motion transform)            42     X^T f (force transform)          42
  I x (rigid-body inertia apply)    42     v x* f (force cross product)     30
  (m x) S, S x* f                    0     composite inertia to parent     158
  E_z(q) E_T                        18
"""
from __future__ import annotations

import numpy as np

XM = 42
XTF = 42
IX = 42
CRF = 30
CONGRUENCE = 158
EZ_ET = 18


def _structure(parent):
    parent = [int(p) for p in parent]
    n = len(parent)
    anc = [[] for _ in range(n)]
    for i in range(n):
        a = parent[i]
        while a >= 0:
            anc[i].append(a)
            a = parent[a]
    branch = [i if parent[i] < 0 else None for i in range(n)]
    for i in range(n):
        if branch[i] is None:
            branch[i] = branch[parent[i]]
    sizes = {}
    for b in branch:
        sizes[b] = sizes.get(b, 0) + 1
    return n, parent, anc, branch, list(sizes.values())


def fdgrad_flops(parent) -> dict:
    """Per-knot FLOP count of each step; 'total' is their sum."""
    n, parent, anc, branch, blocks = _structure(parent)
    roots = sum(1 for p in parent if p < 0)
    nonroot = n - roots
    sum_depth = sum(len(a) + 1 for a in anc)          # (body, ancestor-or-self) pairs
    strict_pairs = sum(len(a) for a in anc)
    f = {}
    f["transforms"] = EZ_ET * n
    # RNEA(q, qd, 0): v (X m + S qd), a (X m + (v x S) qd), f = I a + v x* (I v)
    f["rnea_bias"] = (XM * nonroot + n) + (XM * n + 8 * n) + (2 * IX + CRF + 6) * n \
        + (XTF + 6) * nonroot + n
    # composite inertias, then M by walking each column up its ancestors
    f["crba"] = CONGRUENCE * nonroot + XTF * strict_pairs
    # Gauss-Jordan inverse of each base-branch block of M (b^3 updates of 3 FLOP)
    f["minv"] = sum(3 * b ** 3 + 2 * b * b for b in blocks)
    f["qdd"] = sum(2 * b * b for b in blocks)
    # RNEA at qdd: a (X m + S qdd + (v x S) qd), f = I a + (v x* I v reused), inward,
    # and the backward source X^T (S x* f)
    f["rnea_qdd"] = (XM + 9) * n + (IX + 6) * n + (XTF + 6) * nonroot + XTF * nonroot
    # dRNEA forward: per column, per reached body (j itself and its descendants):
    # X dv, X da, (dv x S) qd, df = I da + dv x* gamma + v x* (I dv)
    per_pair = XM + XM + 8 + (2 * IX + 2 * CRF + 12)
    at_source = 8 + (2 * IX + 2 * CRF + 12) + 10
    f["drnea_fwd"] = 2 * (per_pair * (sum_depth - n) + at_source * n)
    # backward: X^T df into the parent for every non-root body with a nonzero df
    # (descendants of j, j, and ancestors of j)
    reach = 0
    for j in range(n):
        desc = [i for i in range(n) if j in anc[i]]
        touched = set(desc) | {j} | set(anc[j])
        reach += sum(1 for i in touched if parent[i] >= 0)
    f["drnea_bwd"] = 2 * (XTF + 6) * reach + 6 * nonroot
    # -M^-1 dtau, block by block
    f["fdgrad_product"] = sum(4 * b ** 3 for b in blocks)
    f["total"] = int(sum(f.values()))
    return f


def io_bytes_per_knot(n: int) -> int:
    """HBM bytes one knot must move: q, qd, tau in; qdd, M^-1, dqdd/dq, dqdd/dqd out."""
    return 4 * (3 * n) + 4 * (n + 3 * n * n)


if __name__ == "__main__":
    from paper_2109_06976_amd import synth
    for name, p in [("chain7", synth.chain_parent(7)), ("quad12", synth.quadruped_parent()),
                    ("humanoid30", synth.humanoid_parent())]:
        f = fdgrad_flops(p)
        print(name, f, io_bytes_per_knot(len(p)))
