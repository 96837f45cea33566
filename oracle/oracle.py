"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use this
module. It imports nothing from the product package: a model is any object with the
attributes parent, E_T, r, mass, com, Ic and gravity (float64 arrays as produced by
the seeded input generator).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GRID_ORACLE_LIB names another build of the same source (the sanitized build of the tests)
_LIB_PATH = os.environ.get("GRID_ORACLE_LIB") or os.path.join(_HERE, "libgrid_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Model(C.Structure):
    _fields_ = [("n", C.c_int), ("parent", _ip), ("E_T", _dp), ("r", _dp), ("mass", _dp),
                ("com", _dp), ("Ic", _dp), ("gravity", C.c_double * 3), ("axis", _dp),
                ("prismatic", _ip)]


class OracleError(RuntimeError):
    pass


def _load(path):
    handle = C.CDLL(path)
    for name in ("orc_rnea", "orc_crba", "orc_minv_cholesky", "orc_minv_direct", "orc_fd",
                 "orc_rnea_grad", "orc_fd_grad", "orc_fd_grad_batch", "orc_rnea_z", "orc_fd_z",
                 "orc_joint_transform", "orc_spatial_inertia", "orc_num_threads"):
        getattr(handle, name).restype = C.c_int
    handle.orc_set_num_threads.restype = None
    handle.orc_set_num_threads.argtypes = [C.c_int]
    return handle


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location("_oracle_build", os.path.join(_HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _lib = _load(_LIB_PATH)
    return _lib


def use_library(path: str):
    """Load another build of the same oracle source (the CPU-baseline timing build) for every
    later call of this module."""
    global _lib
    _lib = _load(path)
    return _lib


def set_num_threads(k: int):
    """OpenMP threads of later batch calls."""
    lib().orc_set_num_threads(int(k))


def _f64(x, shape=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _c128(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _ptr(a):
    if a is None:
        return None
    if a.dtype == np.complex128:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    return a.ctypes.data_as(_dp)


class OracleModel:
    """Holds the C view of a robot model (and keeps its arrays alive)."""

    def __init__(self, model):
        self.parent = np.ascontiguousarray(np.asarray(model.parent, dtype=np.int32))
        self.n = int(self.parent.shape[0])
        n = self.n
        self.E_T = _f64(model.E_T, (n, 9))
        self.r = _f64(model.r, (n, 3))
        self.mass = _f64(model.mass, (n,))
        self.com = _f64(model.com, (n, 3))
        self.Ic = _f64(model.Ic, (n, 6))
        g = _f64(model.gravity, (3,))
        ax = getattr(model, "axis", None)
        self.axis = None if ax is None else _f64(ax, (n, 3))
        # joint_type codes 0 revolute, 1 prismatic, 2 fixed; a fixed joint is handed over as
        # the revolute joint it would be, which the tests hold at q = qd = qdd = 0
        jt = getattr(model, "joint_type", None)
        self.prismatic = (None if jt is None else
                          np.ascontiguousarray((np.asarray(jt) == 1).astype(np.int32)))
        self.c = _Model(n, _ptr(self.parent), _ptr(self.E_T), _ptr(self.r), _ptr(self.mass),
                        _ptr(self.com), _ptr(self.Ic), (C.c_double * 3)(*g), _ptr(self.axis),
                        _ptr(self.prismatic))

    @property
    def ref(self):
        return C.byref(self.c)


def _om(model) -> OracleModel:
    return model if isinstance(model, OracleModel) else OracleModel(model)


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def crm(v):
    out = np.zeros(36)
    lib().orc_crm(_ptr(_f64(v, (6,))), _ptr(out))
    return out.reshape(6, 6)


def crf(v):
    out = np.zeros(36)
    lib().orc_crf(_ptr(_f64(v, (6,))), _ptr(out))
    return out.reshape(6, 6)


def joint_transform(model, i, q):
    om = _om(model)
    X = np.zeros(36)
    _check(lib().orc_joint_transform(om.ref, C.c_int(i), C.c_double(q), _ptr(X)), "transform")
    return X.reshape(6, 6)


def spatial_inertia(model, i):
    om = _om(model)
    Ib = np.zeros(36)
    _check(lib().orc_spatial_inertia(om.ref, C.c_int(i), _ptr(Ib)), "inertia")
    return Ib.reshape(6, 6)


def rnea(model, q, qd, qdd, gravity=True, return_bodies=False):
    om = _om(model)
    n = om.n
    q, qd, qdd = _f64(q, (n,)), _f64(qd, (n,)), _f64(qdd, (n,))
    tau = np.zeros(n)
    v = np.zeros((n, 6)) if return_bodies else None
    a = np.zeros((n, 6)) if return_bodies else None
    f = np.zeros((n, 6)) if return_bodies else None
    _check(lib().orc_rnea(om.ref, _ptr(q), _ptr(qd), _ptr(qdd), C.c_int(int(gravity)),
                          _ptr(tau), _ptr(v), _ptr(a), _ptr(f)), "rnea")
    return (tau, v, a, f) if return_bodies else tau


def rnea_complex(model, q, qd, qdd, gravity=True):
    om = _om(model)
    n = om.n
    q, qd, qdd = _c128(q), _c128(qd), _c128(qdd)
    tau = np.zeros(n, dtype=np.complex128)
    _check(lib().orc_rnea_z(om.ref, _ptr(q), _ptr(qd), _ptr(qdd), C.c_int(int(gravity)),
                            _ptr(tau)), "rnea_z")
    return tau


def crba(model, q):
    om = _om(model)
    M = np.zeros((om.n, om.n))
    _check(lib().orc_crba(om.ref, _ptr(_f64(q, (om.n,))), _ptr(M)), "crba")
    return M


def minv_cholesky(model, q):
    om = _om(model)
    Minv = np.zeros((om.n, om.n))
    _check(lib().orc_minv_cholesky(om.ref, _ptr(_f64(q, (om.n,))), _ptr(Minv)), "minv")
    return Minv


def minv_direct(model, q):
    om = _om(model)
    Minv = np.zeros((om.n, om.n))
    _check(lib().orc_minv_direct(om.ref, _ptr(_f64(q, (om.n,))), _ptr(Minv)), "minv_direct")
    return Minv


def fd(model, q, qd, tau):
    om = _om(model)
    n = om.n
    qdd = np.zeros(n)
    _check(lib().orc_fd(om.ref, _ptr(_f64(q, (n,))), _ptr(_f64(qd, (n,))),
                        _ptr(_f64(tau, (n,))), _ptr(qdd)), "fd")
    return qdd


def fd_complex(model, q, qd, tau):
    om = _om(model)
    n = om.n
    qdd = np.zeros(n, dtype=np.complex128)
    _check(lib().orc_fd_z(om.ref, _ptr(_c128(q)), _ptr(_c128(qd)), _ptr(_c128(tau)),
                          _ptr(qdd)), "fd_z")
    return qdd


def rnea_grad(model, q, qd, qdd):
    om = _om(model)
    n = om.n
    dq = np.zeros((n, n))
    dqd = np.zeros((n, n))
    _check(lib().orc_rnea_grad(om.ref, _ptr(_f64(q, (n,))), _ptr(_f64(qd, (n,))),
                               _ptr(_f64(qdd, (n,))), _ptr(dq), _ptr(dqd)), "rnea_grad")
    return dq, dqd


def fd_grad(model, q, qd, tau):
    """One knot: (qdd, Minv, dqdd/dq, dqdd/dqd)."""
    om = _om(model)
    n = om.n
    qdd = np.zeros(n)
    Minv = np.zeros((n, n))
    dq = np.zeros((n, n))
    dqd = np.zeros((n, n))
    _check(lib().orc_fd_grad(om.ref, _ptr(_f64(q, (n,))), _ptr(_f64(qd, (n,))),
                             _ptr(_f64(tau, (n,))), _ptr(qdd), _ptr(Minv), _ptr(dq), _ptr(dqd)),
           "fd_grad")
    return qdd, Minv, dq, dqd


def fd_grad_batch(model, q, qd, tau):
    """N knots (knot-major [N, n] inputs) -> dict of float64 outputs; OpenMP over knots."""
    om = _om(model)
    n = om.n
    q = _f64(q).reshape(-1, n)
    N = q.shape[0]
    qd = _f64(qd).reshape(N, n)
    tau = _f64(tau).reshape(N, n)
    out = {"qdd": np.zeros((N, n)), "Minv": np.zeros((N, n, n)),
           "dqdd_dq": np.zeros((N, n, n)), "dqdd_dqd": np.zeros((N, n, n))}
    _check(lib().orc_fd_grad_batch(om.ref, C.c_int(N), _ptr(q), _ptr(qd), _ptr(tau),
                                   _ptr(out["qdd"]), _ptr(out["Minv"]), _ptr(out["dqdd_dq"]),
                                   _ptr(out["dqdd_dqd"])), "fd_grad_batch")
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())
