"""Python binding of libgrid (include/grid.h): argument marshalling only.

Every step of the path runs in the HIP library; this module converts Python objects
to the C types of the interface and raises GridError on a non-zero status. It loads
the in-tree libgrid.so and fails loudly when it has not been built. Device arrays are
passed as torch tensors (or raw integer device addresses); PyTorch only provides the
memory and the stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GRID_LIB names another build of the same library (the sanitized host build of the tests)
LIB_PATH = os.environ.get("GRID_LIB") or os.path.join(_HERE, "libgrid.so")

GRID_OK = 0
GRID_EINVAL = -1
GRID_ENOMEM = -2
GRID_EDEVICE = -3
GRID_EUNSUPPORTED = -4
GRID_ECOMPILE = -5
GRID_EBUSY = -6
GRID_ETIMEDOUT = -7
GRID_ECANCELED = -8
GRID_NOALLOC_SCRATCH_BYTES = 16 << 20
IO_COPY_KERNEL = 0           # grid_fd_grad_mapped output modes
IO_DIRECT = 1
GRID_MAX_KNOTS = 1 << 24      # the largest N of one call
GRID_SERVER_PER_REQUEST = 1
GRID_SERVER_MAPPED_IO = 2
GRID_SERVER_DIRECT_PINNED = 4
# M^-1 routes of grid_minv_route
MINV_QUAD, MINV_LANE_LTL, MINV_LANE_DIRECT = 0, 1, 2
GRID_CODEGEN_PIPE_MODULE = 1 << 16

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_f32p = C.POINTER(C.c_float)


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("parent", _i32p), ("joint_type", _i32p), ("axis", _f64p),
                ("tree_rot", _f64p), ("tree_pos", _f64p), ("mass", _f64p), ("com", _f64p),
                ("inertia_com", _f64p), ("gravity", C.c_double * 3)]


class GridTiming(C.Structure):
    _fields_ = [("h2d_ms", C.c_float), ("kernel_ms", C.c_float), ("d2h_ms", C.c_float),
                ("total_ms", C.c_float)]


class ServerConfig(C.Structure):
    _fields_ = [("device_budget_bytes", C.c_size_t), ("max_batch_knots", C.c_int32),
                ("contexts_per_model", C.c_int32), ("flags", C.c_uint32),
                ("batch_window_us", C.c_int32), ("min_batch_knots", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("canceled", C.c_uint64),
                ("knots_completed", C.c_uint64), ("launches", C.c_uint64),
                ("max_inflight_bytes", C.c_uint64), ("inplace_launches", C.c_uint64)]


class LoadgenConfig(C.Structure):
    _fields_ = [("rate_per_s", C.c_double), ("duration_s", C.c_double), ("warmup_s", C.c_double),
                ("model_prob", _f64p), ("n_min", C.c_int32), ("n_max", C.c_int32),
                ("seed", C.c_uint64), ("pinned", C.c_int32)]


class LatencySplit(C.Structure):
    _fields_ = [("queue_us", C.c_double), ("h2d_us", C.c_double), ("kernel_us", C.c_double),
                ("d2h_us", C.c_double), ("complete_us", C.c_double), ("copyout_us", C.c_double)]


class LoadgenResult(C.Structure):
    _fields_ = [("requests", C.c_uint64), ("knots", C.c_uint64), ("seconds", C.c_double),
                ("p50_us", C.c_double), ("p90_us", C.c_double), ("p99_us", C.c_double),
                ("max_us", C.c_double), ("mean_us", C.c_double),
                ("offered_rate_per_s", C.c_double), ("requests_per_launch", C.c_double),
                ("p50", LatencySplit), ("p99", LatencySplit),
                ("model_requests", C.c_uint64 * 8), ("model_p50_us", C.c_double * 8),
                ("model_p99_us", C.c_double * 8)]


class GridItem(C.Structure):
    _fields_ = [("model", C.c_void_p), ("N", C.c_int32), ("q", C.c_void_p), ("qd", C.c_void_p),
                ("tau", C.c_void_p), ("qdd", C.c_void_p), ("Minv", C.c_void_p),
                ("dqdd_dq", C.c_void_p), ("dqdd_dqd", C.c_void_p)]


class GridMixedItem(C.Structure):
    _fields_ = [("robot", C.c_int32), ("N", C.c_int32), ("q", C.c_void_p), ("qd", C.c_void_p),
                ("tau", C.c_void_p), ("qdd", C.c_void_p), ("Minv", C.c_void_p),
                ("dqdd_dq", C.c_void_p), ("dqdd_dqd", C.c_void_p)]


class GridError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "grid_status_string": (C.c_char_p, [C.c_int32]),
    "grid_last_error": (C.c_char_p, []),
    "grid_model_create": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_uint32,
                                      C.POINTER(C.c_void_p)]),
    "grid_model_destroy": (C.c_int32, [C.c_void_p]),
    "grid_model_code_hash": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "grid_model_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_size_t),
                                    C.POINTER(C.c_int32)]),
    "grid_fd_grad": (C.c_int32, [C.c_void_p, C.c_int32] + [C.c_void_p] * 7 + [C.c_void_p]),
    "grid_fd_vjp": (C.c_int32, [C.c_void_p, C.c_int32] + [C.c_void_p] * 7 + [C.c_void_p]),
    "grid_fd_grad_staged": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32] + [C.c_void_p] * 7 +
                            [C.c_void_p]),
    "grid_fd_grad_staged_noalloc": (C.c_int32, [C.c_void_p, C.c_int32] + [C.c_void_p] * 7 +
                                    [C.c_void_p]),
    "grid_workspace_create": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "grid_fd_grad_batch": (C.c_int32, [C.POINTER(GridItem), C.c_int32, C.c_void_p]),
    "grid_graph_create": (C.c_int32, [C.POINTER(GridItem), C.c_int32, C.POINTER(C.c_void_p)]),
    "grid_graph_launch": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "grid_graph_update": (C.c_int32, [C.c_void_p, C.POINTER(GridItem), C.c_int32]),
    "grid_graph_destroy": (C.c_int32, [C.c_void_p]),
    "grid_tune": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_char_p,
                              C.POINTER(C.c_int32)]),
    "grid_tune_apply": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.c_int32]),
    "grid_build_for": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "grid_id": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p]),
    "grid_fd": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p]),
    "grid_minv": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "grid_minv_route": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.c_void_p]),
    "grid_id_grad": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "grid_dt_jacobians": (C.c_int32, [C.c_void_p, C.c_int32, C.c_float, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "grid_fd_vjp_adjoint": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "grid_server_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(ServerConfig),
                                       C.POINTER(C.c_void_p)]),
    "grid_server_submit": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32] + [C.c_void_p] * 7 +
                           [C.POINTER(C.c_uint64)]),
    "grid_server_wait": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_int64]),
    "grid_server_stats_get": (C.c_int32, [C.c_void_p, C.POINTER(ServerStats)]),
    "grid_server_destroy": (C.c_int32, [C.c_void_p]),
    "grid_server_pin_range": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "grid_server_unpin_range": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "grid_server_loadgen": (C.c_int32, [C.c_void_p, C.POINTER(LoadgenConfig),
                                        C.POINTER(LoadgenResult)]),
    "grid_workspace_destroy": (C.c_int32, [C.c_void_p]),
    "grid_fd_grad_host": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32] + [C.c_void_p] * 7 +
                          [C.POINTER(GridTiming)]),
    "grid_codegen_source": (C.c_int32, [C.POINTER(GridDesc), C.c_uint32, C.c_char_p,
                                        C.POINTER(C.c_size_t)]),
    "grid_codegen_precompile": (C.c_int32, [C.POINTER(GridDesc), C.c_uint32]),
    "grid_mixed_create": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_int32,
                                      C.POINTER(C.c_void_p)]),
    "grid_mixed_launch": (C.c_int32, [C.c_void_p, C.POINTER(GridMixedItem), C.c_int32,
                                      C.c_void_p]),
    "grid_mixed_destroy": (C.c_int32, [C.c_void_p]),
    "grid_mixed_launch_mode": (C.c_int32, [C.c_void_p, C.POINTER(GridMixedItem), C.c_int32,
                                           C.c_int32, C.c_void_p]),
    "grid_mixed_graph_create": (C.c_int32, [C.c_void_p, C.POINTER(GridMixedItem), C.c_int32,
                                            C.c_int32, C.POINTER(C.c_void_p)]),
    "grid_mixed_graph_update": (C.c_int32, [C.c_void_p, C.POINTER(GridMixedItem), C.c_int32]),
    "grid_mixed_tune": (C.c_int32, [C.c_void_p, C.POINTER(GridMixedItem), C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "grid_workspace_host_buffers": (C.c_int32, [C.c_void_p, C.POINTER(C.POINTER(C.c_float)),
                                                C.POINTER(C.POINTER(C.c_float))]),
    "grid_fd_grad_pinned": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(GridTiming)]),
    "grid_fd_grad_mapped": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(GridTiming)]),
    "grid_mixed_source": (C.c_int32, [C.POINTER(GridDesc), C.c_int32, C.c_char_p,
                                      C.POINTER(C.c_size_t)]),
    "grid_mixed_precompile": (C.c_int32, [C.POINTER(GridDesc), C.c_int32]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load the in-tree libgrid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GridError(GRID_EDEVICE, f"{LIB_PATH} is missing: run __graft_entry__.build()")
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status: int) -> str:
    return lib().grid_status_string(status).decode()


def last_error() -> str:
    return lib().grid_last_error().decode()


def _check(status: int):
    if status != GRID_OK:
        raise GridError(status, last_error())


def _dev(x, numel: int, device: int, what: str) -> int | None:
    """Device address of a float32 buffer that a kernel will read or write `numel` elements
    of. A torch tensor must be a contiguous float32 tensor on GPU `device` holding at least
    `numel` elements; anything else raises GridError(GRID_EINVAL) before the call, so that no
    kernel is launched on a host pointer, a short buffer or data of another type. None and
    int addresses are passed through (the library rejects NULL itself)."""
    if x is None or isinstance(x, int):
        return x
    if not getattr(x, "is_cuda", False):
        raise GridError(GRID_EINVAL, f"{what}: not a GPU tensor")
    if x.get_device() != device:
        raise GridError(GRID_EINVAL, f"{what}: on GPU {x.get_device()}, the model is on {device}")
    if str(x.dtype) != "torch.float32":
        raise GridError(GRID_EINVAL, f"{what}: dtype {x.dtype}, float32 required")
    if not x.is_contiguous():
        raise GridError(GRID_EINVAL, f"{what}: not contiguous")
    if x.numel() < numel:
        raise GridError(GRID_EINVAL, f"{what}: {x.numel()} elements, {numel} required")
    return int(x.data_ptr())


def _host_addr(x) -> int:
    """Address of a host buffer: an int, a numpy array, or a (pinned) CPU torch tensor."""
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    return int(x.data_ptr())


def _vec_mat(N: int, n: int):
    """Elements of an [N][n] and an [N][n][n] array (0 when N <= 0: the library handles it)."""
    N = max(int(N), 0)
    return N * n, N * n * n


def _fd_grad_ptrs(N, n, device, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd):
    """The seven checked device addresses of a gradient-of-forward-dynamics call."""
    v, m = _vec_mat(N, n)
    return (_dev(q, v, device, "q"), _dev(qd, v, device, "qd"), _dev(tau, v, device, "tau"),
            _dev(qdd, v, device, "qdd"), _dev(Minv, m, device, "Minv"),
            _dev(dqdd_dq, m, device, "dqdd_dq"), _dev(dqdd_dqd, m, device, "dqdd_dqd"))


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class _Desc:
    """C view of a robot model (keeps the numpy buffers alive)."""

    def __init__(self, robot):
        self.parent = np.ascontiguousarray(robot.parent, dtype=np.int32)
        n = int(self.parent.shape[0])
        self.arrays = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n, -1))
                       for a in (robot.E_T, robot.r, robot.mass, robot.com, robot.Ic)]
        E_T, r, mass, com, Ic = self.arrays
        g = np.asarray(robot.gravity, dtype=np.float64).reshape(3)
        p = lambda a: a.ctypes.data_as(_f64p)
        ax = getattr(robot, "axis", None)
        self.axis = None if ax is None else np.ascontiguousarray(
            np.asarray(ax, dtype=np.float64).reshape(n, 3))
        jt = getattr(robot, "joint_type", None)
        self.joint_type = None if jt is None else np.ascontiguousarray(jt, dtype=np.int32)
        self.c = GridDesc(n, self.parent.ctypes.data_as(_i32p),
                          None if self.joint_type is None else self.joint_type.ctypes.data_as(_i32p),
                          None if self.axis is None else p(self.axis), p(E_T), p(r),
                          p(mass), p(com), p(Ic), (C.c_double * 3)(*g))


class Model:
    """A robot model on one device (grid_model)."""

    def __init__(self, robot, device: int = 0, flags: int = 0):
        self._h = None
        desc = _Desc(robot)
        h = C.c_void_p()
        _check(lib().grid_model_create(C.byref(desc.c), int(device), int(flags), C.byref(h)))
        self._h = h
        n = C.c_int32()
        io = C.c_size_t()
        lanes = C.c_int32()
        _check(lib().grid_model_info(h, C.byref(n), C.byref(io), C.byref(lanes)))
        self.n, self.io_bytes_per_knot, self.lanes_per_knot = n.value, io.value, lanes.value
        self.device = device
        self.flags = flags

    @property
    def handle(self):
        return self._h

    @property
    def code_hash(self) -> str:
        """grid_model_code_hash: hash of the loaded code object, as 16 hex digits."""
        h = C.c_uint64()
        _check(lib().grid_model_code_hash(self._h, C.byref(h)))
        return f"{h.value:016x}"

    def close(self):
        if self._h is not None and self._h.value:
            lib().grid_model_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fd_grad(self, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd, N=None, stream=None):
        """grid_fd_grad on device buffers (torch tensors or addresses), asynchronous."""
        if N is None:
            N = int(q.shape[0])
        ptrs = _fd_grad_ptrs(N, self.n, self.device, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd)
        _check(lib().grid_fd_grad(self._h, int(N), *ptrs, _stream_handle(stream)))


    def fd_grad_staged_noalloc(self, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd, N=None,
                               stream=None):
        """grid_fd_grad_staged_noalloc: the five-launch pipeline with its intermediates in the
        library's static scratch array (no allocation; calls on one device must not overlap)."""
        if N is None:
            N = int(q.shape[0])
        ptrs = _fd_grad_ptrs(N, self.n, self.device, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd)
        _check(lib().grid_fd_grad_staged_noalloc(self._h, int(N), *ptrs,
                                                 _stream_handle(stream)))

    def fd_grad_call(self, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd, N=None, stream=None):
        """grid_fd_grad bound to fixed device buffers: returns a callable that makes the call.
        For loops that launch on the same buffers again and again (the arguments are
        converted to C once, which takes most of the Python-side cost of a call). The
        callable keeps the buffers alive; it raises GridError like fd_grad."""
        if N is None:
            N = int(q.shape[0])
        bufs = (q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd)
        ptrs = _fd_grad_ptrs(N, self.n, self.device, *bufs)
        args = (self._h, C.c_int(int(N)), *(C.c_void_p(x) for x in ptrs),
                C.c_void_p(_stream_handle(stream)))
        fn = lib().grid_fd_grad

        def call():
            st = fn(*args)
            if st != GRID_OK:
                raise GridError(st, last_error())

        call.buffers = bufs
        return call

    # the paper's other algorithms (device buffers, asynchronous)
    def id(self, q, qd, qdd, tau, N=None, stream=None):
        """grid_id: tau = ID(q, qd, qdd)."""
        N = int(q.shape[0]) if N is None else N
        v, _ = _vec_mat(N, self.n)
        d = self.device
        _check(lib().grid_id(self._h, int(N), _dev(q, v, d, "q"), _dev(qd, v, d, "qd"),
                             _dev(qdd, v, d, "qdd"), _dev(tau, v, d, "tau"),
                             _stream_handle(stream)))

    def fd(self, q, qd, tau, qdd, N=None, stream=None):
        """grid_fd: qdd = FD(q, qd, tau)."""
        N = int(q.shape[0]) if N is None else N
        v, _ = _vec_mat(N, self.n)
        d = self.device
        _check(lib().grid_fd(self._h, int(N), _dev(q, v, d, "q"), _dev(qd, v, d, "qd"),
                             _dev(tau, v, d, "tau"), _dev(qdd, v, d, "qdd"),
                             _stream_handle(stream)))

    def minv(self, q, Minv, N=None, stream=None):
        """grid_minv: M(q)^-1."""
        N = int(q.shape[0]) if N is None else N
        v, m = _vec_mat(N, self.n)
        _check(lib().grid_minv(self._h, int(N), _dev(q, v, self.device, "q"),
                               _dev(Minv, m, self.device, "Minv"), _stream_handle(stream)))

    def minv_route(self, q, Minv, route, N=None, stream=None):
        """grid_minv_route: M(q)^-1 by MINV_QUAD, MINV_LANE_LTL or MINV_LANE_DIRECT."""
        N = int(q.shape[0]) if N is None else N
        v, m = _vec_mat(N, self.n)
        _check(lib().grid_minv_route(self._h, int(N), _dev(q, v, self.device, "q"),
                                     _dev(Minv, m, self.device, "Minv"), int(route),
                                     _stream_handle(stream)))

    def id_grad(self, q, qd, qdd, dtau_dq, dtau_dqd, N=None, stream=None):
        """grid_id_grad: dtau/dq and dtau/dqd at the given qdd."""
        N = int(q.shape[0]) if N is None else N
        v, m = _vec_mat(N, self.n)
        d = self.device
        _check(lib().grid_id_grad(self._h, int(N), _dev(q, v, d, "q"), _dev(qd, v, d, "qd"),
                                  _dev(qdd, v, d, "qdd"), _dev(dtau_dq, m, d, "dtau_dq"),
                                  _dev(dtau_dqd, m, d, "dtau_dqd"), _stream_handle(stream)))


def fd_vjp_adjoint(model, q, qd, qdd, gbar, qbar, qdbar, taubar, N=None, stream=None):
    """grid_fd_vjp_adjoint: the VJP of FD by one reverse sweep (no Jacobians needed)."""
    if N is None:
        N = int(gbar.shape[0])
    v, _ = _vec_mat(N, model.n)
    d = model.device
    _check(lib().grid_fd_vjp_adjoint(model.handle, int(N), _dev(q, v, d, "q"),
                                     _dev(qd, v, d, "qd"), _dev(qdd, v, d, "qdd"),
                                     _dev(gbar, v, d, "gbar"), _dev(qbar, v, d, "qbar"),
                                     _dev(qdbar, v, d, "qdbar"), _dev(taubar, v, d, "taubar"),
                                     _stream_handle(stream)))


def fd_vjp(model, dqdd_dq, dqdd_dqd, Minv, gbar, qbar, qdbar, taubar, N=None, stream=None):
    """grid_fd_vjp on device buffers (torch tensors or addresses), asynchronous."""
    if N is None:
        N = int(gbar.shape[0])
    v, m = _vec_mat(N, model.n)
    d = model.device
    _check(lib().grid_fd_vjp(model.handle, int(N), _dev(dqdd_dq, m, d, "dqdd_dq"),
                             _dev(dqdd_dqd, m, d, "dqdd_dqd"), _dev(Minv, m, d, "Minv"),
                             _dev(gbar, v, d, "gbar"), _dev(qbar, v, d, "qbar"),
                             _dev(qdbar, v, d, "qdbar"), _dev(taubar, v, d, "taubar"),
                             _stream_handle(stream)))


def dt_jacobians(model, dt, dqdd_dq, dqdd_dqd, Minv, A, B, N=None, stream=None):
    """grid_dt_jacobians: A = d(q', qd')/d(q, qd), B = d(q', qd')/dtau of one semi-implicit
    Euler step from the dFD outputs (device buffers, asynchronous)."""
    if N is None:
        N = int(dqdd_dq.shape[0])
    _, m = _vec_mat(N, model.n)
    d = model.device
    _check(lib().grid_dt_jacobians(model.handle, int(N), float(dt),
                                   _dev(dqdd_dq, m, d, "dqdd_dq"), _dev(dqdd_dqd, m, d, "dqdd_dqd"),
                                   _dev(Minv, m, d, "Minv"), _dev(A, 4 * m, d, "A"),
                                   _dev(B, 2 * m, d, "B"), _stream_handle(stream)))


class Workspace:
    """grid_workspace: pinned staging + device buffers for the host-pointer call."""

    def __init__(self, model: Model, max_knots: int):
        self._h = None
        h = C.c_void_p()
        _check(lib().grid_workspace_create(model.handle, int(max_knots), C.byref(h)))
        self._h = h
        self.model = model
        self.max_knots = max_knots

    def close(self):
        if self._h is not None and self._h.value:
            lib().grid_workspace_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fd_grad_staged(self, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd, N=None, stream=None):
        """grid_fd_grad_staged: the five-launch pipeline on device buffers, asynchronous."""
        if N is None:
            N = int(q.shape[0])
        ptrs = _fd_grad_ptrs(N, self.model.n, self.model.device, q, qd, tau, qdd, Minv,
                             dqdd_dq, dqdd_dqd)
        _check(lib().grid_fd_grad_staged(self.model.handle, self._h, int(N), *ptrs,
                                         _stream_handle(stream)))

    def host_buffers(self, N):
        """The pinned buffers as numpy views for a call on N knots: (inputs dict q, qd, tau;
        outputs dict qdd, Minv, dqdd_dq, dqdd_dqd), packed as grid_workspace_host_buffers
        lays them out. Write the inputs in place, call fd_grad_pinned, read the outputs."""
        if not 0 <= N <= self.max_knots:
            raise GridError(GRID_EINVAL, "N must be in 0..max_knots of the workspace")
        pin, pout = C.POINTER(C.c_float)(), C.POINTER(C.c_float)()
        _check(lib().grid_workspace_host_buffers(self._h, C.byref(pin), C.byref(pout)))
        n = self.model.n
        vec, mat = N * n, N * n * n
        fin = np.ctypeslib.as_array(pin, shape=(3 * vec,)) if N else np.zeros(0, np.float32)
        fout = (np.ctypeslib.as_array(pout, shape=(vec + 3 * mat,)) if N
                else np.zeros(0, np.float32))
        ins = {k: fin[i * vec:(i + 1) * vec].reshape(N, n)
               for i, k in enumerate(("q", "qd", "tau"))}
        outs = {"qdd": fout[:vec].reshape(N, n)}
        for i, k in enumerate(("Minv", "dqdd_dq", "dqdd_dqd")):
            outs[k] = fout[vec + i * mat:vec + (i + 1) * mat].reshape(N, n, n)
        return ins, outs

    def fd_grad_pinned(self, N, pieces=1):
        """grid_fd_grad_pinned on the inputs already in the pinned buffers; returns the timing
        dict (with pieces > 1 only total_ms is measured)."""
        t = GridTiming()
        _check(lib().grid_fd_grad_pinned(self.model.handle, self._h, int(N), int(pieces),
                                         C.byref(t)))
        return {k: float(getattr(t, k)) for k in ("h2d_ms", "kernel_ms", "d2h_ms", "total_ms")}

    def fd_grad_mapped(self, N, out_mode=0, timed=True):
        """grid_fd_grad_mapped on the inputs already in the pinned buffers, no copy-engine
        transfers (out_mode IO_COPY_KERNEL or IO_DIRECT); returns the timing dict (None when
        timed is False: no events are recorded)."""
        if not timed:
            _check(lib().grid_fd_grad_mapped(self.model.handle, self._h, int(N), int(out_mode),
                                             None))
            return None
        t = GridTiming()
        _check(lib().grid_fd_grad_mapped(self.model.handle, self._h, int(N), int(out_mode),
                                         C.byref(t)))
        return {k: float(getattr(t, k)) for k in ("h2d_ms", "kernel_ms", "d2h_ms", "total_ms")}

    def fd_grad_host(self, q, qd, tau):
        """grid_fd_grad_host on numpy arrays; returns (outputs dict, timing dict)."""
        n = self.model.n
        q = np.ascontiguousarray(q, dtype=np.float32).reshape(-1, n)
        N = q.shape[0]
        qd = np.ascontiguousarray(qd, dtype=np.float32).reshape(N, n)
        tau = np.ascontiguousarray(tau, dtype=np.float32).reshape(N, n)
        out = {"qdd": np.empty((N, n), np.float32), "Minv": np.empty((N, n, n), np.float32),
               "dqdd_dq": np.empty((N, n, n), np.float32),
               "dqdd_dqd": np.empty((N, n, n), np.float32)}
        t = GridTiming()
        ptr = lambda a: a.ctypes.data
        _check(lib().grid_fd_grad_host(self.model.handle, self._h, N, ptr(q), ptr(qd), ptr(tau),
                                       ptr(out["qdd"]), ptr(out["Minv"]), ptr(out["dqdd_dq"]),
                                       ptr(out["dqdd_dqd"]), C.byref(t)))
        timing = {k: float(getattr(t, k)) for k in ("h2d_ms", "kernel_ms", "d2h_ms", "total_ms")}
        return out, timing


def _items(items):
    """items: sequence of (model, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd) with device
    tensors (N taken from q)."""
    arr = (GridItem * len(items))()
    for k, (m, q, qd, tau, qdd, Mi, dq, dqd) in enumerate(items):
        N = int(q.shape[0])
        arr[k] = GridItem(m.handle.value, N,
                          *_fd_grad_ptrs(N, m.n, m.device, q, qd, tau, qdd, Mi, dq, dqd))
    return arr


def fd_grad_batch(items, stream=None):
    arr = _items(items)
    _check(lib().grid_fd_grad_batch(arr, len(items), _stream_handle(stream)))


class Graph:
    """grid_graph: a mixed batch of robots captured as one hipGraph."""

    def __init__(self, items):
        self._h = None
        arr = _items(items)
        h = C.c_void_p()
        _check(lib().grid_graph_create(arr, len(items), C.byref(h)))
        self._h = h
        self.count = len(items)

    def launch(self, stream=None):
        _check(lib().grid_graph_launch(self._h, _stream_handle(stream)))

    def update(self, items):
        arr = _items(items)
        _check(lib().grid_graph_update(self._h, arr, len(items)))

    def close(self):
        if self._h is not None and self._h.value:
            lib().grid_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _desc_array(robots):
    descs = [_Desc(r) for r in robots]
    arr = (GridDesc * len(descs))(*[d.c for d in descs])
    return descs, arr


class Mixed:
    """grid_mixed: one module for several robots; a table of items runs as one launch."""

    def __init__(self, robots, device: int = 0):
        self._h = None
        _descs, arr = _desc_array(robots)
        h = C.c_void_p()
        _check(lib().grid_mixed_create(arr, len(robots), int(device), C.byref(h)))
        self._h = h
        self.count = len(robots)
        self.device = device
        # joints the arrays of each robot hold (fixed joints merged away)
        self.dofs = [int(np.sum(np.asarray(r.joint_type) != JOINT_FIXED))
                     if getattr(r, "joint_type", None) is not None else len(r.parent)
                     for r in robots]

    def _items(self, items):
        arr = (GridMixedItem * len(items))()
        for k, (r, q, qd, tau, qdd, Mi, dq, dqd) in enumerate(items):
            N = int(q.shape[0])
            # an index out of range is the library's to reject; its buffers are not checked
            n = self.dofs[r] if 0 <= int(r) < len(self.dofs) else 0
            arr[k] = GridMixedItem(int(r), N,
                                   *_fd_grad_ptrs(N if n else 0, n, self.device, q, qd, tau,
                                                  qdd, Mi, dq, dqd))
        return arr

    def launch(self, items, stream=None, mode=None):
        """items: sequence of (robot index, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd) with
        device tensors (N taken from q). mode None: the tuned (or default) mode; else one of
        MIXED_ONE_LAUNCH, MIXED_PERSISTENT, MIXED_PER_ROBOT."""
        arr = self._items(items)
        if mode is None:
            _check(lib().grid_mixed_launch(self._h, arr, len(items), _stream_handle(stream)))
        else:
            _check(lib().grid_mixed_launch_mode(self._h, arr, len(items), int(mode),
                                                _stream_handle(stream)))

    def launch_call(self, items, stream=None, mode=None):
        """The launch bound to fixed items (converted to C once) for timing loops."""
        arr = self._items(items)
        h, cnt, st = self._h, len(items), C.c_void_p(_stream_handle(stream))
        fn = lib().grid_mixed_launch if mode is None else lib().grid_mixed_launch_mode
        extra = () if mode is None else (int(mode),)

        def call():
            rc = fn(h, arr, cnt, *extra, st)
            if rc != GRID_OK:
                raise GridError(rc, last_error())

        call.buffers = items
        return call

    def graph(self, items, mode=None):
        """grid_mixed_graph_create: one mixed launch of these items captured in a hipGraph
        (mode None: the mode grid_mixed_launch picks for the batch size). Returns a MixedGraph;
        close it before this module."""
        return MixedGraph(self, items, -1 if mode is None else int(mode))

    def tune(self, items):
        """grid_mixed_tune: (chosen mode, {mode: us per launch})."""
        arr = self._items(items)
        chosen = C.c_int32()
        us = (C.c_float * 3)()
        _check(lib().grid_mixed_tune(self._h, arr, len(items), C.byref(chosen), us))
        return chosen.value, {m: float(us[m]) for m in range(3)}

    def close(self):
        if self._h is not None and self._h.value:
            lib().grid_mixed_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MixedGraph:
    """grid_graph made by grid_mixed_graph_create: one mixed launch as a replayable graph."""

    def __init__(self, mixed: Mixed, items, mode: int):
        self._h = None
        self.mixed = mixed
        self._arr = mixed._items(items)
        self.buffers = items
        h = C.c_void_p()
        _check(lib().grid_mixed_graph_create(mixed._h, self._arr, len(items), int(mode),
                                             C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().grid_graph_launch(self._h, _stream_handle(stream)))

    def launch_call(self, stream=None):
        """The replay with its arguments converted to C once (timing loops)."""
        h, st, fn = self._h, C.c_void_p(_stream_handle(stream)), lib().grid_graph_launch

        def call():
            rc = fn(h, st)
            if rc != GRID_OK:
                raise GridError(rc, last_error())

        return call

    def update(self, items):
        self._arr = self.mixed._items(items)
        self.buffers = items
        _check(lib().grid_mixed_graph_update(self._h, self._arr, len(items)))

    def close(self):
        if self._h is not None and self._h.value:
            lib().grid_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mixed_source(robots) -> str:
    """Generated HIP source of a mixed module (no device needed)."""
    _descs, arr = _desc_array(robots)
    ln = C.c_size_t(0)
    _check(lib().grid_mixed_source(arr, len(robots), None, C.byref(ln)))
    buf = C.create_string_buffer(ln.value)
    _check(lib().grid_mixed_source(arr, len(robots), buf, C.byref(ln)))
    return buf.value.decode()


def mixed_precompile(robots):
    """Compile a mixed module into the on-disk cache (no device needed)."""
    _descs, arr = _desc_array(robots)
    _check(lib().grid_mixed_precompile(arr, len(robots)))


def tune(model, Ns, table_path=None):
    """grid_tune: time the fused kernel builds for each N; returns the chosen build per N."""
    Ns = np.ascontiguousarray(Ns, dtype=np.int32)
    chosen = np.zeros(len(Ns), np.int32)
    path = table_path.encode() if table_path else None
    _check(lib().grid_tune(model.handle, Ns.ctypes.data_as(_i32p), len(Ns), path,
                           chosen.ctypes.data_as(_i32p)))
    return dict(zip(Ns.tolist(), chosen.tolist()))


def tune_apply(model, table):
    """grid_tune_apply: {largest N: build} (ascending N); {} returns to the untuned choice."""
    items = sorted(table.items())
    Ns = np.ascontiguousarray([n for n, _ in items], dtype=np.int32)
    builds = np.ascontiguousarray([b for _, b in items], dtype=np.int32)
    _check(lib().grid_tune_apply(model.handle, Ns.ctypes.data_as(_i32p),
                                 builds.ctypes.data_as(_i32p), len(items)))


BUILD_QUAD, BUILD_LANE, BUILD_LANE_W2, BUILD_LANE_W4, BUILD_PIPE, BUILD_SERIAL, BUILD_SERIAL4, \
    BUILD_SERIAL2 = range(8)
MIXED_ONE_LAUNCH, MIXED_PERSISTENT, MIXED_PER_ROBOT = range(3)
MIXED_MODES = ("one_launch", "persistent", "per_robot")
JOINT_REVOLUTE, JOINT_PRISMATIC, JOINT_FIXED = 0, 1, 2
BUILD_KERNELS = ("grid_fdgrad_quad", "grid_fdgrad_fused", "grid_fdgrad_fused_w2",
                 "grid_fdgrad_fused_w4", "grid_fdgrad_pipe", "grid_fdgrad_serial",
                 "grid_fdgrad_serial4", "grid_fdgrad_serial2")


def build_for(model, N):
    """grid_build_for: the build index a batch of N knots runs."""
    b = C.c_int32(0)
    _check(lib().grid_build_for(model.handle, int(N), C.byref(b)))
    return b.value


class Server:
    """grid_server: continuous batching of dFD requests over several models."""

    def __init__(self, models, budget_bytes=1 << 30, max_batch_knots=1024, contexts_per_model=3,
                 flags=0, batch_window_us=0, min_batch_knots=0):
        self._h = None
        self.models = list(models)
        handles = (C.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        cfg = ServerConfig(int(budget_bytes), int(max_batch_knots), int(contexts_per_model),
                           int(flags), int(batch_window_us), int(min_batch_knots))
        h = C.c_void_p()
        _check(lib().grid_server_create(handles, len(self.models), C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, model_index, q, qd, tau, out=None):
        """Queue one request on host arrays; returns (ticket, outputs dict being filled).
        out: the caller's own output arrays (dict qdd, Minv, dqdd_dq, dqdd_dqd; contiguous
        float32 of the right shapes), e.g. views of pinned memory for in-place requests."""
        n = self.models[model_index].n
        q = np.ascontiguousarray(q, dtype=np.float32).reshape(-1, n)
        N = q.shape[0]
        qd = np.ascontiguousarray(qd, dtype=np.float32).reshape(N, n)
        tau = np.ascontiguousarray(tau, dtype=np.float32).reshape(N, n)
        if out is None:
            out = {"qdd": np.empty((N, n), np.float32), "Minv": np.empty((N, n, n), np.float32),
                   "dqdd_dq": np.empty((N, n, n), np.float32),
                   "dqdd_dqd": np.empty((N, n, n), np.float32)}
        else:
            shapes = {"qdd": (N, n), "Minv": (N, n, n), "dqdd_dq": (N, n, n),
                      "dqdd_dqd": (N, n, n)}
            for k, sh in shapes.items():
                a = out[k]
                if a.dtype != np.float32 or a.shape != sh or not a.flags.c_contiguous:
                    raise GridError(GRID_EINVAL, f"out[{k}]: contiguous float32 {sh} required")
        t = C.c_uint64()
        ptr = lambda a: a.ctypes.data
        _check(lib().grid_server_submit(self._h, int(model_index), N, ptr(q), ptr(qd), ptr(tau),
                                        ptr(out["qdd"]), ptr(out["Minv"]), ptr(out["dqdd_dq"]),
                                        ptr(out["dqdd_dqd"]), C.byref(t)))
        self._keep[t.value] = (q, qd, tau, out)      # buffers must live until wait returns
        return t.value, out

    def pin_range(self, ptr, nbytes):
        """grid_server_pin_range: register a pinned host range (an address, or an array or
        tensor whose data pointer is taken) for in-place requests."""
        _check(lib().grid_server_pin_range(self._h, _host_addr(ptr), int(nbytes)))

    def unpin_range(self, ptr):
        _check(lib().grid_server_unpin_range(self._h, _host_addr(ptr)))

    def wait(self, ticket, timeout_us=-1):
        st = lib().grid_server_wait(self._h, C.c_uint64(ticket), C.c_int64(int(timeout_us)))
        if st != GRID_ETIMEDOUT:
            self._keep.pop(ticket, None)
        _check(st)

    def stats(self):
        s = ServerStats()
        _check(lib().grid_server_stats_get(self._h, C.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in ServerStats._fields_}

    def loadgen(self, rate_per_s, duration_s, model_prob, n_min=16, n_max=256, warmup_s=1.0,
                seed=7, pinned=False):
        probs = np.ascontiguousarray(model_prob, dtype=np.float64)
        cfg = LoadgenConfig(float(rate_per_s), float(duration_s), float(warmup_s),
                            probs.ctypes.data_as(_f64p), int(n_min), int(n_max), int(seed),
                            int(bool(pinned)))
        r = LoadgenResult()
        _check(lib().grid_server_loadgen(self._h, C.byref(cfg), C.byref(r)))
        out = {}
        for k, t in LoadgenResult._fields_:
            v = getattr(r, k)
            if k.startswith("model_"):
                out[k] = [v[i] for i in range(len(self.models))][:8]
                continue
            if t is LatencySplit:
                out[k + "_split"] = {f: float(getattr(v, f)) for f, _ in LatencySplit._fields_}
            else:
                out[k] = float(v) if t is C.c_double else int(v)
        return out

    def close(self):
        if self._h is not None and self._h.value:
            lib().grid_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def codegen_source(robot, flags: int = 0) -> str:
    """Generated HIP source for a robot model (no device needed)."""
    desc = _Desc(robot)
    ln = C.c_size_t(0)
    _check(lib().grid_codegen_source(C.byref(desc.c), flags, None, C.byref(ln)))
    buf = C.create_string_buffer(ln.value)
    _check(lib().grid_codegen_source(C.byref(desc.c), flags, buf, C.byref(ln)))
    return buf.value.decode()


def codegen_precompile(robot, flags: int = 0):
    """Compile a robot's kernel into the on-disk cache (no device needed)."""
    desc = _Desc(robot)
    _check(lib().grid_codegen_precompile(C.byref(desc.c), flags))


def fd_grad_torch(model: Model, q, qd, tau, stream=None):
    """Allocate outputs with torch on q's device and launch on the current stream."""
    import torch
    q, qd, tau = (x.contiguous().float() for x in (q, qd, tau))
    N, n = q.shape
    dev = q.device
    out = {"qdd": torch.empty((N, n), device=dev, dtype=torch.float32),
           "Minv": torch.empty((N, n, n), device=dev, dtype=torch.float32),
           "dqdd_dq": torch.empty((N, n, n), device=dev, dtype=torch.float32),
           "dqdd_dqd": torch.empty((N, n, n), device=dev, dtype=torch.float32)}
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    model.fd_grad(q, qd, tau, out["qdd"], out["Minv"], out["dqdd_dq"], out["dqdd_dqd"], N=N,
                  stream=stream)
    return out
