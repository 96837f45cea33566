"""Host-side checks of the C ABI: the library loads, exports every declared call,
validates arguments before touching a device, and generates per-robot code. No GPU."""
import os
import re

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "grid.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(grid_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = grid.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(grid.EXPORTED)


def test_status_strings():
    assert grid.status_string(0) == "GRID_OK"
    assert grid.status_string(-1) == "GRID_EINVAL"
    assert grid.status_string(-5) == "GRID_ECOMPILE"
    assert grid.status_string(17) == "GRID_UNKNOWN"


def _bad(robot, **changes):
    r = robot.copy()
    for k, v in changes.items():
        setattr(r, k, v)
    return r


@pytest.mark.parametrize("mutate,status", [
    (lambda r: _bad(r, parent=np.array([-1, 0, 2, 2, 3, 4, 5], np.int32)), grid.GRID_EINVAL),
    (lambda r: _bad(r, mass=np.where(np.arange(7) == 3, -1.0, r.mass)), grid.GRID_EINVAL),
    (lambda r: _bad(r, E_T=r.E_T * 2.0), grid.GRID_EINVAL),
    (lambda r: _bad(r, Ic=np.tile([0.1, 0.1, 0.1, 0.5, 0, 0], (7, 1))), grid.GRID_EINVAL),
    (lambda r: _bad(r, r=np.where(np.arange(21).reshape(7, 3) == 4, np.nan, r.r)),
     grid.GRID_EINVAL),
    (lambda r: _bad(r, axis=np.tile([0.0, 0.0, 1.01], (7, 1))), grid.GRID_EINVAL),
])
def test_model_create_rejects_bad_descriptions_before_device_work(mutate, status):
    with pytest.raises(grid.GridError) as e:
        grid.Model(mutate(synth.chain7()))
    assert e.value.status == status


def test_model_create_rejects_too_many_bodies():
    robot = synth.random_model(synth.chain_parent(33), 0)
    with pytest.raises(grid.GridError) as e:
        grid.Model(robot)
    assert e.value.status == grid.GRID_EUNSUPPORTED


def test_unknown_flags_rejected():
    with pytest.raises(grid.GridError) as e:
        grid.Model(synth.chain7(), flags=8)
    assert e.value.status == grid.GRID_EINVAL


def _shapes(src):
    """(B, L, parent list, anc masks) of every generated branch shape."""
    return [(B, L, parent, anc) for B, L, Q, W, parent, anc in _shapes_quad(src)]


def _shapes_quad(src):
    """(B, L, Q, W, parent list, anc masks) of every generated branch shape."""
    out = []
    for m in re.finditer(r"struct Shape<(\d+)> \{\s*static constexpr int B = (\d+);\s*"
                         r"static constexpr int L = (\d+);\s*static constexpr int Q = (\d+);\s*"
                         r"static constexpr int W = (\d+);\s*static constexpr int PP = \d+;\s*"
                         r"static constexpr int parent\[B\] = "
                         r"\{([^}]*)\};\s*static constexpr unsigned long long anc\[B\] = \{([^}]*)\}",
                         src):
        parent = [int(x) for x in m.group(6).split(",")]
        anc = [int(x.strip().replace("ull", "")) for x in m.group(7).split(",")]
        out.append((int(m.group(2)), int(m.group(3)), int(m.group(4)), int(m.group(5)), parent,
                    anc))
    return out


def _insts(src):
    out = []
    for m in re.finditer(r"struct Inst<(\d+)> \{\s*using S = Shape<(\d+)>;\s*"
                         r"static constexpr int N = \d+;\s*"
                         r"static constexpr int body\[S::B\] = \{([^}]*)\};", src):
        out.append((int(m.group(2)), [int(x) for x in m.group(3).split(",")]))
    return out


def test_codegen_quadruped_has_four_identical_branches():
    src = grid.codegen_source(synth.quad12())
    assert src.count("static constexpr int N = 12;") == 4   # one per branch
    shapes = _shapes(src)
    assert shapes == [(3, 8, [-1, 0, 1], [0, 0b1, 0b11])]
    insts = _insts(src)
    assert [b for _, b in insts] == [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11]]
    # each branch's constants are emitted as exact float literals, 24 per body
    robot = synth.quad12()
    for k in range(4):
        m = re.search(r"grid_const_%d\[(\d+)\] = \{([^}]*)\}" % k, src)
        vals = [float.fromhex(x.strip().rstrip("f")) for x in m.group(2).split(",")]
        assert int(m.group(1)) == 72 and len(vals) == 72
        for b in range(3):
            i = 3 * k + b
            np.testing.assert_array_equal(vals[24 * b:24 * b + 9], robot.E_T[i].reshape(9))
            np.testing.assert_array_equal(vals[24 * b + 9:24 * b + 12], robot.r[i])
            assert vals[24 * b + 21] == np.float32(robot.mass[i])


def test_codegen_quad_layout_shapes():
    # one quad per derivative column: Q quads in each of W wavefronts cover the 2B columns
    for robot in (synth.chain7(), synth.quad12(), synth.humanoid30()):
        src = grid.codegen_source(robot)
        shapes = _shapes_quad(src)
        waves = int(re.search(r"#define GRID_WAVES (\d+)", src).group(1))
        assert waves == max(W for _, _, _, W, _, _ in shapes)
        for B, L, Q, W, _, _ in shapes:
            assert Q * W >= 2 * B and Q <= 16 and 16 % Q == 0 and waves % W == 0
            assert (W == 1 and Q == L) or (Q == 16 and 16 * (W // 2) < 2 * B)
        # the three-role kernel: roles B and C cover the B columns of M and M^-1 with
        # QB = 16 / PP quads, one column per quad up to 16 bodies and two beyond; role A needs
        # ceil(2B / 16) wavefronts (at least two), all within GRID_PIPE_WAVES
        pp = [int(x) for x in re.findall(r"static constexpr int PP = (\d+);", src)]
        pw = int(re.search(r"#define GRID_PIPE_WAVES (\d+)", src).group(1))
        for (B, *_), p in zip(shapes, pp):
            qb = 16 // p
            assert qb * (1 if B <= 16 else 2) >= B and (qb == 16 or qb < 2 * B or qb == 1)
            assert pw >= max(2, (2 * B + 15) // 16) + 1 + (B <= 16)
        # the three-role kernel is generated into its own module only
        assert "grid_dispatch_p(" not in src and "grid_fdgrad_pipe(" not in src
        assert "grid_dispatch_p(const grid::Args& a, int block)" in \
            grid.codegen_source(robot, grid.GRID_CODEGEN_PIPE_MODULE)


def test_codegen_humanoid_branches():
    parent = synth.humanoid_parent("anatomical")
    src = grid.codegen_source(synth.humanoid30())
    shapes = _shapes(src)
    insts = _insts(src)
    # torso tree (torso, head, arms) and two identical legs
    assert sorted(len(b) for _, b in insts) == [6, 6, 18]
    assert len(shapes) == 2
    covered = sorted(i for _, b in insts for i in b)
    assert covered == list(range(30))
    for sid, bodies in insts:
        B, L, lparent, anc = shapes[sid]
        assert B == len(bodies) and L >= 2 * B and L & (L - 1) == 0
        for k, i in enumerate(bodies):
            p = parent[i]
            assert lparent[k] == (-1 if p < 0 else bodies.index(p))
            # strict-ancestor masks follow the local parents
            expect, a = 0, lparent[k]
            while a >= 0:
                expect |= 1 << a
                a = lparent[a]
            assert anc[k] == expect


def test_codegen_bfs_numbering_branches_are_local_orders():
    parent = np.array([-1, -1, -1, -1, 0, 1, 2, 3, 4, 5, 6, 7], np.int32)
    insts = _insts(grid.codegen_source(synth.random_model(parent, 3)))
    assert [b for _, b in insts] == [[0, 4, 8], [1, 5, 9], [2, 6, 10], [3, 7, 11]]


def test_codegen_rejects_bad_topology():
    robot = synth.random_model(np.array([-1, 0], np.int32), 1)
    robot.parent = np.array([-1, 1], np.int32)
    with pytest.raises(grid.GridError) as e:
        grid.codegen_source(robot)
    assert e.value.status == grid.GRID_EINVAL


def test_server_rejects_bad_arguments_without_a_device():
    import ctypes as C
    lib = grid.lib()
    h = C.c_void_p()
    cfg = grid.ServerConfig(1 << 20, 64, 1, 0)
    assert lib.grid_server_create(None, 1, C.byref(cfg), C.byref(h)) == grid.GRID_EINVAL
    t = C.c_uint64()
    assert lib.grid_server_submit(None, 0, 1, *([None] * 7), C.byref(t)) == grid.GRID_EINVAL
    assert lib.grid_server_wait(None, 1, 0) == grid.GRID_EINVAL
    assert lib.grid_server_destroy(None) == grid.GRID_OK
    assert grid.status_string(grid.GRID_ETIMEDOUT) == "GRID_ETIMEDOUT"


def test_model_queries_reject_null_without_a_device():
    import ctypes as C
    h = C.c_uint64()
    assert grid.lib().grid_model_code_hash(None, C.byref(h)) == grid.GRID_EINVAL
    n = C.c_int32()
    assert grid.lib().grid_model_info(None, C.byref(n), None, None) == grid.GRID_EINVAL


def test_mixed_module_source_holds_every_branch_of_every_robot():
    robots = [synth.chain7(), synth.quad12(), synth.humanoid30()]
    src = grid.mixed_source(robots)
    assert "#define GRID_PIPE_ONLY" in src
    assert 'extern "C" __global__' in src and "grid_fdgrad_pipe_mixed(" in src
    # the persistent form: each segment's workgroups stride over that segment's blocks, the
    # loop inside the segment's case
    assert "grid_fdgrad_pipe_mixed_persistent(MixedArgs args)" in src
    assert re.search(r"struct MixedArgs \{\s*int nseg;\s*int nblocks;", src)
    # the robots' branches, numbered across the robots, one switch case each in both kernels
    per = [len(_insts(grid.codegen_source(r))) for r in robots]
    assert per[:2] == [1, 4]
    total = sum(per)
    assert len(re.findall(r"^\s*case \d+: gridq::run_pipe<Inst<\d+>>", src, re.M)) == total - 1
    assert len(re.findall(r"^\s*default: gridq::run_pipe<Inst<%d>>" % (total - 1), src,
                          re.M)) == 1
    loops = re.findall(r"^\s*(case \d+|default):\n\s*for \(int lb = lw; lb < nb; lb \+= nw\)\n"
                       r"\s*gridq::run_pipe<Inst<(\d+)>, true>\(x, lb\);", src, re.M)
    assert [int(k) for _, k in loops] == list(range(total))
    assert [b for _, b in _insts(src)] == sum((
        [b for _, b in _insts(grid.codegen_source(r))] for r in robots), [])
    # each robot carries its own joint count and gravity
    assert src.count("static constexpr int N = 7;") == per[0]
    assert src.count("static constexpr int N = 12;") == per[1]
    assert src.count("static constexpr int N = 30;") == per[2]
    assert all(f"grid_a0_{r}[3]" in src for r in range(3))
    # the one-robot kernels are compiled out of the module
    tail = src.split('#line 1 "grid_fused.hip"')[-1]
    assert tail.index("#ifndef GRID_PIPE_ONLY") < tail.index("grid_fdgrad_quad(")


def test_mixed_rejects_bad_arguments_without_a_device():
    import ctypes as C
    lib = grid.lib()
    h = C.c_void_p()
    assert lib.grid_mixed_create(None, 1, 0, C.byref(h)) == grid.GRID_EINVAL
    _d, arr = grid._desc_array([synth.chain7()])
    assert lib.grid_mixed_create(arr, 0, 0, C.byref(h)) == grid.GRID_EINVAL
    _d17, arr17 = grid._desc_array([synth.chain7()] * 17)
    assert lib.grid_mixed_create(arr17, 17, 0, C.byref(h)) == grid.GRID_EINVAL
    bad = synth.chain7()
    bad.parent = bad.parent.copy()
    bad.parent[3] = 5                                   # a parent after its child
    _db, arrb = grid._desc_array([synth.chain7(), bad])
    assert lib.grid_mixed_create(arrb, 2, 0, C.byref(h)) == grid.GRID_EINVAL
    assert "model 1" in grid.last_error()
    assert lib.grid_mixed_create(arr, 1, 0, None) == grid.GRID_EINVAL
    item = grid.GridMixedItem()
    assert lib.grid_mixed_launch(None, C.byref(item), 1, None) == grid.GRID_EINVAL
    assert lib.grid_mixed_destroy(None) == grid.GRID_OK
    ln = C.c_size_t(0)
    assert lib.grid_mixed_source(arr, 1, None, None) == grid.GRID_EINVAL
    assert lib.grid_mixed_source(arr, 1, None, C.byref(ln)) == grid.GRID_OK and ln.value > 1000


def test_pipe_kernel_has_a_module_of_its_own():
    robot = synth.chain7()
    main = grid.codegen_source(robot)
    pipe = grid.codegen_source(robot, grid.GRID_CODEGEN_PIPE_MODULE)
    assert "#define GRID_PIPE_ONLY" in pipe and "#define GRID_PIPE_ONLY" not in main
    assert 'grid_fdgrad_pipe(grid::Args args)' in pipe
    assert "grid_dispatch_p(args, (int)blockIdx.x)" in pipe
    # the same robot: identical branch structures and constants in both preludes
    assert _insts(pipe) == _insts(main)
    assert pipe.split('#line 1 "grid_device.hip"')[0].split("\n", 2)[2] == \
        main.split('#line 1 "grid_device.hip"')[0].split("\n", 1)[1]
    with pytest.raises(grid.GridError) as e:
        grid.codegen_source(robot, 1 << 3)
    assert e.value.status == grid.GRID_EINVAL
    with pytest.raises(grid.GridError) as e:
        grid.Model(robot, flags=grid.GRID_CODEGEN_PIPE_MODULE)   # a codegen flag only
    assert e.value.status == grid.GRID_EINVAL


class _FakeTensor:
    """Just enough of a torch tensor's interface for the binding's checks (no GPU here)."""

    def __init__(self, numel, dtype="torch.float32", is_cuda=True, device=0, contiguous=True):
        self._n, self.dtype, self.is_cuda = numel, dtype, is_cuda
        self._dev, self._contig = device, contiguous

    def get_device(self):
        return self._dev if self.is_cuda else -1

    def is_contiguous(self):
        return self._contig

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


def test_binding_rejects_unusable_tensors_before_the_call():
    """A kernel must never see a host pointer, a short buffer, another dtype, a strided view
    or memory of another GPU: the binding raises GRID_EINVAL first."""
    ok = _FakeTensor(4 * 7)
    assert grid._dev(ok, 28, 0, "q") == 0x1000
    assert grid._dev(None, 28, 0, "q") is None and grid._dev(0x2000, 28, 0, "q") == 0x2000
    bad = {"host": _FakeTensor(28, is_cuda=False), "short": _FakeTensor(27),
           "float64": _FakeTensor(28, dtype="torch.float64"),
           "strided": _FakeTensor(28, contiguous=False), "other GPU": _FakeTensor(28, device=1)}
    for what, t in bad.items():
        with pytest.raises(grid.GridError) as e:
            grid._dev(t, 28, 0, what)
        assert e.value.status == grid.GRID_EINVAL, what
    # the sizes a gradient-of-forward-dynamics call needs: [N][n] vectors, [N][n][n] matrices
    v, m = grid._vec_mat(4, 7)
    assert (v, m) == (28, 196) and grid._vec_mat(-1, 7) == (0, 0)
    vecs = [_FakeTensor(28)] * 4
    mats = [_FakeTensor(196)] * 3
    assert len(grid._fd_grad_ptrs(4, 7, 0, *vecs[:3], vecs[3], *mats)) == 7
    with pytest.raises(grid.GridError):
        grid._fd_grad_ptrs(4, 7, 0, *vecs[:3], vecs[3], mats[0], mats[1], _FakeTensor(195))
    import torch
    with pytest.raises(grid.GridError):
        grid._dev(torch.zeros(28), 28, 0, "q")          # a real host tensor


def test_max_knots_constant_matches_the_header():
    hdr = open(HEADER).read()
    assert re.search(r"#define GRID_MAX_KNOTS \(1 << 24\)", hdr)
    assert grid.GRID_MAX_KNOTS == 1 << 24


def test_mixed_modes_reject_bad_arguments_without_a_device():
    import ctypes as C
    lib = grid.lib()
    item = grid.GridMixedItem()
    assert lib.grid_mixed_launch_mode(None, C.byref(item), 1, 0, None) == grid.GRID_EINVAL
    assert lib.grid_mixed_tune(None, C.byref(item), 1, None, None) == grid.GRID_EINVAL
    assert (grid.MIXED_ONE_LAUNCH, grid.MIXED_PERSISTENT, grid.MIXED_PER_ROBOT) == (0, 1, 2)
    hdr = open(HEADER).read()
    for name, v in (("ONE_LAUNCH", 0), ("PERSISTENT", 1), ("PER_ROBOT", 2)):
        assert re.search(r"#define GRID_MIXED_%s %d" % (name, v), hdr)


def test_pinned_path_rejects_bad_arguments_without_a_device():
    import ctypes as C
    lib = grid.lib()
    pin, pout = C.POINTER(C.c_float)(), C.POINTER(C.c_float)()
    assert lib.grid_workspace_host_buffers(None, C.byref(pin), C.byref(pout)) == grid.GRID_EINVAL
    assert lib.grid_fd_grad_pinned(None, None, 4, 1, None) == grid.GRID_EINVAL
