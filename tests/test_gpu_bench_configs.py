"""Parity at every configuration the benchmark times, through the C ABI, on an MI355X.

* every build of the fused kernel (the tuner may pick any of them) at every batch size the
  benchmark runs: the multiple-computation sweep N = 32 .. 1024 on the three robots, and the
  7-dof chain's throughput sizes up to 65536 knots;
* every build at the quadruped's and the humanoid's large batches (16384 and 65536 knots;
  4096 and 16384), on sampled knots, every output element written;
* the one-launch mixed module at the benchmark's quadruped + chain plans, each item bitwise
  equal to its robot's three-role build run alone;
* the largest batch one call accepts (GRID_MAX_KNOTS), on sampled knots.

Against the FP64 oracle with the tolerances of the parity tests: normwise per knot, qdd 1e-4,
M^-1, dqdd/dq and dqdd/dqd 1e-3 (the maximum over the knots must pass); M^-1 exactly
symmetric.
"""
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth

pytestmark = pytest.mark.gpu

OUTS = ("qdd", "Minv", "dqdd_dq", "dqdd_dqd")
TOL = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def normwise(got, ref):
    """Worst per-knot normwise error of one output."""
    N = ref.shape[0]
    y = np.asarray(got, np.float64).reshape(N, -1)
    r = ref.reshape(N, -1)
    scale = np.abs(r).max(1)
    return float((np.abs(y - r).max(1) / np.where(scale > 0, scale, 1.0)).max())


def check(ref, got, label):
    errs = {k: normwise(got[k], ref[k]) for k in OUTS}
    say(f"  {label}: " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    for k, b in TOL.items():
        assert errs[k] <= b, (label, k, errs[k])
    Mi = got["Minv"]
    np.testing.assert_array_equal(Mi, np.swapaxes(Mi, 1, 2))


def device_run(torch, model, kn):
    ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
    out = grid.fd_grad_torch(model, *ins)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


BENCH_SIZES = {
    "chain7": sorted(set(synth.SWEEP_KNOTS) | set(synth.THROUGHPUT_KNOTS)),
    "quad12": list(synth.SWEEP_KNOTS),
    "humanoid30": list(synth.SWEEP_KNOTS),
}


@pytest.mark.parametrize("name", list(BENCH_SIZES))
def test_every_build_at_every_benchmark_size(orc, name):
    import torch
    robot = synth.model_by_name(name)
    m = grid.Model(robot)
    try:
        for N in BENCH_SIZES[name]:
            kn = synth.random_knots(robot.n, N, 500 + N)
            ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
            for build in range(len(grid.BUILD_KERNELS)):
                grid.tune_apply(m, {1 << 22: build})
                say(f"[gpu] {name}: build {build} ({grid.BUILD_KERNELS[build]}), N={N}")
                check(ref, device_run(torch, m, kn), f"{name} build {build} N={N}")
    finally:
        m.close()


@pytest.mark.parametrize("name", list(synth.ROBOT_THROUGHPUT_KNOTS))
def test_every_build_at_robot_throughput_sizes(orc, name):
    """The large batches the benchmark times on the quadruped and the humanoid: every build
    runs the whole batch into arrays filled with NaN beforehand (every element must come out
    finite), and 64 sampled knots, the first and the last included, are checked against the
    oracle."""
    import torch
    robot = synth.model_by_name(name)
    n = robot.n
    m = grid.Model(robot)
    try:
        for N in synth.ROBOT_THROUGHPUT_KNOTS[name]:
            kn = synth.random_knots(n, N, 520 + N)
            rng = np.random.default_rng(521 + N)
            idx = np.unique(np.concatenate([[0, N - 1], rng.integers(0, N, 62)]))
            ref = orc.fd_grad_batch(robot, kn.q[idx], kn.qd[idx], kn.tau[idx])
            ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
            it = torch.from_numpy(idx).cuda()
            for build in range(len(grid.BUILD_KERNELS)):
                grid.tune_apply(m, {1 << 22: build})
                say(f"[gpu] {name}: build {build} ({grid.BUILD_KERNELS[build]}), N={N}, sampled")
                outs = [torch.full((N, n), float("nan"), device="cuda")] + \
                    [torch.full((N, n, n), float("nan"), device="cuda") for _ in range(3)]
                m.fd_grad(*ins, *outs, N=N)
                torch.cuda.synchronize()
                for k, o in zip(OUTS, outs):
                    assert bool(torch.isfinite(o).all()), (name, build, N, k)
                got = {k: o[it].cpu().numpy() for k, o in zip(OUTS, outs)}
                check(ref, got, f"{name} build {build} N={N}, {len(idx)} sampled knots")
                del outs
    finally:
        grid.tune_apply(m, {})
        m.close()
        torch.cuda.empty_cache()


def test_mixed_one_launch_at_benchmark_plans(orc):
    """The benchmark's quad12 + chain7 mixes in one launch of the two-robot module: every item
    equals, bit for bit, the same robot's three-role build run alone (same arithmetic per
    knot, only the workgroup-to-segment mapping differs), and the oracle within tolerance."""
    import torch
    robots = [synth.quad12(), synth.chain7()]
    mx = grid.Mixed(robots)
    models = [grid.Model(r) for r in robots]
    for m in models:
        grid.tune_apply(m, {1 << 22: grid.BUILD_PIPE})
    try:
        for nq, nc in synth.MIXED_PLANS:
            say(f"[gpu] mixed one launch: quad12 {nq} + chain7 {nc}")
            kns = [synth.random_knots(robots[0].n, nq, 600 + nq),
                   synth.random_knots(robots[1].n, nc, 700 + nc)]
            items, alone = [], []
            for r, kn in enumerate(kns):
                N, n = kn.N, robots[r].n
                ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
                outs = [torch.full((N, n), float("nan"), device="cuda")] + \
                       [torch.full((N, n, n), float("nan"), device="cuda") for _ in range(3)]
                items.append((r, *ins, *outs))
                alone.append(device_run(torch, models[r], kn))
            mx.launch(items)
            torch.cuda.synchronize()
            for r, (item, kn) in enumerate(zip(items, kns)):
                got = {k: t.cpu().numpy() for k, t in zip(OUTS, item[4:])}
                for k in OUTS:
                    np.testing.assert_array_equal(got[k], alone[r][k],
                                                  err_msg=f"{robots[r].name} N={kn.N} {k}")
                ref = orc.fd_grad_batch(robots[r], kn.q, kn.qd, kn.tau)
                check(ref, got, f"mixed {robots[r].name} N={kn.N}")
    finally:
        mx.close()
        for m in models:
            m.close()


def test_largest_batch_one_call_accepts(orc):
    """N = GRID_MAX_KNOTS (2^24) knots of the 7-dof chain in one call (about 12 GB of inputs
    and outputs): 64 sampled knots against the oracle, including the first and the last;
    one knot more is rejected before any launch."""
    import torch
    robot = synth.chain7()
    n, N = robot.n, grid.GRID_MAX_KNOTS
    m = grid.Model(robot)
    try:
        say(f"[gpu] chain7 N={N} (build {grid.build_for(m, N)})")
        g = torch.Generator(device="cuda")
        g.manual_seed(900)
        q = (torch.rand((N, n), device="cuda", generator=g) * 2 - 1) * np.pi
        qd = torch.randn((N, n), device="cuda", generator=g)
        tau = 5.0 * torch.randn((N, n), device="cuda", generator=g)
        out = grid.fd_grad_torch(m, q, qd, tau)
        torch.cuda.synchronize()
        rng = np.random.default_rng(901)
        idx = np.unique(np.concatenate([[0, N - 1], rng.integers(0, N, 62)]))
        it = torch.from_numpy(idx).cuda()
        kn = synth.Knots(*(x[it].cpu().numpy() for x in (q, qd, tau)))
        ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
        got = {k: out[k][it].cpu().numpy() for k in OUTS}
        check(ref, got, f"chain7 N={N}, {len(idx)} sampled knots")
        del out
        # raw addresses, so that the library's own limit is what rejects the call
        a = [int(x.data_ptr()) for x in (q, qd, tau)]
        with pytest.raises(grid.GridError) as e:
            m.fd_grad(*a, a[0], a[0], a[0], a[0], N=N + 1)
        assert e.value.status == grid.GRID_EINVAL
    finally:
        m.close()
        torch.cuda.empty_cache()
