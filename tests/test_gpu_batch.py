"""Mixed-robot batches (serial launches and one hipGraph) and the autotuner's kernel
builds, on an MI355X through the C ABI."""
import os
import sys

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth

pytestmark = pytest.mark.gpu
OUTS = ("qdd", "Minv", "dqdd_dq", "dqdd_dqd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_item(torch, model, robot, N, seed):
    kn = synth.random_knots(robot.n, N, seed)
    ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
    n = robot.n
    outs = [torch.full((N, n), float("nan"), device="cuda")] + \
           [torch.full((N, n, n), float("nan"), device="cuda") for _ in range(3)]
    return (model, *ins, *outs), kn


def alone(torch, model, item):
    outs = [torch.empty_like(t) for t in item[4:]]
    model.fd_grad(*item[1:4], *outs)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def test_mixed_graph_equals_alone_and_updates():
    import torch
    quad, chain = synth.quad12(), synth.chain7()
    mq, mc = grid.Model(quad), grid.Model(chain)
    pairs = [(64, 37), (256, 181), (1024, 613)]
    items, _ = zip(*[make_item(torch, mq, quad, 64, 1), make_item(torch, mc, chain, 37, 2)])
    say("[gpu] mixed graph quad12 64 + chain7 37")
    g = grid.Graph(list(items))
    for step, (nq, nc) in enumerate(pairs):
        if step:
            say(f"[gpu] graph update quad12 {nq} + chain7 {nc}")
            items, _ = zip(*[make_item(torch, mq, quad, nq, 10 + step),
                             make_item(torch, mc, chain, nc, 20 + step)])
            g.update(list(items))
        for _ in range(3):                             # replays, with eager work between them
            g.launch()
            torch.cuda.synchronize()
            for item in items:
                ref = alone(torch, item[0], item)
                for got, want in zip(item[4:], ref):
                    np.testing.assert_array_equal(got.cpu().numpy(), want)
            for t in items[0][4:]:
                t.fill_(float("nan"))
    g.close()
    # the same items through serial launches
    grid.fd_grad_batch(list(items))
    torch.cuda.synchronize()
    for item in items:
        ref = alone(torch, item[0], item)
        for got, want in zip(item[4:], ref):
            np.testing.assert_array_equal(got.cpu().numpy(), want)
    mq.close()
    mc.close()


@pytest.mark.parametrize("robot_name,variant",
                         [(r, v) for r in ("chain7", "quad12", "humanoid30") for v in range(len(grid.BUILD_KERNELS))])
def test_every_tuned_build_matches_oracle(orc, tmp_path, variant, robot_name):
    import torch
    robot = synth.model_by_name(robot_name)
    table = tmp_path / "tune.json"
    N = 77   # ragged for every knot-to-workgroup packing
    say(f"[gpu] {robot_name} with fused build {variant}, N={N}")
    # tune once to obtain the table line keyed by this model, then force `variant` for
    # every N and apply it at model creation
    m = grid.Model(robot)
    tuned = grid.tune(m, [64], table_path=str(table))
    assert set(tuned.values()) <= set(range(len(grid.BUILD_KERNELS)))
    line = table.read_text().strip().splitlines()[-1]
    forced = line.split('"buckets"')[0] + f'"buckets": [[4194304, {variant}]]}}\n'
    table.write_text(forced)
    os.environ["GRID_TUNE_TABLE"] = str(table)
    try:
        m2 = grid.Model(robot)
    finally:
        del os.environ["GRID_TUNE_TABLE"]
    kn = synth.random_knots(robot.n, N, 104)
    out = grid.fd_grad_torch(m2, *(torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)))
    torch.cuda.synchronize()
    ref = orc.fd_grad_batch(robot, kn.q, kn.qd, kn.tau)
    tol = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}
    for k, b in tol.items():
        y = out[k].cpu().numpy().astype(np.float64).reshape(N, -1)
        r = ref[k].reshape(N, -1)
        err = (np.abs(y - r).max(1) / np.abs(r).max(1)).max()
        say(f"  {k} worst normwise error {err:.2e}")
        assert err <= b, k
    if robot.n > 1:
        np.testing.assert_array_equal(out["Minv"].cpu().numpy(),
                                      np.swapaxes(out["Minv"].cpu().numpy(), 1, 2))
    m.close()
    m2.close()


def test_tune_picks_builds_per_size(tmp_path):
    m = grid.Model(synth.chain7())
    say("[gpu] tune chain7 at 128, 1024, 16384 knots")
    chosen = grid.tune(m, [128, 1024, 16384], table_path=str(tmp_path / "t.json"))
    say(f"  chosen builds {chosen}")
    assert sorted(chosen) == [128, 1024, 16384]
    assert (tmp_path / "t.json").read_text().count("buckets") == 1
    m.close()


def test_graph_rejects_bad_items():
    import torch
    m = grid.Model(synth.chain7())
    t = torch.zeros((4, 7), device="cuda")
    with pytest.raises(grid.GridError) as e:
        grid.Graph([(m, t, None, t, t, t, t, t)])
    assert e.value.status == grid.GRID_EINVAL
    m.close()


def test_mixed_one_launch_equals_pipe_build_alone(orc):
    """One kernel launch over items of six robots (a chain, four legs, a 30-body tree,
    prismatic joints, fixed joints, 32 one-body branches), with a robot used twice, an empty
    item and ragged N: every item equals, bit for bit, the same robot's pipe build run alone,
    and the oracle within tolerance."""
    import torch
    from paper_2109_06976_amd import build
    robots = build.mixed_sets()[1]
    say("[gpu] mixed module: " + " + ".join(r.name for r in robots))
    mx = grid.Mixed(robots)
    models = []
    for r in robots:
        m = grid.Model(r)
        grid.tune_apply(m, {1 << 22: grid.BUILD_PIPE})
        models.append(m)
    plan = [(0, 37), (1, 64), (2, 5), (0, 1), (3, 0), (4, 19), (5, 3), (2, 2)]
    for launch in range(2):                      # a second launch reuses the module
        items, knots = [], []
        for j, (r, N) in enumerate(plan):
            n = models[r].n                      # degrees of freedom (fixed joints removed)
            kn = synth.random_knots(n, N, 700 + 10 * launch + j)
            ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
            outs = [torch.full((N, n), float("nan"), device="cuda")] + \
                   [torch.full((N, n, n), float("nan"), device="cuda") for _ in range(3)]
            items.append((models[r], *ins, *outs))
            knots.append(kn)
        say(f"[gpu] mixed launch {launch}: items {plan}")
        mx.launch([(r, *it[1:]) for (r, _), it in zip(plan, items)])
        torch.cuda.synchronize()
        tol = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}
        for (r, N), item, kn in zip(plan, items, knots):
            if N == 0:
                continue
            got = [t.cpu().numpy() for t in item[4:]]
            want = alone(torch, models[r], item)
            for k, g, w in zip(OUTS, got, want):
                np.testing.assert_array_equal(g, w, err_msg=f"{robots[r].name} N={N} {k}")
            if getattr(robots[r], "joint_type", None) is not None and \
                    (robots[r].joint_type == grid.JOINT_FIXED).any():
                continue                         # the locked-joint oracle covers its pipe build
            ref = orc.fd_grad_batch(robots[r], kn.q, kn.qd, kn.tau)
            for k, g in zip(OUTS, got):
                y = g.astype(np.float64).reshape(N, -1)
                w = ref[k].reshape(N, -1)
                err = (np.abs(y - w).max(1) / np.maximum(np.abs(w).max(1), 1e-30)).max()
                assert err <= tol[k], (robots[r].name, N, k, err)
    # host-side rejections: robot index, too many (item, branch) segments
    t = torch.zeros((4, 7), device="cuda")
    with pytest.raises(grid.GridError) as e:
        mx.launch([(6, t, t, t, t, t, t, t)])
    assert e.value.status == grid.GRID_EINVAL
    s32 = torch.zeros((1, 32), device="cuda")
    s32m = torch.zeros((1, 32, 32), device="cuda")
    with pytest.raises(grid.GridError) as e:
        mx.launch([(5, s32, s32, s32, s32, s32m, s32m, s32m)] * 3)   # 96 segments
    assert e.value.status == grid.GRID_EINVAL
    mx.close()
    for m in models:
        m.close()


def _mixed_items(torch, models, plan, seed):
    items, knots = [], []
    for j, (r, N) in enumerate(plan):
        n = models[r].n
        kn = synth.random_knots(n, N, seed + j)
        ins = [torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)]
        outs = [torch.full((N, n), float("nan"), device="cuda")] + \
               [torch.full((N, n, n), float("nan"), device="cuda") for _ in range(3)]
        items.append((r, *ins, *outs))
        knots.append(kn)
    return items, knots


@pytest.mark.parametrize("plan_name", ["six_robots_oversubscribed", "bench_1024_613"])
def test_mixed_persistent_equals_one_launch(orc, plan_name):
    """The persistent form (resident workgroups striding over the blocks, largest branches
    first) gives bitwise the one-launch outputs, also when there are several times more blocks
    than resident workgroups; both within tolerance of the oracle. The per-robot mode runs each
    item on its robot's own module and matches the oracle."""
    import torch
    from paper_2109_06976_amd import build
    if plan_name == "six_robots_oversubscribed":
        robots = build.mixed_sets()[1]
        plan = [(0, 1500), (1, 1100), (2, 300), (4, 77), (5, 9), (3, 0), (0, 3)]
    else:
        robots = build.mixed_sets()[0]
        plan = [(0, 1024), (1, 613)]
    say(f"[gpu] mixed persistent vs one launch: {plan_name} {plan}")
    mx = grid.Mixed(robots)
    models = [grid.Model(r) for r in robots]
    try:
        items, knots = _mixed_items(torch, models, plan, 900)
        results = {}
        for mode in (grid.MIXED_ONE_LAUNCH, grid.MIXED_PERSISTENT, grid.MIXED_PER_ROBOT):
            for it in items:
                for t in it[4:]:
                    t.fill_(float("nan"))
            say(f"  mode {grid.MIXED_MODES[mode]}")
            mx.launch(items, mode=mode)
            torch.cuda.synchronize()
            results[mode] = [[t.cpu().numpy() for t in it[4:]] for it in items]
        for j, (r, N) in enumerate(plan):
            for k, a, b in zip(OUTS, results[grid.MIXED_ONE_LAUNCH][j],
                               results[grid.MIXED_PERSISTENT][j]):
                np.testing.assert_array_equal(b, a, err_msg=f"{robots[r].name} N={N} {k}")
            if N == 0 or (getattr(robots[r], "joint_type", None) is not None and
                          (robots[r].joint_type == grid.JOINT_FIXED).any()):
                continue                     # the locked-joint oracle covers these robots
            ref = orc.fd_grad_batch(robots[r], knots[j].q, knots[j].qd, knots[j].tau)
            tol = {"qdd": 1e-4, "Minv": 1e-3, "dqdd_dq": 1e-3, "dqdd_dqd": 1e-3}
            for mode in (grid.MIXED_PERSISTENT, grid.MIXED_PER_ROBOT):
                for k, g in zip(OUTS, results[mode][j]):
                    y = g.astype(np.float64).reshape(N, -1)
                    w = ref[k].reshape(N, -1)
                    scale = np.abs(w).max(1)
                    err = (np.abs(y - w).max(1) / np.where(scale > 0, scale, 1.0)).max()
                    assert err <= tol[k], (robots[r].name, N, k, grid.MIXED_MODES[mode], err)
        # the tuner times the three modes on these items and keeps one for this size
        chosen, us = mx.tune(items)
        say(f"  tuned: {grid.MIXED_MODES[chosen]} ({', '.join(f'{grid.MIXED_MODES[m]} {t:.1f} us' for m, t in us.items())})")
        assert chosen in (0, 1, 2) and all(t > 0 for t in us.values())
        with pytest.raises(grid.GridError) as e:
            mx.launch(items, mode=3)
        assert e.value.status == grid.GRID_EINVAL
    finally:
        mx.close()
        for m in models:
            m.close()


@pytest.mark.parametrize("mode", [None, grid.MIXED_ONE_LAUNCH, grid.MIXED_PERSISTENT,
                                  grid.MIXED_PER_ROBOT])
def test_mixed_launch_graph_replays_and_updates(mode):
    """One mixed launch captured in a hipGraph (grid_mixed_graph_create): every replay, with
    eager work and synchronisations between replays, equals the eager launch in the same mode
    bit for bit; after grid_mixed_graph_update to other items (another count, other N) the
    replays equal the eager launch of those items."""
    import torch
    from paper_2109_06976_amd import build
    robots = build.mixed_sets()[0]                    # quad12, chain7
    models = [grid.Model(r) for r in robots]
    mx = grid.Mixed(robots)
    label = "tuned" if mode is None else grid.MIXED_MODES[mode]
    try:
        for plan, plan2 in [([(0, 64), (1, 37)], [(1, 181), (0, 256), (1, 5)]),
                            ([(0, 1024), (1, 613)], [(0, 3)])]:
            say(f"[gpu] mixed graph ({label}): {plan} then {plan2}")
            items, _ = _mixed_items(torch, models, plan, 1100)
            mx.launch(items, mode=mode)
            torch.cuda.synchronize()
            eager = [[t.clone() for t in it[4:]] for it in items]
            g = mx.graph(items, mode=mode)
            try:
                for rep in range(3):
                    for it in items:
                        for t in it[4:]:
                            t.fill_(float("nan"))
                    torch.cuda.synchronize()
                    g.launch(torch.cuda.current_stream())
                    torch.cuda.synchronize()
                    for it, ref in zip(items, eager):
                        for k, a, b in zip(OUTS, it[4:], ref):
                            assert torch.equal(a, b), f"replay {rep} {k}"
                    _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between
                items2, _ = _mixed_items(torch, models, plan2, 1200)
                mx.launch(items2, mode=mode)
                torch.cuda.synchronize()
                eager2 = [[t.clone() for t in it[4:]] for it in items2]
                g.update(items2)
                for rep in range(2):
                    for it in items2:
                        for t in it[4:]:
                            t.fill_(float("nan"))
                    g.launch(torch.cuda.current_stream())
                    torch.cuda.synchronize()
                    for it, ref in zip(items2, eager2):
                        for k, a, b in zip(OUTS, it[4:], ref):
                            assert torch.equal(a, b), f"updated replay {rep} {k}"
            finally:
                g.close()
        # an unknown mode is rejected
        with pytest.raises(grid.GridError) as e:
            mx.graph(items, mode=7)
        assert e.value.status == grid.GRID_EINVAL
    finally:
        mx.close()
        for m in models:
            m.close()
