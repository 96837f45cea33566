#!/usr/bin/env python3
"""Benchmark: gradient of forward dynamics, knot-evals/s, 7-DoF chain, N = 128 knots.

One step = one batched call of the whole path (transforms, RNEA, M and its factor,
M^-1, qdd, RNEA at qdd, dRNEA forward and backward, -M^-1 dtau) over 128 knot points, as
one fused kernel launch, with inputs and outputs resident in device memory. Prints one
JSON line.

Also reported (extra fields of the same line):
  plain         the staged pipeline (five launches, intermediates in device memory) on
                the same batch, and fused_vs_plain = plain step time / fused step time;
  roofline      the fused kernel's algorithmic FLOP rate against the FP32 vector peak,
                from HIP-event kernel durations measured here;
  builds        each build of the fused kernel at this N, and the autotuner's choices
                (the timed steps run the tuned build);
  io_inclusive  the host call on pinned buffers (H2D + kernel + D2H by copy engines; the
                mapped call with no copy engines; the pageable-array call);
  served        p50/p99 latency and throughput of an open-loop Poisson request stream
                (20k req/s over the three robots) through the continuous-batching
                server, and through one plain staged launch per request;
  mixed         quad12 + chain7 batches at uneven knot counts per step: two calls, one
                batch call, one hipGraph launch;
  autograd      the humanoid autograd workload (forward + backward per step) with the
                stored-Jacobian and the reverse-sweep backward, eager and graph-replayed;
  single_knot_us  one knot (N = 1) of ID, M^-1, FD, dID and dFD on each robot, as the
                paper's single-computation table, with the paper's GPU numbers as context;
  minv_routes_us  M^-1 alone by the factorisation (quad layout, one lane per knot) and by
                the paper's direct inverse (one lane per knot), per robot and knot count;
  sweep         the headline robot at larger batches (tuned build per size);
  sweep_robots  quad12 and humanoid30 at large batches, each model tuned at those sizes;
  cpu_baseline  the FP64 oracle on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector (published)
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused.json")


FLOPS_FILE = os.path.join(ROOT, "profiles", "flops_per_knot.json")


def algorithmic_flops(robot: str) -> int:
    """FLOPs per knot of the path, counted on the oracle's formulation by an instrumented
    replay of its steps (the stored record; recomputed by the command it names)."""
    return int(json.load(open(FLOPS_FILE))["robots"][robot]["total"])


def measured_counters(workload: str, kernel: str, code_hash: str):
    """The committed rocprofv3 counter record (HBM bytes and VALU instructions per launch)
    for this kernel and workload, if it was taken on the same machine code (the hash of the
    model's loaded code object)."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return {}
    entry = rec.get(workload)
    if not entry or entry.get("code_hash") != code_hash or entry.get("kernel") != kernel:
        return {}
    return entry


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--robot", default="chain7")
    ap.add_argument("--knots", type=int, default=128)
    ap.add_argument("--seed", type=int, default=102)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bounded CPU sample for the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-io", action="store_true")
    ap.add_argument("--sweep", default=",".join(map(str, synth_throughput_knots())),
                    help="comma-separated extra knot counts to time (\"\" for none)")
    ap.add_argument("--sweep-robots",
                    default=";".join(f"{r}:{','.join(map(str, ns))}"
                                     for r, ns in synth_robot_sweep().items()),
                    help="robot:knot counts;... timed like the sweep on their own models, "
                         "with the sweep (none when --sweep is \"\")")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="measured seconds of the served load (0 disables serving)")
    ap.add_argument("--serve-rate", type=float, default=20000.0)
    ap.add_argument("--serve-sweep", default="5000,10000,40000",
                    help="extra request rates, comma-separated")
    ap.add_argument("--serve-sweep-seconds", type=float, default=3.0,
                    help="measured seconds per extra rate")
    ap.add_argument("--serve-contexts", type=int, default=2,
                    help="batch contexts per model of the batched server")
    ap.add_argument("--serve-window-us", type=int, default=60,
                    help="batch window of the batched server (microseconds)")
    ap.add_argument("--serve-min-knots", type=int, default=512,
                    help="knots at which a waiting batch launches before its window closes")
    ap.add_argument("--no-io-sweep", action="store_true",
                    help="skip the per-robot batch-size sweep with host transfers")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-knot latency table (ID, Minv, FD, dID, dFD at N = 1)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-batch leg (quad12 + chain7 in one step)")
    ap.add_argument("--no-autograd", action="store_true",
                    help="skip the autograd leg (humanoid forward + backward)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (untuned build choice)")
    ap.add_argument("--build", type=int, default=-1,
                    help="pin one build of the fused kernel (skips the per-build timings and "
                         "the autotuner; used for profiling one kernel)")
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="also run a plain device copy of this size (for counter scaling)")
    return ap.parse_args()


def progress(msg):
    """One line per finished leg on stderr (the JSON result line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(torch, launch, steps, warmup):
    """Wall time per step (barrier + synchronize on both sides) and GPU time per launch
    from a HIP event pair on the launch stream around the same back-to-back launches."""
    for _ in range(warmup):
        launch()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        launch()
    end.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return wall, start.elapsed_time(end) * 1e-3 / steps


# the paper's single-computation GPU latencies (Table I; RTX 3080, microseconds): context
PAPER_TABLE1_GPU_US = {
    "chain7": {"ID": 3.0, "Minv": 5.2, "FD": 7.7, "dID": 6.3, "dFD": 12.9},
    "quad12": {"ID": 3.2, "Minv": 5.6, "FD": 6.9, "dID": 5.8, "dFD": 11.0},
    "humanoid30": {"ID": 8.0, "Minv": 17.4, "FD": 22.4, "dID": 19.5, "dFD": 42.1},
}


def single_knot_table(torch, grid, synth, steps):
    """Latency of one knot (N = 1) for each algorithm on each robot: HIP-event time per
    launch over back-to-back launches, as the paper's single-computation table."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    table = {}
    for name in ("chain7", "quad12", "humanoid30"):
        robot = synth.model_by_name(name)
        n = robot.n
        m = grid.Model(robot)
        k = synth.random_knots(n, 1, 9)
        q, qd, tau = (torch.from_numpy(a).to(dev) for a in (k.q, k.qd, k.tau))
        v = [torch.empty((1, n), device=dev) for _ in range(2)]
        mats = [torch.empty((1, n, n), device=dev) for _ in range(3)]
        ops = {
            "ID": lambda: m.id(q, qd, tau, v[0], N=1, stream=stream),
            "Minv": lambda: m.minv(q, mats[0], N=1, stream=stream),
            "FD": lambda: m.fd(q, qd, tau, v[0], N=1, stream=stream),
            "dID": lambda: m.id_grad(q, qd, tau, mats[0], mats[1], N=1, stream=stream),
            "dFD": lambda: m.fd_grad(q, qd, tau, v[1], *mats, N=1, stream=stream),
        }
        table[name] = {op: round(time_steps(torch, f, steps, 100)[1] * 1e6, 3)
                       for op, f in ops.items()}
        m.close()
    return table


def minv_routes(torch, grid, synth):
    """M^-1 alone by its three routes (grid_minv_route): the quad layout's factorisation, and
    one lane per knot with composite bodies + L^T L or with the paper's direct articulated-body
    inverse; HIP-event time per launch over back-to-back launches, per robot and knot count."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    names = {grid.MINV_QUAD: "quad_ltl", grid.MINV_LANE_LTL: "lane_ltl",
             grid.MINV_LANE_DIRECT: "lane_direct"}
    out = {"workload": "M^-1 only, us per launch (HIP events, back to back)"}
    for name in ("chain7", "quad12", "humanoid30"):
        robot = synth.model_by_name(name)
        m = grid.Model(robot)
        res = {}
        for N in (1, 128, 16384, 65536):
            q = torch.from_numpy(synth.random_knots(robot.n, N, 11).q).to(dev)
            mi = torch.empty((N, robot.n, robot.n), device=dev)
            steps = 1000 if N <= 128 else 100
            res[str(N)] = {
                label: round(time_steps(torch, lambda r=route: m.minv_route(q, mi, r, N=N,
                                                                           stream=stream),
                                        steps, 20)[1] * 1e6, 3)
                for route, label in names.items()}
            del q, mi
        out[name] = res
        m.close()
    return out


def synth_throughput_knots():
    from paper_2109_06976_amd import synth
    return synth.THROUGHPUT_KNOTS


def synth_robot_sweep():
    from paper_2109_06976_amd import synth
    return synth.ROBOT_THROUGHPUT_KNOTS


def robot_sweeps(torch, grid, synth, args):
    """Other robots at large batches: each model tuned over its sizes, then every size timed
    on the tuned build like the headline sweep (HIP events, back-to-back launches)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}
    for spec in args.sweep_robots.split(";"):
        name, ns = spec.split(":")
        ns = [int(x) for x in ns.split(",") if x]
        robot = synth.model_by_name(name)
        n = robot.n
        model = grid.Model(robot, device=0)
        grid.tune(model, ns)
        res = {}
        for NK in ns:
            k = synth.random_knots(n, NK, args.seed + NK)
            ins = [torch.from_numpy(a).to(dev) for a in (k.q, k.qd, k.tau)]
            outs = [torch.empty((NK, n), device=dev)] + \
                [torch.empty((NK, n, n), device=dev) for _ in range(3)]
            call = model.fd_grad_call(*ins, *outs, N=NK, stream=stream)
            s, a = time_steps(torch, call, max(200, args.steps // 5), 50)
            res[str(NK)] = {"knot_evals_per_s": NK / s, "ms_per_step": s * 1e3,
                            "kernel_avg_us": a * 1e6,
                            "kernel": grid.BUILD_KERNELS[grid.build_for(model, NK)],
                            "alu_frac": algorithmic_flops(name) * NK / a / 1e12 / PEAK_FP32_TFLOPS}
            del ins, outs, call
        model.close()
        out[name] = res
    return out


def autograd_steps(torch, grid, synth, steps):
    """The autograd workload (humanoid, N = 128 knots as two 64-knot trajectories,
    L = sum of squared qdd): time per forward + backward step, for the stored-Jacobian and
    the reverse-sweep backward."""
    from paper_2109_06976_amd.autograd import CapturedStep, forward_dynamics
    dev = torch.device("cuda:0")
    robot = synth.humanoid30()
    m = grid.Model(robot)
    kn = synth.random_knots(robot.n, 128, 104)
    leaves = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in (kn.q, kn.qd, kn.tau)]
    out = {}
    for mode in ("jacobians", "adjoint"):
        def step():
            for x in leaves:
                x.grad = None
            qdd = forward_dynamics(m, *leaves, mode=mode)
            (qdd * qdd).sum().backward()
        wall, _ = time_steps(torch, step, steps, 20)
        out[mode] = {"us_per_step": round(wall * 1e6, 2),
                     "knot_evals_per_s": round(128 / wall, 1)}
        # the same step captured once in a HIP graph and replayed (host cost of one launch)
        captured = CapturedStep(m, *leaves, mode=mode)
        wall, _ = time_steps(torch, captured.replay, steps, 20)
        out[mode + "_graph"] = {"us_per_step": round(wall * 1e6, 2),
                                "knot_evals_per_s": round(128 / wall, 1)}
        del captured
    m.close()
    return {"workload": "humanoid30, N=128 (2 x 64 knots), L = sum |qdd|^2, forward + backward "
                        "(eager through torch, and the step captured in a HIP graph)",
            **out}


def mixed_batches(torch, grid, synth, chain_model, steps):
    """Quad12 and chain7 batches at uneven knot counts in one step, issued several ways: two
    fd_grad calls, one grid_fd_grad_batch call, the items' kernels captured as one hipGraph,
    the module holding both robots (grid_mixed) in each of its three modes (one launch,
    persistent, per robot), and its one-launch and persistent launches captured in a
    hipGraph; then the module's tuner's choice."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    quad = grid.Model(synth.quad12())
    mixed = grid.Mixed([synth.quad12(), synth.chain7()])
    out = {"workload": "quad12 + chain7 at uneven knot counts in one step (knot-evals/s over "
                       "both robots)",
           "resident_workgroups_note": "persistent: resident workgroups of the mixed kernel "
                                       "stride over the blocks, largest branches first"}
    for nq, nc in synth.MIXED_PLANS:
        items = []
        for m, n, NK, seed in ((quad, 12, nq, 300 + nq), (chain_model, 7, nc, 400 + nc)):
            k = synth.random_knots(n, NK, seed)
            ins = [torch.from_numpy(a).to(dev) for a in (k.q, k.qd, k.tau)]
            outs = [torch.empty((NK, n), device=dev)] + \
                [torch.empty((NK, n, n), device=dev) for _ in range(3)]
            items.append((m, *ins, *outs))
        calls = [it[0].fd_grad_call(*it[1:], stream=stream) for it in items]

        def separate():
            for c in calls:
                c()

        graph = grid.Graph(items)
        table = [(r, *it[1:]) for r, it in enumerate(items)]   # robot 0: quad12, 1: chain7
        res = {}
        modes = [(grid.MIXED_MODES[m], mixed.launch_call(table, stream=stream, mode=m))
                 for m in (grid.MIXED_ONE_LAUNCH, grid.MIXED_PERSISTENT, grid.MIXED_PER_ROBOT)]
        # one mixed launch (one-launch and persistent forms) captured in a hipGraph
        mgraphs = {m: mixed.graph(table, mode=m)
                   for m in (grid.MIXED_ONE_LAUNCH, grid.MIXED_PERSISTENT)}
        modes += [("graph_" + grid.MIXED_MODES[m], g.launch_call(stream=stream))
                  for m, g in mgraphs.items()]
        for label, fn in [("two_calls", separate),
                          ("batch_call", lambda: grid.fd_grad_batch(items, stream=stream)),
                          ("graph", lambda: graph.launch(stream=stream))] + modes:
            wall, gpu = time_steps(torch, fn, steps, 50)
            res[label] = {"us_per_step": round(wall * 1e6, 3), "gpu_us": round(gpu * 1e6, 3),
                          "knot_evals_per_s": round((nq + nc) / wall, 1)}
        # the module's tuner times the three mixed modes and keeps one for this size
        chosen, us = mixed.tune(table)
        res["tuned"] = {"mode": grid.MIXED_MODES[chosen],
                        "tuner_us": {grid.MIXED_MODES[m]: round(t, 3) for m, t in us.items()}}
        graph.close()
        for g in mgraphs.values():
            g.close()
        out[f"{nq}+{nc}"] = res
    mixed.close()
    quad.close()
    return out


def io_sweep(torch, grid, synth, reps):
    """The paper's multiple-computation sweep (Sec. V-B, Fig. 4) on each robot: per batch size,
    the fused kernel with inputs resident in device memory (compute only), and the host call on
    the workspace's pinned buffers split into H2D / kernel / D2H (HIP events), the same call
    cut into overlapping pieces, the mapped call (no copy engines: the kernel reads the pinned
    inputs, a copy kernel or the fused kernel itself writes the pinned outputs), and the call on
    pageable host arrays (staged through the pinned buffers)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {"workload": "gradient of forward dynamics per robot and batch size; compute only "
                       "(device-resident) and with host transfers"}
    for name in ("chain7", "quad12", "humanoid30"):
        robot = synth.model_by_name(name)
        n = robot.n
        m = grid.Model(robot)
        tuned = grid.tune(m, list(synth.SWEEP_KNOTS))
        ws = grid.Workspace(m, max(synth.SWEEP_KNOTS))
        rows = {}
        for N in synth.SWEEP_KNOTS:
            kn = synth.random_knots(n, N, 500 + N)
            ins = [torch.from_numpy(a).to(dev) for a in (kn.q, kn.qd, kn.tau)]
            outs = [torch.empty((N, n), device=dev)] + \
                [torch.empty((N, n, n), device=dev) for _ in range(3)]
            call = m.fd_grad_call(*ins, *outs, stream=stream)
            wall, gpu = time_steps(torch, call, reps, 50)
            pin_in, _ = ws.host_buffers(N)
            pin_in["q"][:], pin_in["qd"][:], pin_in["tau"][:] = kn.q, kn.qd, kn.tau
            legs = {}
            for pieces in (1, 2, 4):
                for _ in range(10):
                    ws.fd_grad_pinned(N, pieces)
                acc = {"h2d_ms": 0.0, "kernel_ms": 0.0, "d2h_ms": 0.0, "total_ms": 0.0}
                t0 = time.perf_counter()
                for _ in range(reps):
                    t = ws.fd_grad_pinned(N, pieces)
                    for k in acc:
                        acc[k] += t[k]
                legs[pieces] = {"wall_us": (time.perf_counter() - t0) / reps * 1e6,
                                **{k.replace("_ms", "_us"): v / reps * 1e3
                                   for k, v in acc.items()}}
            # no copy engines: the kernel reads the pinned inputs through the device mapping,
            # the outputs go out by a copy kernel or by the fused kernel's own stores
            # (wall time of untimed calls; device phases from timed calls)
            mapped = {}
            for label, mode in (("copy_kernel", grid.IO_COPY_KERNEL), ("direct", grid.IO_DIRECT)):
                for _ in range(10):
                    ws.fd_grad_mapped(N, mode, timed=False)
                t0 = time.perf_counter()
                for _ in range(reps):
                    ws.fd_grad_mapped(N, mode, timed=False)
                w_m = (time.perf_counter() - t0) / reps
                acc = {"kernel_ms": 0.0, "d2h_ms": 0.0, "total_ms": 0.0}
                for _ in range(reps):
                    t = ws.fd_grad_mapped(N, mode)
                    for k in acc:
                        acc[k] += t[k]
                mapped[label] = {"wall_us": round(w_m * 1e6, 2),
                                 **{k.replace("_ms", "_us").replace("d2h", "copy"):
                                    round(v / reps * 1e3, 2) for k, v in acc.items()}}
            one = legs[1]
            best = min(legs, key=lambda k: legs[k]["wall_us"])
            best_mapped = min(mapped, key=lambda k: mapped[k]["wall_us"])
            for _ in range(10):
                ws.fd_grad_host(kn.q, kn.qd, kn.tau)
            t0 = time.perf_counter()
            for _ in range(reps):
                ws.fd_grad_host(kn.q, kn.qd, kn.tau)
            pageable = (time.perf_counter() - t0) / reps * 1e6
            rows[str(N)] = {
                "build": grid.BUILD_KERNELS[tuned[N]],
                "compute_knot_evals_per_s": N / wall, "kernel_us": gpu * 1e6,
                "alu_frac": algorithmic_flops(name) * N / gpu / 1e12 / PEAK_FP32_TFLOPS,
                "step_us": wall * 1e6,
                "pinned": {k: round(v, 2) for k, v in one.items()},
                "io_share": (one["h2d_us"] + one["d2h_us"]) / one["total_us"],
                "overlapped": {"pieces": best, "wall_us": round(legs[best]["wall_us"], 2),
                               "device_us": round(legs[best]["total_us"], 2)},
                "with_io_knot_evals_per_s": N / (legs[best]["wall_us"] * 1e-6),
                "mapped": mapped,
                "mapped_knot_evals_per_s": N / (mapped[best_mapped]["wall_us"] * 1e-6),
                "pageable_wall_us": round(pageable, 2),
            }
        ws.close()
        m.close()
        out[name] = rows
    return out


def serve(args, grid, synth, chain_model=None):
    """Open-loop Poisson requests over the three robots (50/30/20 %, N ~ U{16..256}),
    served with continuous batching and, as the baseline, one staged launch per request."""
    robots = [synth.chain7(), synth.quad12(), synth.humanoid30()]
    models = [chain_model or grid.Model(robots[0]), grid.Model(robots[1]), grid.Model(robots[2])]
    probs = [0.5, 0.3, 0.2]
    # the server's launches run the build each model's tuning picks for the batch's knot
    # count: tune at the batch sizes it can launch (requests of 16-256 knots, batches up to
    # 2048); untuned, a batch beyond one wavefront per SIMD would take the lane layout
    batch_ns = [16, 32, 64, 128, 256, 512, 1024, 2048]
    tuned_builds = {rb.name.split("-")[0]: {str(k): grid.BUILD_KERNELS[v]
                                            for k, v in grid.tune(m, batch_ns).items()}
                    for rb, m in zip(robots, models)}
    out = {"workload": "Poisson arrivals, chain7/quad12/humanoid30 at 50/30/20 %, "
                       "N ~ U{16..256}, latency = outputs in host memory - scheduled arrival",
           "measured_s": args.serve_seconds, "warmup_s": 1.0}
    rates = [args.serve_rate] + [float(x) for x in args.serve_sweep.split(",")
                                 if x and float(x) != args.serve_rate]
    out["tuned_builds"] = tuned_builds
    out["policy"] = {"contexts_per_model": args.serve_contexts,
                     "batch_window_us": args.serve_window_us,
                     "min_batch_knots": args.serve_min_knots}
    # batched: fused launches reading and writing the pinned staging through the device mapping;
    # batched_in_place: the clients' arrays are pinned and registered, and a batch of one request
    # runs on them directly (no staging copy, no copy-out);
    # batched_copy_engines: the staged form with H2D / D2H copies (at the headline rate only);
    # per_request_plain: one staged launch per request with ordinary copies (the baseline)
    mapped, direct = grid.GRID_SERVER_MAPPED_IO, grid.GRID_SERVER_DIRECT_PINNED
    for label, flags, lrates, pinned in (
            ("batched", mapped, rates, False),
            ("batched_in_place", mapped | direct, rates, True),
            ("batched_copy_engines", 0, rates[:1], False),
            ("per_request_plain", grid.GRID_SERVER_PER_REQUEST, rates, False)):
        batched = not flags & grid.GRID_SERVER_PER_REQUEST
        srv = grid.Server(models, budget_bytes=1 << 30, max_batch_knots=2048,
                          contexts_per_model=args.serve_contexts if batched else 3, flags=flags,
                          batch_window_us=args.serve_window_us if batched else 0,
                          min_batch_knots=args.serve_min_knots if batched else 0)
        res = {}
        for rate in lrates:
            secs = args.serve_seconds if rate == args.serve_rate else args.serve_sweep_seconds
            r = srv.loadgen(rate, secs, probs, n_min=16, n_max=256, warmup_s=1.0, seed=7,
                            pinned=pinned)
            progress(f"served {label} at {int(rate)} req/s: p50 {r['p50_us']:.0f} us, "
                     f"p99 {r['p99_us']:.0f} us, {r['requests_per_launch']:.2f} requests/launch")
            res[str(int(rate))] = {"p50_us": r["p50_us"], "p90_us": r["p90_us"],
                                   "p99_us": r["p99_us"], "max_us": r["max_us"],
                                   "requests_per_launch": round(r["requests_per_launch"], 3),
                                   "p50_split_us": {k.replace("_us", ""): round(v, 2)
                                                    for k, v in r["p50_split"].items()},
                                   "p99_split_us": {k.replace("_us", ""): round(v, 2)
                                                    for k, v in r["p99_split"].items()},
                                   "per_model": {
                                       rb.name.split("-")[0]: {
                                           "requests": r["model_requests"][k],
                                           "p50_us": round(r["model_p50_us"][k], 1),
                                           "p99_us": round(r["model_p99_us"][k], 1)}
                                       for k, rb in enumerate(robots)},
                                   "measured_s": secs,
                                   "requests_per_s": r["requests"] / r["seconds"],
                                   "knot_evals_per_s": r["knots"] / r["seconds"]}
        st = srv.stats()
        res["launches"] = st["launches"]
        if pinned:
            res["in_place_launches"] = st["inplace_launches"]
        srv.close()
        out[label] = res
    for m in models[1:] + ([] if chain_model else models[:1]):
        m.close()
    return out


def host_cpu():
    """Host CPU model, physical cores (distinct (core, socket) pairs of lscpu) and the logical
    CPUs this process may run on."""
    import subprocess
    model, phys = "", None
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True,
                             check=True).stdout
        phys = len({ln for ln in out.splitlines() if ln and not ln.startswith("#")})
        info = subprocess.run(["lscpu"], capture_output=True, text=True, check=True).stdout
        for ln in info.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except (OSError, subprocess.CalledProcessError):
        pass
    return model, phys, len(os.sched_getaffinity(0))


def cpu_baseline(args, robot, kn, synth):
    """The FP64 oracle (steps of the path: transforms, RNEA, CRBA, Cholesky M^-1, FD, the
    analytic dRNEA, -M^-1 dtau) as the CPU baseline: built here with -O3 -march=native for
    this host, OpenMP over the knots of a batch, timed with CLOCK_MONOTONIC per batch call at
    one thread and at every CPU this job may use, on the benchmark's batch; then the same
    multi-threaded timing for each robot at the sweep sizes."""
    import tempfile
    import numpy as np
    from oracle import build as oracle_build
    from oracle import oracle as orc
    path = os.path.join(tempfile.mkdtemp(prefix="grid_oracle_timing_"), "liboracle_timing.so")
    cmd = oracle_build.build_timing(path)
    orc.use_library(path)
    model_name, phys, avail = host_cpu()
    threads = avail
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        threads = min(threads, int(env))

    def timed(om, q, qd, tau, seconds, min_reps):
        orc.fd_grad_batch(om, q, qd, tau)
        times = []
        t_end = time.monotonic() + seconds
        while time.monotonic() < t_end or len(times) < min_reps:
            t0 = time.monotonic()
            orc.fd_grad_batch(om, q, qd, tau)
            times.append(time.monotonic() - t0)
        return float(np.mean(times)), float(np.median(times)), len(times)

    om = orc.OracleModel(robot)
    q, qd, tau = (a.astype(np.float64) for a in (kn.q, kn.qd, kn.tau))
    N = q.shape[0]
    legs = {}
    for k in (1, threads):
        orc.set_num_threads(k)
        mean, med, reps = timed(om, q, qd, tau, args.cpu_seconds * (0.6 if k == 1 else 0.4),
                                10)
        legs[k] = {"knot_evals_per_s": N / mean, "mean_ms": mean * 1e3, "median_ms": med * 1e3,
                   "batches": reps}
    orc.set_num_threads(threads)
    sweep = {}
    for name in ("chain7", "quad12", "humanoid30"):
        r = synth.model_by_name(name)
        orm = orc.OracleModel(r)
        for NK in synth.SWEEP_KNOTS:
            k2 = synth.random_knots(r.n, NK, 500 + NK)
            mean, med, reps = timed(orm, *(a.astype(np.float64) for a in (k2.q, k2.qd, k2.tau)),
                                    0.4, 3)
            sweep[f"{name}-N{NK}"] = {"knot_evals_per_s": NK / mean, "mean_us": mean * 1e6,
                                      "median_us": med * 1e6}
    return {
        "value": legs[threads]["knot_evals_per_s"], "unit": "knot-evals/s", "cores": threads,
        "kind": "oracle",
        "sample": f"{legs[1]['batches']} + {legs[threads]['batches']} calls on the same "
                  f"{N}-knot {args.robot} batch at 1 and {threads} threads, then 0.4 s per "
                  "(robot, N) of the sweep; FP64 C oracle, OpenMP over knots",
        "one_thread": legs[1], "all_threads": legs[threads], "sweep": sweep,
        "host": {"cpu": model_name, "physical_cores": phys, "cpus_available": avail,
                 "omp_num_threads_env": env or None},
        "build": cmd.replace(path + ".tmp", "<timing build>"),
        "timer": "CLOCK_MONOTONIC (time.monotonic) around each batch call; mean and median"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU (--gpus 1): the batched gradient of forward dynamics "
              "shards knots across GPUs with no exchange, so a multi-GPU figure is N times "
              "one GPU's share and is not measured here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2109_06976_amd import flops, grid, synth

    robot = synth.model_by_name(args.robot)
    n, N = robot.n, args.knots
    kn = synth.random_knots(n, N, args.seed)
    dev = torch.device("cuda:0")
    model = grid.Model(robot, device=0)
    stream = torch.cuda.current_stream(dev)

    def buffers(NK, seed):
        k = synth.random_knots(n, NK, seed)
        ins = [torch.from_numpy(a).to(dev) for a in (k.q, k.qd, k.tau)]
        outs = [torch.empty((NK, n), device=dev), torch.empty((NK, n, n), device=dev),
                torch.empty((NK, n, n), device=dev), torch.empty((NK, n, n), device=dev)]
        return ins, outs

    ins, outs = buffers(N, args.seed)

    def launch_for(ins_, outs_, NK):
        # the call bound to its buffers (arguments converted to C once, as a loop over
        # preallocated buffers would): every step is still one grid_fd_grad call
        return model.fd_grad_call(*ins_, *outs_, N=NK, stream=stream)

    launch = launch_for(ins, outs, N)
    sweep_ns = [int(x) for x in args.sweep.split(",") if x]

    # every build of the fused kernel at this N (pinned one at a time), then the autotuner
    # over the sizes this run times; the timed steps use the tuned choice
    builds, tuned = {}, None
    if args.build >= 0:
        grid.tune_apply(model, {1 << 22: args.build})
    else:
        for b, name in enumerate(grid.BUILD_KERNELS):
            grid.tune_apply(model, {1 << 22: b})
            st, ks = time_steps(torch, launch, max(200, args.steps // 10), 50)
            builds[name] = {"us_per_step": round(st * 1e6, 3),
                            "kernel_avg_us": round(ks * 1e6, 3)}
        grid.tune_apply(model, {})
        if not args.no_tune:
            tuned = grid.tune(model, sorted(set([N] + sweep_ns)))
    build = grid.build_for(model, N)
    progress(f"builds timed, tuned {tuned}")

    sec_per_step, kernel_s = time_steps(torch, launch, args.steps, args.warmup)
    avg_ms = kernel_s * 1e3

    # the floor of this measurement: a one-element fill kernel timed the same way
    tiny = torch.zeros(1, device=dev)
    floor_step, floor_gpu = time_steps(torch, lambda: tiny.fill_(1.0), max(200, args.steps // 5), 50)

    # the plain staged pipeline (five launches, intermediates in HBM) on the same batch
    ws_plain = grid.Workspace(model, N)
    plain = lambda: ws_plain.fd_grad_staged(*ins, *outs, N=N, stream=stream)
    plain_step, plain_gpu = time_steps(torch, plain, max(200, args.steps // 5), 50)
    ws_plain.close()
    progress("headline and plain pipeline timed")

    fl = {"total": algorithmic_flops(args.robot)}
    kernel_tally = flops.fdgrad_flops(robot.parent)["total"]
    flop_launch = fl["total"] * N
    achieved_tflops = flop_launch / (avg_ms * 1e-3) / 1e12
    workload = f"{args.robot}-N{N}"
    counters = measured_counters(workload, grid.BUILD_KERNELS[build], model.code_hash)
    traffic = counters.get("bytes_per_launch")
    executed = counters.get("executed_fp32_flop_per_launch")
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 4), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_TFLOPS,
                "traffic": traffic,
                "kernel": grid.BUILD_KERNELS[build], "kernel_avg_us": round(avg_ms * 1e3, 3),
                "flop_per_knot": fl["total"],
                "flop_per_knot_source": "oracle formulation, instrumented "
                                        "(profiles/flops_per_knot.json)",
                "flop_per_knot_kernel_tally": kernel_tally,
                "hbm_bytes_per_launch": flops.io_bytes_per_knot(n) * N,
                "hbm_frac": flops.io_bytes_per_knot(n) * N / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "launch_floor_us": round(floor_gpu * 1e6, 3),
                "code_hash": model.code_hash,
                # FP32 FLOP the kernel executes per launch (rocprofv3 VALU instruction counters
                # over all 64 lanes; counts the layout's redundant work), and its rate
                "executed_flop_per_launch": executed,
                "executed_tflops": (round(executed / (avg_ms * 1e-3) / 1e12, 4)
                                    if executed else None)}

    result = {
        "metric": "dFD knot-evals/sec (7-DoF chain, N=128) + p50/p99 latency served, vs plain",
        "value": N / sec_per_step,
        "unit": "knot-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.robot}: {n}-joint fixed-base robot, N={N} knots, "
                               "fused kernel, device-resident inputs",
                   "robot": args.robot, "knots": N, "lanes_per_knot": model.lanes_per_knot},
        "roofline": roofline,
        "plain": {"value": N / plain_step, "unit": "knot-evals/s", "ms_per_step": plain_step * 1e3,
                  "gpu_us_per_step": plain_gpu * 1e6,
                  "note": "staged pipeline: 5 launches (RNEA, M^-1, qdd, dRNEA, dFD), "
                          "intermediates through device memory"},
        "fused_vs_plain": plain_step / sec_per_step,
        "builds": builds,
        "tuned": tuned,
    }

    if not args.no_io:
        ws = grid.Workspace(model, N)
        reps = 500
        pin_in, _ = ws.host_buffers(N)
        pin_in["q"][:], pin_in["qd"][:], pin_in["tau"][:] = kn.q, kn.qd, kn.tau
        for _ in range(20):
            ws.fd_grad_pinned(N)
        tot = {"h2d_ms": 0.0, "kernel_ms": 0.0, "d2h_ms": 0.0, "total_ms": 0.0}
        t0 = time.perf_counter()
        for _ in range(reps):
            t = ws.fd_grad_pinned(N)
            for k in tot:
                tot[k] += t[k]
        wall = (time.perf_counter() - t0) / reps
        mapped = {}
        for label, mode in (("copy_kernel", grid.IO_COPY_KERNEL), ("direct", grid.IO_DIRECT)):
            for _ in range(20):
                ws.fd_grad_mapped(N, mode, timed=False)
            t0 = time.perf_counter()
            for _ in range(reps):
                ws.fd_grad_mapped(N, mode, timed=False)
            w_m = (time.perf_counter() - t0) / reps      # untimed calls
            acc = {"kernel_ms": 0.0, "d2h_ms": 0.0, "total_ms": 0.0}
            for _ in range(reps):
                t = ws.fd_grad_mapped(N, mode)
                for k in acc:
                    acc[k] += t[k]
            mapped[label] = {"value": N / w_m, "wall_ms_per_call": w_m * 1e3,
                             **{k.replace("d2h", "copy"): v / reps for k, v in acc.items()}}
        for _ in range(20):
            ws.fd_grad_host(kn.q, kn.qd, kn.tau)
        t0 = time.perf_counter()
        for _ in range(reps):
            ws.fd_grad_host(kn.q, kn.qd, kn.tau)
        wall_pageable = (time.perf_counter() - t0) / reps
        ws.close()
        result["io_inclusive"] = {
            "value": N / wall, "unit": "knot-evals/s", "wall_ms_per_call": wall * 1e3,
            **{k: v / reps for k, v in tot.items()},
            "mapped": mapped,
            "pageable": {"value": N / wall_pageable, "wall_ms_per_call": wall_pageable * 1e3},
            "note": "host call on the workspace's pinned buffers: H2D, kernel, D2H, wait "
                    "(pageable: the caller's arrays staged through them, Python binding "
                    "included)"}

    if not args.no_io_sweep:
        result["io_sweep"] = io_sweep(torch, grid, synth, 200)
        progress("batch-size sweep with host transfers done")

    if args.sweep:
        sweep = {}
        for NK in sweep_ns:
            i2, o2 = buffers(NK, args.seed + NK)
            l2 = launch_for(i2, o2, NK)
            s, a = time_steps(torch, l2, max(200, args.steps // 5), 50)
            sweep[str(NK)] = {"knot_evals_per_s": NK / s, "ms_per_step": s * 1e3,
                              "kernel_avg_us": a * 1e6,
                              "kernel": grid.BUILD_KERNELS[grid.build_for(model, NK)],
                              "alu_frac": fl["total"] * NK / a / 1e12 / PEAK_FP32_TFLOPS}
            del i2, o2
        result["sweep"] = sweep
        progress("throughput sweep done")

    if args.sweep and args.sweep_robots:
        result["sweep_robots"] = robot_sweeps(torch, grid, synth, args)
        progress("robot sweeps done")

    if not args.no_single:
        if args.robot == "chain7" and not args.no_mixed:
            result["mixed"] = mixed_batches(torch, grid, synth, model, 1000)
            progress("mixed batches done")
        if not args.no_autograd:
            result["autograd"] = autograd_steps(torch, grid, synth, 300)
            progress("autograd done")
        result["single_knot_us"] = single_knot_table(torch, grid, synth, 1000)
        result["single_knot_us"]["paper_table1_gpu_us"] = PAPER_TABLE1_GPU_US
        result["minv_routes_us"] = minv_routes(torch, grid, synth)
        progress("M^-1 routes timed")

    # the served load runs last: timed after it, the autograd step took about 60 us longer
    if args.serve_seconds > 0:
        result["served"] = serve(args, grid, synth, model if args.robot == "chain7" else None)
        progress("serving done")

    if args.copy_calibration_mb > 0:
        nbytes = int(args.copy_calibration_mb * 2**20)
        src = torch.ones(nbytes // 4, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 5}

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, robot, kn, synth)
        progress("cpu baseline done")

    model.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
