"""The continuous-batching server on an MI355X, through the C ABI."""
import sys
import threading

import numpy as np
import pytest

from paper_2109_06976_amd import grid, synth

pytestmark = pytest.mark.gpu

OUTS = ("qdd", "Minv", "dqdd_dq", "dqdd_dqd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def models():
    import torch
    assert torch.cuda.is_available()
    robots = [synth.chain7(), synth.quad12(), synth.humanoid30()]
    ms = [grid.Model(r) for r in robots]
    yield robots, ms
    for m in ms:
        m.close()


_alone_by_flags = {}


@pytest.mark.parametrize("flags", [0, grid.GRID_SERVER_MAPPED_IO])
def test_request_alone_equals_request_in_mix(models, orc, flags):
    """A request's outputs are the same alone and in the middle of a mixed stream (bit for
    bit), with copy-engine transfers and with mapped I/O, and the two I/O modes agree."""
    robots, ms = models
    say(f"[gpu] server identity (flags {flags}): alone vs Poisson-like mix")
    srv = grid.Server(ms, budget_bytes=1 << 28, max_batch_knots=1024, contexts_per_model=3,
                      flags=flags)
    probe = synth.random_knots(robots[2].n, 100, 55)
    t, alone = srv.submit(2, probe.q, probe.qd, probe.tau)
    srv.wait(t)
    # the same request in the middle of a stream of mixed requests from two client threads
    rng = np.random.default_rng(3)
    mixed = {}
    tickets = []

    def client(seed, count):
        r = np.random.default_rng(seed)
        for _ in range(count):
            k = int(r.choice(3, p=[0.5, 0.3, 0.2]))
            N = int(r.integers(16, 257))
            kn = synth.random_knots(robots[k].n, N, int(r.integers(1 << 30)))
            tickets.append(srv.submit(k, kn.q, kn.qd, kn.tau)[0])

    th = [threading.Thread(target=client, args=(s, 40)) for s in (1, 2)]
    for x in th:
        x.start()
    t2, mixed = srv.submit(2, probe.q, probe.qd, probe.tau)
    for x in th:
        x.join()
    srv.wait(t2)
    for t in tickets:
        srv.wait(t)
    for key in OUTS:
        np.testing.assert_array_equal(mixed[key], alone[key])
    _alone_by_flags[flags] = alone
    if len(_alone_by_flags) == 2:
        for key in OUTS:
            np.testing.assert_array_equal(_alone_by_flags[0][key],
                                          _alone_by_flags[grid.GRID_SERVER_MAPPED_IO][key])
    st = srv.stats()
    say(f"  stats {st}")
    assert st["completed"] == st["submitted"] == 82 and st["launches"] <= 82
    ref = orc.fd_grad_batch(robots[2], probe.q, probe.qd, probe.tau)
    e = np.abs(alone["qdd"] - ref["qdd"]).max(axis=1) / np.abs(ref["qdd"]).max(axis=1)
    assert e.max() <= 1e-4
    srv.close()


def test_burst_is_packed_into_few_launches(models, orc):
    # one batch context: requests that arrive while it is busy queue and go out together
    robots, ms = models
    say("[gpu] server packs a burst of 64 requests")
    srv = grid.Server(ms[:1], budget_bytes=1 << 28, max_batch_knots=4096, contexts_per_model=1)
    rng = np.random.default_rng(11)
    reqs = [synth.random_knots(7, int(rng.integers(16, 257)), 500 + i) for i in range(64)]
    tickets = [srv.submit(0, kn.q, kn.qd, kn.tau) for kn in reqs]
    for t, _ in tickets:
        srv.wait(t)
    st = srv.stats()
    say(f"  stats {st}")
    assert st["completed"] == 64 and st["launches"] < 64
    for kn, (_, out) in zip(reqs[::16], tickets[::16]):
        ref = orc.fd_grad_batch(robots[0], kn.q, kn.qd, kn.tau)
        e = np.abs(out["dqdd_dq"] - ref["dqdd_dq"]).reshape(len(kn.q), -1).max(1) / \
            np.abs(ref["dqdd_dq"]).reshape(len(kn.q), -1).max(1)
        assert e.max() <= 1e-3
    srv.close()


def test_server_matches_direct_launch(models):
    import torch
    robots, ms = models
    say("[gpu] server result = direct fused launch")
    srv = grid.Server(ms[:1], budget_bytes=1 << 26, max_batch_knots=512)
    kn = synth.random_knots(7, 77, 9)
    t, out = srv.submit(0, kn.q, kn.qd, kn.tau)
    srv.wait(t)
    d = grid.fd_grad_torch(ms[0], *(torch.from_numpy(a).cuda() for a in (kn.q, kn.qd, kn.tau)))
    torch.cuda.synchronize()
    for key in OUTS:
        np.testing.assert_array_equal(out[key], d[key].cpu().numpy())
    srv.close()


def test_admission_budget(models):
    robots, ms = models
    say("[gpu] server admission under a small budget")
    n = 7
    per_knot = 4 * (4 * n + 3 * n * n)
    srv = grid.Server(ms[:1], budget_bytes=per_knot * 300, max_batch_knots=1024,
                      contexts_per_model=2)
    kn = synth.random_knots(n, 301, 4)
    with pytest.raises(grid.GridError) as e:
        srv.submit(0, kn.q, kn.qd, kn.tau)             # can never fit
    assert e.value.status == grid.GRID_EBUSY
    tickets = []
    for k in range(30):                               # 30 x 100 knots >> budget
        a = synth.random_knots(n, 100, 100 + k)
        tickets.append(srv.submit(0, a.q, a.qd, a.tau))
    for t, out in tickets:
        srv.wait(t)
        assert np.all(np.isfinite(out["qdd"]))
    st = srv.stats()
    assert st["completed"] == 30 and st["max_inflight_bytes"] <= per_knot * 300
    srv.close()


def test_wait_timeout_and_unknown_ticket(models):
    robots, ms = models
    srv = grid.Server(ms[2:], budget_bytes=1 << 28, max_batch_knots=1024)
    kn = synth.random_knots(30, 1024, 5)
    t, _ = srv.submit(0, kn.q, kn.qd, kn.tau)
    try:
        srv.wait(t, timeout_us=0)
        finished_early = True
    except grid.GridError as e:
        assert e.status == grid.GRID_ETIMEDOUT
        finished_early = False
    if not finished_early:
        srv.wait(t)                                   # the ticket stays valid after a timeout
    with pytest.raises(grid.GridError) as e:
        srv.wait(t)                                   # released by the successful wait
    assert e.value.status == grid.GRID_EINVAL
    srv.close()


def test_destroy_with_work_in_flight(models):
    robots, ms = models
    say("[gpu] server destroy with queued and launched work")
    n = 12
    srv = grid.Server(ms[1:2], budget_bytes=4 * (4 * n + 3 * n * n) * 256, max_batch_knots=256,
                      contexts_per_model=1)
    for k in range(40):
        a = synth.random_knots(n, 200, k)
        srv.submit(0, a.q, a.qd, a.tau)
    srv.close()                                       # returns: launched work finished, rest canceled


def test_per_request_plain_mode(models, orc):
    robots, ms = models
    say("[gpu] server per-request staged mode")
    srv = grid.Server(ms, budget_bytes=1 << 28, max_batch_knots=256,
                      flags=grid.GRID_SERVER_PER_REQUEST)
    outs = []
    for k, N in ((0, 16), (1, 100), (2, 37), (0, 256)):
        kn = synth.random_knots(robots[k].n, N, 60 + k)
        t, out = srv.submit(k, kn.q, kn.qd, kn.tau)
        outs.append((k, kn, t, out))
    for k, kn, t, out in outs:
        srv.wait(t)
        ref = orc.fd_grad_batch(robots[k], kn.q, kn.qd, kn.tau)
        e = np.abs(out["dqdd_dq"] - ref["dqdd_dq"]).reshape(kn.N, -1).max(1) / \
            np.abs(ref["dqdd_dq"]).reshape(kn.N, -1).max(1)
        assert e.max() <= 1e-3
    assert srv.stats()["launches"] == 4
    srv.close()


def test_loadgen_short_run(models):
    robots, ms = models
    say("[gpu] load generator 0.5 s at 5000 req/s")
    srv = grid.Server(ms, budget_bytes=1 << 30, max_batch_knots=1024)
    r = srv.loadgen(5000, 0.5, [0.5, 0.3, 0.2], warmup_s=0.2)
    say(f"  {r}")
    assert r["requests"] > 1000 and 0 < r["p50_us"] <= r["p99_us"] <= r["max_us"]
    # where the latency goes: every phase measured, each below the whole
    assert r["requests_per_launch"] >= 1.0
    for q in ("p50_split", "p99_split"):
        sp = r[q]
        assert sp["kernel_us"] > 0 and sp["h2d_us"] > 0 and sp["d2h_us"] > 0
        assert all(0 <= v <= r["max_us"] for v in sp.values()), sp
    # per model: every model served, the counts add up, each model's percentiles ordered
    assert sum(r["model_requests"]) == r["requests"] and all(n > 0 for n in r["model_requests"])
    for k in range(3):
        assert 0 < r["model_p50_us"][k] <= r["model_p99_us"][k] <= r["max_us"]
    srv.close()
    # mapped I/O: no copy-engine phases
    srv = grid.Server(ms, budget_bytes=1 << 30, max_batch_knots=1024,
                      flags=grid.GRID_SERVER_MAPPED_IO)
    r = srv.loadgen(5000, 0.3, [0.5, 0.3, 0.2], warmup_s=0.1)
    say(f"  mapped: p50 {r['p50_us']:.0f} us, p99 {r['p99_us']:.0f} us")
    assert r["requests"] > 500 and r["p50_split"]["h2d_us"] == 0 and r["p99_split"]["d2h_us"] == 0
    assert r["p50_split"]["kernel_us"] > 0
    srv.close()


def test_batch_window_policy(models, orc):
    """With a batch window, requests that arrive while their model has a batch in flight wait
    for company (up to the window or min_batch_knots) instead of taking a free context each: a
    burst submitted faster than batches complete goes out in far fewer launches than requests,
    every result equals the direct launch on its knots within the parity tolerance, and a bad
    policy is rejected."""
    robots, ms = models
    say("[gpu] server batch window 300 us, min fill 512 knots, burst of 100 requests")
    srv = grid.Server(ms[:2], budget_bytes=1 << 28, max_batch_knots=2048, contexts_per_model=2,
                      batch_window_us=300, min_batch_knots=512)
    r = np.random.default_rng(21)
    plan = []
    for _ in range(100):
        k = int(r.integers(0, 2))
        plan.append((k, synth.random_knots(robots[k].n, int(r.integers(16, 129)),
                                           int(r.integers(1 << 30)))))
    got = []
    for k, kn in plan:                       # inputs made beforehand: the submits come in a burst
        got.append((k, kn, *srv.submit(k, kn.q, kn.qd, kn.tau)))
    for k, kn, t, out in got:
        srv.wait(t)
    st = srv.stats()
    say(f"  stats {st}")
    assert st["completed"] == 100 and st["launches"] <= 60, st
    for k, kn, t, out in got[::10]:
        ref = orc.fd_grad_batch(robots[k], kn.q, kn.qd, kn.tau)
        e = np.abs(out["dqdd_dq"] - ref["dqdd_dq"]).reshape(kn.N, -1).max(1) / \
            np.abs(ref["dqdd_dq"]).reshape(kn.N, -1).max(1)
        assert e.max() <= 1e-3
    srv.close()
    for bad in ({"batch_window_us": -1}, {"min_batch_knots": 4096}):
        with pytest.raises(grid.GridError) as e:
            grid.Server(ms[:1], budget_bytes=1 << 26, max_batch_knots=2048, **bad)
        assert e.value.status == grid.GRID_EINVAL


def test_inplace_requests_on_pinned_arrays(models, orc):
    """On a GRID_SERVER_DIRECT_PINNED server, a request whose arrays all lie in registered
    pinned ranges and that forms a batch alone runs in place (no staging copy, no copy-out):
    its outputs equal, bit for bit, the same request on ordinary arrays, and the oracle within
    the parity tolerance; an unregistered or pageable range is refused; a pinned loadgen run
    goes in place."""
    import torch
    robots, ms = models
    say("[gpu] server in place on pinned arrays")
    srv = grid.Server(ms, budget_bytes=1 << 28, max_batch_knots=1024, contexts_per_model=2,
                      flags=grid.GRID_SERVER_MAPPED_IO | grid.GRID_SERVER_DIRECT_PINNED)
    pinned = []

    def pin(shape):
        t = torch.empty(shape, dtype=torch.float32, pin_memory=True)
        srv.pin_range(t, t.numel() * 4)
        pinned.append(t)
        return t.numpy()

    try:
        with pytest.raises(grid.GridError) as e:
            srv.pin_range(np.zeros(16, np.float32), 64)          # pageable memory
        assert e.value.status == grid.GRID_EINVAL
        with pytest.raises(grid.GridError) as e:
            srv.unpin_range(np.zeros(16, np.float32))
        assert e.value.status == grid.GRID_EINVAL
        for k, N, seed in ((0, 37, 61), (2, 100, 62), (1, 256, 63)):
            n = robots[k].n
            kn = synth.random_knots(n, N, seed)
            ins = [pin((N, n)) for _ in range(3)]
            for a, b in zip(ins, (kn.q, kn.qd, kn.tau)):
                a[:] = b
            out = {"qdd": pin((N, n)), "Minv": pin((N, n, n)), "dqdd_dq": pin((N, n, n)),
                   "dqdd_dqd": pin((N, n, n))}
            for a in out.values():
                a[:] = np.nan
            before = srv.stats()["inplace_launches"]
            t, got = srv.submit(k, *ins, out=out)
            srv.wait(t)
            assert srv.stats()["inplace_launches"] == before + 1
            t2, ref_srv = srv.submit(k, kn.q.copy(), kn.qd.copy(), kn.tau.copy())
            srv.wait(t2)
            for key in OUTS:
                np.testing.assert_array_equal(got[key], ref_srv[key], err_msg=f"{k} {key}")
            ref = orc.fd_grad_batch(robots[k], kn.q, kn.qd, kn.tau)
            e = np.abs(got["dqdd_dq"] - ref["dqdd_dq"]).reshape(N, -1).max(1) / \
                np.abs(ref["dqdd_dq"]).reshape(N, -1).max(1)
            assert e.max() <= 1e-3
        for t in pinned:
            srv.unpin_range(t)
        r = srv.loadgen(5000, 0.3, [0.5, 0.3, 0.2], warmup_s=0.1, pinned=True)
        st = srv.stats()
        say(f"  pinned loadgen: p50 {r['p50_us']:.0f} us, p99 {r['p99_us']:.0f} us, "
            f"in place {st['inplace_launches']} of {st['launches']} launches")
        assert r["requests"] > 500 and st["inplace_launches"] > st["launches"] // 2
    finally:
        srv.close()
