"""The serving runtime: every answer equals the oracle and equals the same
query run alone, whatever the mix and arrival order; requests overlap on the
device; budget and error paths."""
import sys
import threading

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def br():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as m
    return m


def request_mix(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        V = int(np.exp(rng.uniform(np.log(64), np.log(20000))))
        d = float(np.exp(rng.uniform(np.log(4), np.log(128))))
        s = min(V, max(32, int(2 * d)))
        k = max(1, V // s)
        g = graphgen.planted(seed * 1000 + r, k=k, vc=V, p=min(1.0, d / max(s - 1, 1)),
                             n_extra=int(round(0.02 * (k - 1))), n_pend=int(round(0.015 * V)))
        out.append((g.edges, g.V))
    return out


def test_mix_equals_oracle_and_alone(br):
    reqs = request_mix(40)
    srv = br.Server(0, mem_budget=8 << 30, max_slots=8)
    tickets = [srv.submit(e, V) for e, V in reqs]
    got = [srv.wait(t, V) for t, (_, V) in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    say("served %d requests, peak in flight %d, p50 %.2f ms p99 %.2f ms" %
        (st["completed"], st["peak_inflight"], st["p50_ms"], st["p99_ms"]))
    assert st["completed"] == len(reqs)
    assert st["peak_inflight"] >= 2            # requests were admitted while others ran
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    ctx = br.Context(0)
    for (e, V), g in zip(reqs, got):
        assert np.array_equal(g, oracle.bridges(e, V))
        alone = ctx.find(torch.from_numpy(e).cuda(), V, 1)
        assert np.array_equal(g, alone)
    ctx.close()


@pytest.mark.parametrize("final_step", [1, 0], ids=["gpu_final_step", "host_search"])
def test_reordered_arrivals_threads_and_device_submission(br, final_step):
    reqs = request_mix(24, seed=3)
    want = [oracle.bridges(e, V) for e, V in reqs]
    srv = br.Server(0, mem_budget=8 << 30, max_slots=4)
    srv.set_final_step(final_step)
    res = [None] * len(reqs)
    dev = [torch.from_numpy(e).cuda() for e, _ in reqs]
    order = np.random.default_rng(5).permutation(len(reqs))

    def worker(part):
        for i in part:
            if i % 2:
                t = srv.submit(dev[i], reqs[i][1])
            else:
                t = srv.submit(reqs[i][0], reqs[i][1])
            res[i] = srv.wait(t, reqs[i][1])

    th = [threading.Thread(target=worker, args=(order[k::3],)) for k in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.close()
    for i in range(len(reqs)):
        assert np.array_equal(res[i], want[i]), i


def test_budget_errors_and_polling(br):
    srv = br.Server(0, mem_budget=64 << 20, max_slots=2)
    big = graphgen.planted(1, k=4, vc=20000, p=0.2, n_pend=10)       # needs more than 64 MiB
    with pytest.raises(br.BridgeError) as ei:
        srv.submit(big.edges, big.V)
    assert ei.value.code == br.BR_ENOMEM
    t_bad = srv.submit(np.array([[0, 1], [1, 9]], np.int32), 5)
    with pytest.raises(br.BridgeError) as ei:
        srv.wait(t_bad, 5)
    assert ei.value.code == br.BR_ERANGE
    e = np.array([[0, 1], [1, 2], [2, 0], [2, 3]], np.int32)
    t = srv.submit(e, 4)
    done, out = False, None
    for _ in range(100000):
        done, out = srv.poll(t, 4)
        if done:
            break
    assert done and np.array_equal(out, [[2, 3]])
    with pytest.raises(br.BridgeError):
        srv.poll(t, 4)                           # the ticket was released
    srv.close()


@pytest.fixture(scope="module")
def served32():
    # the served workload's own requests (graphgen.served_request): V up to
    # 131,072, average degree up to 2,048, up to 7.0e7 edges each
    reqs = []
    for r in range(32):
        g = graphgen.served_request(0, r)
        reqs.append((g.edges, g.V, oracle.bridges(g.edges, g.V)))
    say("served requests: %d, %d edges" % (len(reqs), sum(e.shape[0] for e, _, _ in reqs)))
    return reqs


@pytest.mark.parametrize("final_step", [1, 0], ids=["gpu_final_step", "host_search"])
def test_served_config_requests_equal_oracle_and_alone(br, served32, final_step):
    dev = [torch.from_numpy(e).cuda() for e, _, _ in served32]
    alone_ctx = br.Context(0)
    alone_ctx.set_final_step(final_step)
    alone = [alone_ctx.find(d, V, 1) for d, (_, V, _) in zip(dev, served32)]
    alone_ctx.close()
    for host in (True, False):
        srv = br.Server(0, mem_budget=64 << 30, max_slots=8)
        srv.set_final_step(final_step)
        tickets = [srv.submit(e if host else d, V) for (e, V, _), d in zip(served32, dev)]
        got = [srv.wait(t, V) for t, (_, V, _) in zip(tickets, served32)]
        st = srv.stats()
        srv.close()
        say("served config, %s submission, final step %d: %d done, peak in flight %d" %
            ("host" if host else "device", final_step, st["completed"], st["peak_inflight"]))
        assert st["completed"] == len(served32)
        for i, (g, (e, V, want)) in enumerate(zip(got, served32)):
            assert np.array_equal(g, want), i
            assert np.array_equal(g, alone[i]), i


def test_final_step_changes_only_later_admissions(br):
    # the mode is flipped while requests are queued and running; every answer
    # is still the oracle's (a request keeps the mode it was admitted with)
    reqs = request_mix(48, seed=7)
    srv = br.Server(0, mem_budget=8 << 30, max_slots=4)
    tickets = []
    for i, (e, V) in enumerate(reqs):
        if i % 5 == 0:
            srv.set_final_step((i // 5) % 2)
        tickets.append(srv.submit(e, V))
    for t, (e, V) in zip(tickets, reqs):
        assert np.array_equal(srv.wait(t, V), oracle.bridges(e, V))
    srv.close()


def test_tight_budget_releases_idle_slots(br):
    # a large request on one slot, then another on a second slot under a budget
    # that cannot hold both slots' buffers: the idle slot's memory is released
    # and both succeed; what the slots hold never exceeds the budget
    a = graphgen.planted(11, k=8, vc=40000, p=0.05, n_pend=20)
    b = graphgen.planted(12, k=8, vc=40000, p=0.05, n_pend=20)
    srv0 = br.Server(0, mem_budget=64 << 30, max_slots=1)
    srv0.set_batching(0)                     # both requests on slots
    ta = srv0.submit(a.edges, a.V)
    srv0.wait(ta, a.V)
    one = srv0.stats()["peak_device_bytes"]
    srv0.close()
    budget = int(one * 1.5)
    srv = br.Server(0, mem_budget=budget, max_slots=2)
    srv.set_batching(0)
    for rep in range(3):
        ta = srv.submit(a.edges, a.V)
        tb = srv.submit(b.edges, b.V)        # may run while a's slot still holds its buffers
        assert np.array_equal(srv.wait(ta, a.V), oracle.bridges(a.edges, a.V))
        assert np.array_equal(srv.wait(tb, b.V), oracle.bridges(b.edges, b.V))
    st = srv.stats()
    srv.close()
    say("tight budget: one request holds %d bytes, budget %d, peak held %d" % (one, budget, st["peak_device_bytes"]))
    assert 0 < st["peak_device_bytes"] <= budget


def small_burst(n, seed):
    # small requests (V 16..3000) that the batch lane serves many per tick
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        V = int(np.exp(rng.uniform(np.log(16), np.log(3000))))
        k = max(2, V // 64)
        g = graphgen.planted(seed * 10000 + r, k=k, vc=V, p=min(1.0, 10.0 / max(V / k, 2)),
                             n_extra=1, n_pend=max(1, V // 50))
        out.append((g.edges, g.V))
    return out


def test_batch_lane_serves_many_requests_per_tick(br):
    reqs = small_burst(400, seed=21)
    srv = br.Server(0, mem_budget=8 << 30, max_slots=4)
    dev = [torch.from_numpy(e).cuda() for e, _ in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(dev[i] if i % 3 == 0 else e, V) for i, (e, V) in enumerate(reqs)]
    got = [srv.wait(t, V) for t, (_, V) in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    say("batch lane: %d requests in %d ticks, p50 %.2f ms" % (st["batched_requests"], st["batched_ticks"], st["p50_ms"]))
    assert st["completed"] == len(reqs)
    # a burst keeps the slots busy, so most requests collect in the lane and
    # several share a tick
    assert st["batched_requests"] >= len(reqs) // 2
    assert st["batched_ticks"] < st["batched_requests"]
    for (e, V), g in zip(reqs, got):
        assert np.array_equal(g, oracle.bridges(e, V))


def test_batch_lane_isolates_a_bad_request(br):
    # a request with an id out of range fails alone; the others of its tick
    # are answered
    reqs = small_burst(60, seed=22)
    srv = br.Server(0, mem_budget=8 << 30, max_slots=2)
    tickets = []
    for i, (e, V) in enumerate(reqs):
        tickets.append(srv.submit(e, V))
        if i == 30:
            t_bad = srv.submit(np.array([[0, 1], [1, 7]], np.int32), 4)
    for t, (e, V) in zip(tickets, reqs):
        assert np.array_equal(srv.wait(t, V), oracle.bridges(e, V))
    with pytest.raises(br.BridgeError) as ei:
        srv.wait(t_bad, 4)
    assert ei.value.code == br.BR_ERANGE
    srv.close()


@pytest.mark.parametrize("final_step", [1, 0], ids=["gpu_final_step", "host_search"])
def test_batching_limits(br, final_step):
    # with batching off, or limits no request meets, nothing joins the lane;
    # with the default limits a burst does; every answer is the oracle's, and
    # limits outside their ranges are refused
    reqs = request_mix(40, seed=9)
    srv = br.Server(0, mem_budget=8 << 30, max_slots=4)
    srv.set_final_step(final_step)
    for bad in ((br.lds_max_v() + 1, 1 << 21), (-1, 1 << 21), (1000, -1)):
        with pytest.raises(br.BridgeError) as ei:
            srv.set_batching(*bad)
        assert ei.value.code == br.BR_EINVAL
    got = []
    for limits in ((0, 1 << 21), (br.lds_max_v(), 1)):
        srv.set_batching(*limits)
        tickets = [srv.submit(e, V) for e, V in reqs[:20]]
        got += [srv.wait(t, V) for t, (_, V) in zip(tickets, reqs[:20])]
        assert srv.stats(reset=True)["batched_requests"] == 0
    srv.set_batching(br.lds_max_v(), 1 << 30)
    eligible = sum(1 for _, V in reqs[20:] if V <= br.lds_max_v())
    tickets = [srv.submit(e, V) for e, V in reqs[20:]]
    got += [srv.wait(t, V) for t, (_, V) in zip(tickets, reqs[20:])]
    st = srv.stats()
    srv.close()
    assert st["batched_requests"] <= eligible
    want = [oracle.bridges(e, V) for e, V in reqs[:20]] * 2 + [oracle.bridges(e, V) for e, V in reqs[20:]]
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


def test_batch_lane_under_a_tight_budget(br):
    # lane requests are charged an upper bound of their share of a tick until
    # it completes, and what the lane keeps between ticks stays charged: under
    # a budget a few requests wide, every answer is right and the charge never
    # passes the budget
    reqs = small_burst(120, seed=23)
    budget = 64 << 20
    srv = br.Server(0, mem_budget=budget, max_slots=2)
    tickets = [srv.submit(e, V) for e, V in reqs]
    for t, (e, V) in zip(tickets, reqs):
        assert np.array_equal(srv.wait(t, V), oracle.bridges(e, V))
    st = srv.stats()
    srv.close()
    say("lane, budget %d: peak charged %d, %d ticks" % (budget, st["peak_device_bytes"], st["batched_ticks"]))
    assert 0 < st["peak_device_bytes"] <= budget
