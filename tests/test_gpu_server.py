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
