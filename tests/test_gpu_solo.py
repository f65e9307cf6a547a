"""The one-workgroup-per-node plan forced onto graphs the size rules would not
give it: tiny and empty graphs, more chunks than edges, self-loops and
parallel edges, a star (every hook on one root), a long path, both chunk
orders (and siblings bucketed in the merges), and a slot whose tags run
out and is cleared.  Every bridge set must equal the oracle's."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(e):
    return torch.from_numpy(np.ascontiguousarray(e, dtype=np.int32).reshape(-1, 2)).cuda()


@pytest.fixture(params=[1, 0], ids=["gpu_final_step", "host_search"])
def ctx(request, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    monkeypatch.setenv("BR_SOLO", "1")
    c = br.Context(0)
    c.set_final_step(request.param)
    yield c
    c.close()


def cases():
    rng = np.random.default_rng(17)
    out = [("single vertex", np.zeros((0, 2), np.int32), 1),
           ("no edges", np.zeros((0, 2), np.int32), 50),
           ("one edge", np.array([[0, 1]], np.int32), 2),
           ("self-loops and parallel edges",
            np.array([[0, 0], [0, 1], [1, 0], [1, 2], [2, 2], [2, 3], [3, 2]], np.int32), 5)]
    n = 3000
    out.append(("star", np.stack([np.zeros(n - 1, np.int64), np.arange(1, n)], 1).astype(np.int32), n))
    p = rng.permutation(20000)
    out.append(("long relabelled path", np.stack([p[:-1], p[1:]], 1).astype(np.int32), 20000))
    for k in range(4):
        V = int(rng.integers(3, 400))
        E = int(rng.integers(0, 4 * V))
        out.append(("random multigraph %d" % k, rng.integers(0, V, size=(E, 2)).astype(np.int32), V))
    g = graphgen.config("small")
    out.append(("small config", g.edges, g.V))
    return out


@pytest.mark.parametrize("M", [1, 3, 64, 300])
def test_forced_solo_edge_cases(ctx, M):
    for name, e, V in cases():
        got = ctx.find(dev(e), V, M)
        assert np.array_equal(got, oracle.bridges(e, V)), (name, M)
    say("M=%d: all cases exact" % M)


@pytest.mark.parametrize("order", ["bucketed", "input", "bucketed_merges", "no_maps", "three_edges"])
def test_forced_solo_both_chunk_orders(ctx, monkeypatch, order):
    if order == "three_edges":          # 1,024-thread workers offering three edges per thread
        monkeypatch.setenv("BR_SOLO_VARIANT", "4")
    if order == "input":
        monkeypatch.setenv("BR_SOLO_NBK", "0")
    if order == "bucketed_merges":      # the merges inside the kernel bucket their siblings too
        monkeypatch.setenv("BR_SOLO_MBK", "1")
    if order == "no_maps":              # every word loaded, no written-bits maps
        monkeypatch.setenv("BR_SOLO_WM", "0")
    g = graphgen.planted(77, k=40, vc=6000, p=0.05, n_extra=2, n_pend=60)
    want = oracle.bridges(g.edges, g.V)
    for M in (16, 257):
        for top in (0, 2):
            monkeypatch.setenv("BR_SOLO_TOP", str(top))
            assert np.array_equal(ctx.find(dev(g.edges), g.V, M), want), (order, M, top)


def test_slot_tags_run_out_and_the_slot_is_cleared(monkeypatch):
    # V = 2^26: a state word keeps 26 bits of offset and 6 of tag, so a slot
    # takes 63 tasks before it must be cleared; the tags persist across calls
    # on one context, so 80 calls drive every worker's slot through the clear
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    monkeypatch.setenv("BR_SOLO", "1")
    monkeypatch.setenv("BR_SOLO_TOP", "0")
    rng = np.random.default_rng(5)
    V = 1 << 26
    hub = rng.integers(0, V, size=3000)
    e = np.concatenate([np.stack([hub[:-1], hub[1:]], 1),                       # a path over 3,000 vertices
                        np.stack([hub[::7][:-1], hub[::7][1:]], 1),             # chords over part of it
                        rng.integers(0, V, size=(2000, 2))]).astype(np.int32)   # scattered edges
    want = oracle.bridges(e, V)
    ctx = br.Context(0)
    d = dev(e)
    for call in range(80):
        got = ctx.find(d, V, 16)
        if call % 20 == 19:
            assert np.array_equal(got, want), call
            say("call %d exact" % call)
    assert np.array_equal(got, want)
    ctx.close()


def test_slot_tags_run_out_with_written_bits_maps(monkeypatch):
    # V = 300,000: 19 bits of offset leave 13 of tag (8,191 chunks per slot
    # before it is cleared), and the maps fit in LDS; 100,000 chunks of four
    # edges spread over the slots (three per worker, handed round through the
    # pool and the parking table) give each slot ~130 chunks per call, so 150
    # calls drive the slots through the clear (twice over) with the maps in use
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    monkeypatch.setenv("BR_SOLO", "1")
    rng = np.random.default_rng(9)
    V = 300000
    hub = rng.permutation(V)[:20000]
    e = np.concatenate([np.stack([hub[:-1], hub[1:]], 1),                   # a path over 20,000 vertices
                        np.stack([hub[::5][:-1], hub[::5][1:]], 1),         # chords over part of it
                        rng.integers(0, V, size=(376001, 2))]).astype(np.int32)
    e = e[rng.permutation(len(e))]
    want = oracle.bridges(e, V)
    ctx = br.Context(0)
    ctx.set_profiling(1)
    d = dev(e)
    for call in range(150):
        got = ctx.find(d, V, 100000)
        if call == 0:
            assert ctx.profile()["plan_kind"] == 1
        if call % 25 == 24:
            assert np.array_equal(got, want), call
            say("call %d exact" % call)
    ctx.close()
