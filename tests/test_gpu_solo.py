"""The one-workgroup-per-node plan forced onto graphs the size rules would not
give it (the whole-tree LDS plan, which the rules prefer for graphs this
small, switched off): tiny and empty graphs, more chunks than edges,
self-loops and parallel edges, a star (every hook on one root), a long path,
both chunk orders (and siblings bucketed in the merges), tiles full of edges
that lose hook races, and a slot whose tags run out and is cleared.  Every
bridge set must equal the oracle's."""
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
    monkeypatch.setenv("BR_LDS", "0")
    c = br.Context(0)
    c.set_final_step(request.param)
    c.set_profiling(1)
    yield c
    c.close()


def find_solo(ctx, e, V, M):
    """Bridges through the one-workgroup-per-node plan (checked: a graph with
    edges must not have gone to another plan)."""
    got = ctx.find(dev(e), V, M)
    if len(e):
        assert ctx.profile()["plan_kind"] == 1
    return got


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
        got = find_solo(ctx, e, V, M)
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
            assert np.array_equal(find_solo(ctx, g.edges, g.V, M), want), (order, M, top)


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


def race_cases():
    """Graphs whose tiles are full of edges that hook one root, so that most of
    them lose the race for its claim bit, wait, and are offered after the last
    tile: many copies of a few edges (the copies lose at F, are rejected by it
    later and lose again at F'), a star whose centre has the largest id, and
    hubs of high id joined densely to low ids, with a pendant path."""
    rng = np.random.default_rng(33)
    out = []
    base = rng.integers(0, 60, size=(40, 2))
    dup = np.repeat(base, 1500, axis=0)
    out.append(("copies of 40 edges", dup[rng.permutation(len(dup))].astype(np.int32), 60))
    n = 20001
    star = np.stack([np.full(n - 1, n - 1), rng.permutation(n - 1)], 1)
    out.append(("star with the centre last", star.astype(np.int32), n))
    V = 3000
    bip = np.stack([rng.integers(0, 2000, size=60000), rng.integers(V - 64, V, size=60000)], 1)
    path = np.stack([np.arange(1999, 2100), np.arange(2000, 2101)], 1)
    out.append(("hubs over low ids", np.concatenate([bip, path]).astype(np.int32), V))
    return out


def minus_once(e, f):
    """e without one copy of each edge of f (f: a forest of edges of e)."""
    key = lambda a: np.minimum(a[:, 0], a[:, 1]).astype(np.int64) << 32 | np.maximum(a[:, 0], a[:, 1])
    ke, kf = key(e), key(f)
    order = np.argsort(ke, kind="stable")
    at = np.searchsorted(ke[order], kf)
    assert np.all(ke[order][at] == kf)
    keep = np.ones(len(e), bool)
    keep[order[at]] = False
    return e[keep]


@pytest.mark.parametrize("variant", [1, 4])
def test_lost_races_wait_and_are_offered_last(monkeypatch, variant):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    monkeypatch.setenv("BR_SOLO", "1")
    monkeypatch.setenv("BR_LDS", "0")
    monkeypatch.setenv("BR_SOLO_VARIANT", str(variant))
    ctx = br.Context(0)
    ctx.set_profiling(1)
    for name, e, V in race_cases():
        want = oracle.bridges(e, V)
        # one chunk: F maximal in G and F' maximal in G - F
        f1, f2 = ctx.cert_build(dev(e), V, 1)
        assert ctx.profile()["plan_kind"] == 1
        f1, f2 = f1.cpu().numpy(), f2.cpu().numpy()
        assert f1.shape[0] == V - oracle.components(e, V), name
        assert f2.shape[0] == V - oracle.components(minus_once(e, f1), V), name
        assert oracle.check_certificate(f1, f2, e, V) == [], name
        # merges inside the kernel (their losing edges wait in the copy buffer)
        for M in (2, 8):
            for top in (1, 3):
                monkeypatch.setenv("BR_SOLO_TOP", str(top))
                assert np.array_equal(find_solo(ctx, e, V, M), want), (name, M, top)
        say("%s: exact" % name)
    ctx.close()
