"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bridge sets are integer sets: the bar is bit-exact equality of the canonical
sorted (u < v) pairs.  Certificates are not unique (any maximal forests do),
so they are judged by the properties every valid certificate has.
"""
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


@pytest.fixture(scope="module", params=[1, 0], ids=["gpu_final_step", "host_search"])
def ctx(request):
    # every test runs with both final steps: the GPU bridge step (the
    # library's default) and Algorithm 1's search on the host
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    c = br.Context(0)
    c.set_final_step(request.param)
    say("final step %d" % request.param)
    yield c
    c.close()


def dev(e):
    return torch.from_numpy(np.ascontiguousarray(e, dtype=np.int32).reshape(-1, 2)).cuda()


@pytest.fixture(scope="module")
def small():
    return graphgen.config("small")


@pytest.fixture(scope="module")
def dense():
    g = graphgen.config("dense")
    return g, oracle.bridges(g.edges, g.V), dev(g.edges)


@pytest.mark.parametrize("M", [4, 1, 2, 3, 5, 8, 16, 100, 10051, 10058])
def test_small_config_bit_exact(ctx, small, M):
    say("small M=%d" % M)
    want = oracle.bridges(small.edges, small.V)
    got = ctx.find(dev(small.edges), small.V, M)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("M", [1, 16, 256, 1024])
def test_dense_config_bit_exact(ctx, dense, M):
    g, want, d = dense
    say("dense M=%d" % M)
    got = ctx.find(d, g.V, M)
    assert got.shape == want.shape and np.array_equal(got, want)


def test_dense_certificate_properties(ctx, dense):
    g, want, d = dense
    for M in (1, 16):
        say("dense cert M=%d" % M)
        f1, f2 = ctx.cert_build(d, g.V, M)
        f1, f2 = f1.cpu().numpy(), f2.cpu().numpy()
        assert oracle.check_certificate(f1, f2, g.edges, g.V) == []


def test_phase0_chunk_certificates_are_maximal(ctx, small):
    # a single chunk (M = 1): F is maximal in G and F' is maximal in G - F
    say("phase0 maximality")
    f1, f2 = ctx.cert_build(dev(small.edges), small.V, 1)
    f1, f2 = f1.cpu().numpy(), f2.cpu().numpy()
    assert f1.shape[0] == small.V - oracle.components(small.edges, small.V)
    keys = lambda e: np.minimum(e[:, 0], e[:, 1]).astype(np.int64) << 32 | np.maximum(e[:, 0], e[:, 1])
    rest = small.edges[~np.isin(keys(small.edges), keys(f1))]        # simple graph: F removed by key
    assert f2.shape[0] == small.V - oracle.components(rest, small.V)
    assert oracle.check_certificate(f1, f2, small.edges, small.V) == []


def test_cert_merge_of_two_certificates(ctx, dense):
    g, want, d = dense
    say("cert_merge")
    h = g.E // 2
    a1, a2 = ctx.cert_build(d[:h].contiguous(), g.V, 4)
    b1, b2 = ctx.cert_build(d[h:].contiguous(), g.V, 4)
    xa = torch.cat([a1, a2]).contiguous()
    xb = torch.cat([b1, b2]).contiguous()
    m1, m2 = ctx.cert_merge(xa, xb, g.V)
    s = torch.cat([m1, m2]).cpu().numpy()
    assert s.shape[0] <= 2 * (g.V - 1)
    assert np.array_equal(oracle.bridges(s, g.V), want)
    assert oracle.check_certificate(m1.cpu().numpy(), m2.cpu().numpy(), g.edges, g.V, check_bridges=False) == []


def test_random_multigraphs(ctx):
    rng = np.random.default_rng(21)
    for t in range(60):
        V = int(rng.integers(1, 400))
        E = int(rng.integers(0, 6 * V))
        e = rng.integers(0, V, size=(E, 2)).astype(np.int32)
        M = int(rng.choice([1, 2, 3, 7, 64, max(E, 1)]))
        say("random t=%d V=%d E=%d M=%d" % (t, V, E, M))
        got = ctx.find(dev(e), V, M)
        assert np.array_equal(got, oracle.bridges(e, V)), (V, E, M)


def test_trees_cycles_and_parallel_edges(ctx):
    say("closed forms")
    rng = np.random.default_rng(22)
    V = 5000
    par = np.array([rng.integers(0, i) for i in range(1, V)])
    tree = np.stack([par, np.arange(1, V)], 1).astype(np.int32)
    for M in (1, 3, 64):
        assert np.array_equal(ctx.find(dev(tree), V, M), oracle.bridges(tree, V))
    cyc = np.stack([np.arange(V), (np.arange(V) + 1) % V], 1).astype(np.int32)
    assert ctx.find(dev(cyc), V, 7).shape[0] == 0
    dbl = np.concatenate([tree, tree[::2, ::-1]])
    assert np.array_equal(ctx.find(dev(dbl), V, 5), oracle.bridges(dbl, V))


def test_edge_cases(ctx):
    import paper_2108_07346_amd as br
    say("edge cases")
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    assert ctx.find(empty, 1, 1).shape[0] == 0
    assert ctx.find(empty, 10, 4).shape[0] == 0
    loops = dev([[0, 0], [3, 3], [3, 3]])
    assert ctx.find(loops, 4, 2).shape[0] == 0
    assert np.array_equal(ctx.find(dev([[5, 2]]), 9, 3), [[2, 5]])
    with pytest.raises(br.BridgeError) as ei:
        ctx.find(dev([[0, 1], [1, 7]]), 5, 1)
    assert ei.value.code == br.BR_ERANGE
    with pytest.raises(br.BridgeError) as ei:
        ctx.find(dev([[0, 1], [-1, 2]]), 5, 2)
    assert ei.value.code == br.BR_ERANGE
    # the context still works after an error
    assert np.array_equal(ctx.find(dev([[0, 1], [1, 2], [2, 0], [2, 3]]), 4, 1), [[2, 3]])
    with pytest.raises(br.BridgeError):
        ctx.find(dev([[0, 1]]), 0, 1)
    with pytest.raises(br.BridgeError):
        ctx.find(dev([[0, 1]]), 2, 0)


def test_concurrency_stress_same_bridges(ctx, dense):
    # many interleavings (permutations, chunk counts, repeated runs of one
    # input): certificates vary, bridges must not
    g, want, d0 = dense
    rng = np.random.default_rng(23)

    def cert_key(f1, f2):
        # the certificate as a set of forest edges (the order of appends
        # within a region is not compared)
        k = lambda f: np.sort(np.minimum(f[:, 0], f[:, 1]).astype(np.int64) << 32 | np.maximum(f[:, 0], f[:, 1]))
        return hash(k(f1.cpu().numpy()).tobytes()) ^ (hash(k(f2.cpu().numpy()).tobytes()) * 3)

    perm_sets, repeat_sets = set(), set()
    for t in range(6):
        e = g.edges[rng.permutation(g.E)]
        d = dev(e)
        M = [1, 2, 16, 64, 256, 1][t]
        say("stress t=%d M=%d" % (t, M))
        assert np.array_equal(ctx.find(d, g.V, M), want)
        f1, f2 = ctx.cert_build(d, g.V, 1)
        perm_sets.add(cert_key(f1, f2))
    for t in range(6):                     # one input, run again: only the schedule differs
        f1, f2 = ctx.cert_build(d0, g.V, 16)
        assert oracle.check_certificate(f1.cpu().numpy(), f2.cpu().numpy(), g.edges, g.V, check_bridges=False) == []
        repeat_sets.add(cert_key(f1, f2))
        assert np.array_equal(ctx.find(d0, g.V, 16), want)
    say("distinct certificates: %d over 6 edge orders, %d over 6 runs of one order" % (len(perm_sets), len(repeat_sets)))
    assert len(perm_sets) >= 2
    assert len(perm_sets | repeat_sets) >= 3


def test_deep_trees_paths_and_random(ctx, small, dense):
    # long tours (list ranking), deep subtrees (range tables), random multigraphs
    g, want, d = dense
    for M in (1, 16, 1024):
        say("dense M=%d" % M)
        assert np.array_equal(ctx.find(d, g.V, M), want)
    assert np.array_equal(ctx.find(dev(small.edges), small.V, 4), oracle.bridges(small.edges, small.V))
    rng = np.random.default_rng(24)
    for t in range(80):
        V = int(rng.integers(1, 300))
        e = rng.integers(0, V, size=(int(rng.integers(0, 5 * V)), 2)).astype(np.int32)
        M = int(rng.choice([1, 2, 5, 33]))
        say("random t=%d V=%d E=%d M=%d" % (t, V, e.shape[0], M))
        assert np.array_equal(ctx.find(dev(e), V, M), oracle.bridges(e, V)), (V, M)
    Vt = 3000
    par = np.array([rng.integers(max(0, i - 3), i) for i in range(1, Vt)])      # deep tree
    tree = np.stack([par, np.arange(1, Vt)], 1).astype(np.int32)
    assert np.array_equal(ctx.find(dev(tree), Vt, 3), oracle.bridges(tree, Vt))
    path = np.stack([np.arange(Vt - 1), np.arange(1, Vt)], 1).astype(np.int32)
    assert np.array_equal(ctx.find(dev(path[::-1].copy()), Vt, 1), oracle.bridges(path, Vt))
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    assert ctx.find(empty, 5, 1).shape[0] == 0
    assert ctx.find(dev([[0, 0]]), 1, 1).shape[0] == 0


def test_two_million_vertex_path_and_cycle(ctx):
    # a path of 2.2M vertices (one tour of 4.4M arcs, range tables of more than
    # 32768 blocks), relabelled at random, with a few chords and a detached cycle
    rng = np.random.default_rng(25)
    V = 2_200_000
    perm = rng.permutation(V).astype(np.int32)
    path = np.stack([perm[:-1], perm[1:]], 1)
    chords = np.stack([perm[[10, 500_000, 1_700_000]], perm[[20, 900_000, 1_700_003]]], 1)
    ring = np.arange(V, V + 1000)
    cyc = np.stack([ring, np.roll(ring, -1)], 1)
    e = np.concatenate([path, chords, cyc]).astype(np.int32)
    e = e[rng.permutation(e.shape[0])]
    Vall = V + 1000
    want = oracle.bridges(e, Vall)
    assert want.shape[0] == (V - 1) - (10 + 400_000 + 3)
    for M in (1, 8):
        say("long path M=%d" % M)
        assert np.array_equal(ctx.find(dev(e), Vall, M), want)
    # 2-edge-connected classes in closed form: each chord closes a cycle over
    # its stretch of the path (one class labelled by its smallest vertex), the
    # other path vertices stand alone, the detached cycle is one class
    lab_want = perm.copy()
    for a, b in ((10, 20), (500_000, 900_000), (1_700_000, 1_700_003)):
        lab_want[a:b + 1] = perm[a:b + 1].min()
    pos = np.empty(V, dtype=np.int64)
    pos[perm] = np.arange(V)
    lab_want = np.concatenate([lab_want[pos], np.full(1000, V, dtype=np.int32)]).astype(np.int32)
    say("long path classes")
    lab, n = ctx.two_edge_components(dev(e), Vall, 8)
    assert n == (V - (11 + 400_001 + 4)) + 3 + 1
    assert np.array_equal(lab, lab_want)


def test_two_edge_connected_classes(ctx, small, dense):
    # 2-edge-connected classes through the certificate path equal the oracle's
    g, _, d = dense
    for M in (1, 16):
        say("2ecc dense M=%d" % M)
        lab, n = ctx.two_edge_components(d, g.V, M)
        want = oracle.two_edge_labels(g.edges, g.V)
        assert np.array_equal(lab, want) and n == np.unique(want).shape[0]
    rng = np.random.default_rng(25)
    for t in range(40):
        V = int(rng.integers(1, 200))
        e = rng.integers(0, V, size=(int(rng.integers(0, 4 * V)), 2)).astype(np.int32)
        lab, n = ctx.two_edge_components(dev(e), V, int(rng.choice([1, 3, 16])))
        want = oracle.two_edge_labels(e, V)
        assert np.array_equal(lab, want), (V, e.shape[0])
        assert n == np.unique(want).shape[0]
    # edge cases: no edges, loops only, one vertex, a doubled edge, an id out of range
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    lab, n = ctx.two_edge_components(empty, 1)
    assert n == 1 and lab.tolist() == [0]
    lab, n = ctx.two_edge_components(empty, 5, 3)
    assert n == 5 and lab.tolist() == [0, 1, 2, 3, 4]
    lab, n = ctx.two_edge_components(dev([[1, 1], [3, 3]]), 4)
    assert n == 4 and lab.tolist() == [0, 1, 2, 3]
    lab, n = ctx.two_edge_components(dev([[2, 1], [1, 2], [2, 3]]), 4)
    assert n == 3 and lab.tolist() == [0, 1, 1, 3]
    import paper_2108_07346_amd as br
    with pytest.raises(br.BridgeError) as ei:
        ctx.two_edge_components(dev([[0, 1], [1, 7]]), 4)
    assert ei.value.code == br.BR_ERANGE
    lab, n = ctx.two_edge_components(dev([[0, 1], [1, 2], [2, 0]]), 3)     # still usable
    assert n == 1 and lab.tolist() == [0, 0, 0]


def test_bridge_tree(ctx, small, dense):
    # the classes contracted, the bridges kept: labels and tree edges equal the
    # oracle's bridge tree (itself pinned by the definitions on tiny graphs)
    g, _, d = dense
    for M in (1, 16):
        say("bridge tree dense M=%d" % M)
        lab, tree = ctx.bridge_tree(d, g.V, M)
        wl, wt = oracle.bridge_tree(g.edges, g.V)
        assert np.array_equal(lab, wl) and np.array_equal(tree, wt)
    lab, tree = ctx.bridge_tree(dev(small.edges), small.V, 4)
    wl, wt = oracle.bridge_tree(small.edges, small.V)
    assert np.array_equal(lab, wl) and np.array_equal(tree, wt)
    rng = np.random.default_rng(26)
    for t in range(40):
        V = int(rng.integers(1, 300))
        e = rng.integers(0, V, size=(int(rng.integers(0, 3 * V)), 2)).astype(np.int32)
        M = int(rng.choice([1, 3, 16]))
        lab, tree = ctx.bridge_tree(dev(e), V, M)
        wl, wt = oracle.bridge_tree(e, V)
        assert np.array_equal(lab, wl) and np.array_equal(tree, wt), (V, e.shape[0], M)
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    lab, tree = ctx.bridge_tree(empty, 3)
    assert lab.tolist() == [0, 1, 2] and tree.shape[0] == 0
    lab, tree = ctx.bridge_tree(dev([[0, 1], [1, 2], [2, 0], [2, 3], [3, 4], [4, 3]]), 5)
    assert lab.tolist() == [0, 0, 0, 3, 3] and tree.tolist() == [[0, 3]]


@pytest.mark.parametrize("V", [4096, 4097, 40944, 40945])
def test_lds_limits(ctx, V):
    # the whole phase tree in LDS up to the kernels' limits (4,096 vertices in
    # the small kernel, 40,944 in the one that takes a CU's whole LDS) and the
    # other plans just past them
    import paper_2108_07346_amd as br
    rng = np.random.default_rng(V)
    k = 8
    g = graphgen.planted(V, k=k, vc=V - 20, p=min(1.0, 40.0 / (V / k)), n_extra=1, n_pend=20)
    assert g.V == V
    want = oracle.bridges(g.edges, V)
    d = dev(g.edges)
    for M in (1, 7, 64):
        say("lds limit V=%d E=%d M=%d" % (V, g.E, M))
        ctx.set_profiling(True)
        got = ctx.find(d, V, M)
        kind = ctx.profile()["plan_kind"]
        ctx.set_profiling(False)
        assert np.array_equal(got, want), (V, M, kind)
        if V <= br.lds_max_v() and g.E // M <= (1 << 18):
            assert kind == 2, kind
        f1, f2 = ctx.cert_build(d, V, M)
        assert oracle.check_certificate(f1.cpu().numpy(), f2.cpu().numpy(), g.edges, V) == []
    e = rng.integers(0, V, size=(3 * V, 2)).astype(np.int32)
    assert np.array_equal(ctx.find(dev(e), V, 5), oracle.bridges(e, V))


def test_small_config_runs_in_lds(ctx, small):
    ctx.set_profiling(True)
    got = ctx.find(dev(small.edges), small.V, 4)
    assert ctx.profile()["plan_kind"] == 2
    ctx.set_profiling(False)
    assert np.array_equal(got, oracle.bridges(small.edges, small.V))


@pytest.mark.parametrize("plan", ["team", "solo"])
def test_method_bytes_on_a_path(ctx, monkeypatch, plan):
    # a path of 2k edges in two chunks: each chunk is a forest, so each
    # certificate keeps its whole chunk and node 0's region ends with the
    # whole path -- 8 * 2k bytes read by phase 0, 8 * 2k written to node 0,
    # 8 * k written to node 1 and read again by the merge
    monkeypatch.setenv("BR_LDS", "0")
    monkeypatch.setenv("BR_SOLO", "1" if plan == "solo" else "0")
    k = 5000
    V = 2 * k + 1
    e = np.stack([np.arange(2 * k), np.arange(1, 2 * k + 1)], 1).astype(np.int32)
    ctx.set_profiling(2)
    got = ctx.find(dev(e), V, 2)
    p = ctx.profile()
    ctx.set_profiling(0)
    assert np.array_equal(got, oracle.bridges(e, V))
    assert p["plan_kind"] == (1 if plan == "solo" else 0)
    assert p["cert_f1"] == 2 * k and p["cert_f2"] == 0
    assert p["alg_bytes"] == 8 * 2 * k + 8 * 2 * k + 16 * k
