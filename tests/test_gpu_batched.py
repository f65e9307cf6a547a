"""GPU parity of the batched path (one persistent launch over many graphs)
against the CPU oracle, graph by graph, bit-exact."""
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


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    c = br.Context(0)
    yield c
    c.close()


def pack(graphs):
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([g[0].shape[0] for g in graphs])
    e = np.concatenate([g[0] for g in graphs]).astype(np.int32) if off[-1] else np.zeros((0, 2), np.int32)
    return e, off, np.array([g[1] for g in graphs], dtype=np.int32)


def check_all(ctx, e, off, Vs, chunk):
    d = torch.from_numpy(np.ascontiguousarray(e)).cuda()
    pairs, boff = ctx.find_batched(d, off, Vs, chunk)
    for g in range(len(Vs)):
        want = oracle.bridges(e[off[g]:off[g + 1]], int(Vs[g]))
        got = pairs[boff[g]:boff[g + 1]]
        assert np.array_equal(got, want), (g, int(Vs[g]), int(off[g + 1] - off[g]), chunk)
    return pairs, boff


def test_batched_workload_prefix_all_chunk_sizes(ctx):
    b = graphgen.batched(0, n_graphs=192)
    for chunk in (4096, 16384, 65536, 0):
        say("batched prefix chunk=%d" % chunk)
        check_all(ctx, b.edges, b.offsets, b.V, chunk)


def test_batched_full_workload(ctx):
    b = graphgen.batched(0, n_graphs=4096)
    say("batched full: %d graphs, %d edges" % (b.G, b.edges.shape[0]))
    check_all(ctx, b.edges, b.offsets, b.V, 0)


def test_mixed_sizes_and_edge_cases(ctx):
    rng = np.random.default_rng(31)
    graphs = []
    for t in range(40):
        V = int(rng.integers(1, 300))
        graphs.append((rng.integers(0, V, size=(int(rng.integers(0, 4 * V)), 2)).astype(np.int32), V))
    graphs.append((np.zeros((0, 2), np.int32), 1))                      # empty, V = 1
    graphs.append((np.array([[0, 0], [0, 0]], np.int32), 1))            # loops only
    graphs.append((np.array([[3, 1]], np.int32), 4096))                 # at the LDS limit
    for Vb in (1023, 1024, 1025):                                        # both sides of the final step's size split
        path = np.stack([np.arange(Vb - 1), np.arange(1, Vb)], 1).astype(np.int32)
        chords = rng.integers(0, Vb, size=(Vb // 3, 2)).astype(np.int32)
        graphs.append((np.concatenate([path, chords])[rng.permutation(Vb - 1 + Vb // 3)], Vb))
    big = graphgen.planted(5, k=4, vc=6000, p=0.05, n_extra=1, n_pend=7)    # above the LDS limit
    graphs.append((big.edges, big.V))
    tree = np.stack([np.arange(4095), np.arange(1, 4096)], 1).astype(np.int32)
    graphs.append((tree[np.random.default_rng(1).permutation(4095)], 4096))
    e, off, Vs = pack(graphs)
    for chunk in (64, 1000, 0):
        say("mixed chunk=%d" % chunk)
        check_all(ctx, e, off, Vs, chunk)


def test_shared_parent_lists(ctx):
    # graphs that drive the per-wavefront lists of edges the shared-parent
    # test cannot reject to both ends: paths and trees (every edge is such an
    # edge and is accepted), complete graphs and dense multigraphs (after the
    # first compression nearly none is), a star (every hook on one vertex),
    # parallel edges and self-loops, at chunk sizes below and above one
    # workgroup step (512 threads x 4 edges)
    rng = np.random.default_rng(97)
    graphs = []
    for V in (2, 64, 700, 4096):
        p = rng.permutation(V)
        graphs.append((np.stack([p[:-1], p[1:]], 1).astype(np.int32), V))                 # a path
    for n in (40, 90):
        iu = np.triu_indices(n, 1)
        k = np.stack(iu, 1).astype(np.int32)
        graphs.append((np.concatenate([k, k[::3]])[rng.permutation(len(k) + len(k[::3]))], n))   # complete, doubled in part
    graphs.append((np.stack([np.zeros(3000, np.int64), np.arange(1, 3001)], 1).astype(np.int32), 3001))   # a star
    V = 500
    dense = rng.integers(0, V, size=(60 * V, 2)).astype(np.int32)
    dense[::17, 1] = dense[::17, 0]                                                     # self-loops
    graphs.append((dense, V))
    parent = np.array([rng.integers(0, i) for i in range(1, 2000)])
    tree = np.stack([parent, np.arange(1, 2000)], 1).astype(np.int32)
    graphs.append((np.concatenate([tree, tree[:50]])[rng.permutation(2049)], 2000))    # a tree, 50 edges doubled
    e, off, Vs = pack(graphs)
    for chunk in (1000, 2048, 4096, 0):
        say("shared-parent lists chunk=%d" % chunk)
        check_all(ctx, e, off, Vs, chunk)


def test_replay_and_alone_vs_batched(ctx):
    b = graphgen.batched(7, n_graphs=64)
    d = torch.from_numpy(b.edges).cuda()
    p1, o1 = ctx.find_batched(d, b.offsets, b.V, 8192)
    p2, o2 = ctx.find_batched(d, b.offsets, b.V, 8192)       # replayed HIP graph
    assert np.array_equal(p1, p2) and np.array_equal(o1, o2)
    d2 = d.clone()
    p3, o3 = ctx.find_batched(d2, b.offsets, b.V, 8192)      # new buffer: recaptured
    assert np.array_equal(p1, p3)
    for g in range(0, 64, 7):
        alone = ctx.find(d[b.offsets[g]:b.offsets[g + 1]].contiguous(), int(b.V[g]), 3)
        assert np.array_equal(alone, p1[o1[g]:o1[g + 1]])


def test_out_of_range_id_reported(ctx):
    import paper_2108_07346_amd as br
    e, off, Vs = pack([(np.array([[0, 1], [1, 2]], np.int32), 3), (np.array([[0, 5]], np.int32), 4)])
    d = torch.from_numpy(e).cuda()
    with pytest.raises(br.BridgeError) as ei:
        ctx.find_batched(d, off, Vs, 64)
    assert ei.value.code == br.BR_ERANGE
    # and the context keeps working
    e, off, Vs = pack([(np.array([[0, 1], [1, 2]], np.int32), 3)])
    pairs, boff = ctx.find_batched(torch.from_numpy(e).cuda(), off, Vs, 64)
    assert np.array_equal(pairs, [[0, 1], [1, 2]])


def test_batched_host_search(ctx):
    # the other tests use the default final step (one bridge step on the GPU
    # over all certificates as a disjoint union); this one runs Algorithm 1's
    # search per graph on the host
    ctx.set_final_step(0)
    try:
        b = graphgen.batched(0, n_graphs=192)
        for chunk in (4096, 65536):
            say("batched host search chunk=%d" % chunk)
            check_all(ctx, b.edges, b.offsets, b.V, chunk)
        rng = np.random.default_rng(32)
        graphs = [(rng.integers(0, V, size=(int(rng.integers(0, 4 * V)), 2)).astype(np.int32), V)
                  for V in rng.integers(1, 200, size=30).tolist()]
        graphs.append((np.zeros((0, 2), np.int32), 1))
        graphs.append((np.array([[0, 0]], np.int32), 1))
        big = graphgen.planted(6, k=3, vc=5000, p=0.05, n_pend=4)
        graphs.append((big.edges, big.V))
        e, off, Vs = pack(graphs)
        say("batched host search mixed")
        check_all(ctx, e, off, Vs, 128)
        full = graphgen.batched(0, n_graphs=4096)
        say("batched host search full")
        check_all(ctx, full.edges, full.offsets, full.V, 0)
    finally:
        ctx.set_final_step(1)


@pytest.mark.parametrize("final_step", [1, 0], ids=["gpu_final_step", "host_search"])
def test_medium_class_in_the_160kb_kernel(ctx, final_step):
    # graphs above the small kernel's 4,096 vertices and up to the 160 KB
    # kernel's 40,944 run in the same call (their final step: one bridge step
    # over the union of their certificates); beyond that, the plain path
    import paper_2108_07346_amd as br
    big = br.lds_max_v()
    assert big == 40944
    graphs = []
    for k, V in enumerate([4096, 4097, 6000, 100, 17000, big, big + 1, 300, 25000, 4097]):
        kk = max(2, V // 500)
        g = graphgen.planted(900 + k, k=kk, vc=V - 10, p=min(1.0, 24.0 / max(V / kk, 2)), n_extra=1, n_pend=10)
        assert g.V == V
        graphs.append((g.edges, V))
    graphs.append((np.zeros((0, 2), np.int32), 5000))                       # medium class, no edges
    rng = np.random.default_rng(9)
    graphs.append((rng.integers(0, 30000, size=(60000, 2)).astype(np.int32), 30000))   # many bridges, multigraph
    e, off, Vs = pack(graphs)
    ctx.set_final_step(final_step)
    try:
        for chunk in (8192, 0):
            say("medium class final step %d chunk %d: %d graphs, %d edges" % (final_step, chunk, len(Vs), e.shape[0]))
            pairs, boff = check_all(ctx, e, off, Vs, chunk)
            pairs2, boff2 = check_all(ctx, e, off, Vs, chunk)          # replayed graph, same answers
            assert np.array_equal(pairs, pairs2) and np.array_equal(boff, boff2)
    finally:
        ctx.set_final_step(1)
