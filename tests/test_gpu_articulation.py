"""GPU parity of the articulation points ("failure points" of the abstract):
the scan-first certificate built on the GPU, then the cut-vertex test on it
(on the GPU by default, or the low-link search on the host), against the CPU
oracle (low-link search on the whole graph), bit-exact."""
import itertools
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


@pytest.fixture(scope="module", params=[1, 0], ids=["gpu_test", "host_search"])
def ctx(request):
    # both final steps: the block test on the GPU (default) and the low-link
    # search on the host over the copied certificate
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


@pytest.mark.parametrize("name", ["small", "dense"])
def test_configs_bit_exact(ctx, name):
    g = graphgen.config(name)
    say("articulation %s V=%d E=%d" % (name, g.V, g.E))
    want = oracle.articulation_points(g.edges, g.V)
    got = ctx.articulation_points(dev(g.edges), g.V)
    assert np.array_equal(got, want)
    p = ctx.profile()
    say("  %d articulation points, |F| %d |F'| %d, %d levels" % (got.shape[0], p["cert_f1"], p["cert_f2"], p["rounds"]))
    assert p["cert_f1"] + p["cert_f2"] <= 2 * (g.V - 1)


def test_random_multigraphs(ctx):
    rng = np.random.default_rng(61)
    for t in range(80):
        V = int(rng.integers(1, 300))
        e = rng.integers(0, V, size=(int(rng.integers(0, 5 * V)), 2)).astype(np.int32)
        say("articulation random t=%d V=%d E=%d" % (t, V, e.shape[0]))
        assert np.array_equal(ctx.articulation_points(dev(e), V), oracle.articulation_points(e, V)), (V, e.tolist())


def test_planted_clusters(ctx):
    # clusters joined by trees: every joint and every pendant's neighbour cuts
    for seed in range(6):
        g = graphgen.planted(70 + seed, k=12, vc=1200, p=0.05, n_extra=1, n_pend=9)
        say("articulation planted seed=%d V=%d E=%d" % (seed, g.V, g.E))
        assert np.array_equal(ctx.articulation_points(dev(g.edges), g.V), oracle.articulation_points(g.edges, g.V))


def test_closed_forms_and_edge_cases(ctx):
    import paper_2108_07346_amd as br
    rng = np.random.default_rng(62)
    n = 3000
    perm = rng.permutation(n)
    path = np.stack([perm[:-1], perm[1:]], 1)
    assert np.array_equal(ctx.articulation_points(dev(path), n), np.sort(perm[1:-1]))
    cyc = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    assert ctx.articulation_points(dev(cyc), n).shape[0] == 0
    star = np.stack([np.zeros(n - 1, dtype=np.int64), np.arange(1, n)], 1)
    assert np.array_equal(ctx.articulation_points(dev(star), n), [0])
    kn = np.array(list(itertools.combinations(range(40), 2)))
    assert ctx.articulation_points(dev(kn), 40).shape[0] == 0
    two = np.concatenate([kn, kn + 39])                       # two K40 sharing vertex 39
    assert np.array_equal(ctx.articulation_points(dev(two[rng.permutation(two.shape[0])]), 79), [39])
    par = np.array([rng.integers(max(0, i - 5), i) for i in range(1, 2000)])
    tree = np.stack([par, np.arange(1, 2000)], 1)
    assert np.array_equal(ctx.articulation_points(dev(tree), 2000), oracle.articulation_points(tree, 2000))
    doubled = np.concatenate([tree, tree[:, ::-1]])            # parallel edges protect no vertex
    assert np.array_equal(ctx.articulation_points(dev(doubled), 2000), oracle.articulation_points(tree, 2000))
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    assert ctx.articulation_points(empty, 1).shape[0] == 0
    assert ctx.articulation_points(empty, 7).shape[0] == 0
    assert ctx.articulation_points(dev([[0, 0], [2, 2]]), 3).shape[0] == 0
    assert ctx.articulation_points(dev([[0, 1]]), 2).shape[0] == 0
    with pytest.raises(br.BridgeError) as ei:
        ctx.articulation_points(dev([[0, 1], [1, 9]]), 4)
    assert ei.value.code == br.BR_ERANGE
    assert np.array_equal(ctx.articulation_points(dev([[0, 1], [1, 2]]), 3), [1])   # still usable


def test_same_answer_on_permuted_inputs(ctx):
    # the certificate depends on vertex ids and edge order; the answer must not
    g = graphgen.config("small")
    want = oracle.articulation_points(g.edges, g.V)
    rng = np.random.default_rng(63)
    for t in range(4):
        e = g.edges[rng.permutation(g.E)].copy()
        flip = rng.random(g.E) < 0.5
        e[flip] = e[flip][:, ::-1]
        relabel = rng.permutation(g.V).astype(np.int32)
        got = ctx.articulation_points(dev(relabel[e]), g.V)
        assert np.array_equal(np.sort(got), np.sort(relabel[want]))


@pytest.mark.parametrize("V", [1 << 25, (1 << 25) + 4096], ids=["bucketed_limit", "direct_build"])
def test_random_recursive_tree_at_the_bucket_limit(ctx, V):
    # 2^25 vertices is the most the bucketed adjacency build takes (4,096
    # buckets of 8,192); past it the direct build runs.  A random recursive
    # tree, relabelled: its cut vertices are exactly its vertices of degree >= 2.
    rng = np.random.default_rng(64)
    i = np.arange(1, V, dtype=np.int64)
    par = (rng.random(V - 1) * i).astype(np.int64)
    relabel = rng.permutation(V).astype(np.int32)
    e = np.stack([relabel[par], relabel[i]], 1)
    deg = np.bincount(e.ravel(), minlength=V)
    say("articulation random recursive tree V=%d" % V)
    got = ctx.articulation_points(dev(e), V)
    assert np.array_equal(got, np.flatnonzero(deg >= 2))
