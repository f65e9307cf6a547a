"""The seeded generator: determinism, sizes and planted structure."""
import numpy as np
import pytest

import graphgen


def test_deterministic_and_seeded():
    a = graphgen.config("small", seed=0)
    b = graphgen.config("small", seed=0)
    c = graphgen.config("small", seed=1)
    assert np.array_equal(a.edges, b.edges)
    assert not np.array_equal(a.edges[:100], c.edges[:100])


def test_thread_count_does_not_change_bytes(monkeypatch):
    g = graphgen.planted(7, k=8, vc=4000, p=0.3, n_extra=2, n_cross=3_000_000, n_pend=10)
    monkeypatch.setenv("GG_THREADS", "1")
    h = graphgen.planted(7, k=8, vc=4000, p=0.3, n_extra=2, n_cross=3_000_000, n_pend=10)
    assert np.array_equal(g.edges, h.edges)


def test_small_and_dense_shapes():
    for name, V, k, pend in [("small", 2030, 20, 30), ("dense", 66536, 256, 1000)]:
        g = graphgen.config(name)
        p = graphgen.PLAIN[name]
        assert g.V == V
        assert g.E == g.n_intra + (k - 1) + p["n_extra"] + pend
        pairs = k * (p["vc"] // k) * (p["vc"] // k - 1) // 2
        mean, sd = pairs * p["p"], np.sqrt(pairs * p["p"] * (1 - p["p"]))
        assert abs(g.n_intra - mean) < 6 * sd
        e = g.edges
        assert e.min() >= 0 and e.max() < g.V
        assert not np.any(e[:, 0] == e[:, 1])
        keys = np.minimum(e[:, 0], e[:, 1]).astype(np.int64) << 32 | np.maximum(e[:, 0], e[:, 1])
        assert np.unique(keys).shape[0] == g.E             # simple graph
        deg = np.bincount(e.ravel(), minlength=g.V)
        assert np.all(deg[g.pend[:, 0]] == 1)              # pendants hang by one edge
        assert np.all(g.cluster[g.pend[:, 0]] == -1) and np.all(g.cluster[g.pend[:, 1]] >= 0)
        ct = g.cluster[g.tree]
        assert np.all(ct[:, 0] != ct[:, 1])                # tree edges join distinct clusters
        assert np.bincount(g.cluster[g.cluster >= 0]).min() == p["vc"] // k
        flipped = np.mean(e[:, 0] > e[:, 1])
        assert 0.45 < flipped < 0.55


def test_cluster_tree_is_a_spanning_tree_of_clusters():
    import oracle
    g = graphgen.config("dense")
    ct = g.cluster[g.tree]
    assert oracle.components(ct, 256) == 1 and ct.shape[0] == 255


def test_cross_edges_join_distinct_clusters():
    g = graphgen.planted(3, k=16, vc=4096, p=1.0, n_cross=200_000, n_pend=5)
    e = g.edges
    inter = g.cluster[e[:, 0]] != g.cluster[e[:, 1]]
    assert inter.sum() == 200_000 + 15 + 5       # cross + tree + pendant (cluster -1)
    assert g.E == 16 * 256 * 255 // 2 + 15 + 5 + 200_000


def test_batched_and_served_recipes():
    ps = [graphgen.batched_params(0, g) for g in range(4096)]
    Vs = np.array([p["vc"] for p in ps])
    assert Vs.min() >= 64 and Vs.max() <= 4096
    assert 500 < np.median(Vs) < 1000                       # log-uniform median ~ 512
    ks = np.array([p["k"] for p in ps])
    assert ks.min() == 2 and ks.max() == 16
    assert all(0.05 <= p["p"] <= 0.5 for p in ps)
    assert max(p["n_extra"] for p in ps) <= 1
    b = graphgen.batched(0, n_graphs=32)
    assert b.offsets[0] == 0 and b.offsets[-1] == b.edges.shape[0]
    for g in range(32):
        e = b.graph(g)
        assert e.shape[0] == 0 or (e.min() >= 0 and e.max() < b.V[g])
    sp = [graphgen.served_params(0, r) for r in range(2000)]
    Vr = np.array([p["vc"] for p in sp])
    assert Vr.min() >= 256 and Vr.max() <= 131072


def test_blocked_cross_edges_stay_in_blocks_and_leave_the_block_tree_bridges():
    # cross edges join two clusters of one block; the cluster tree is a tree
    # per block plus a tree over the blocks, so the bridges are exactly the
    # pendant edges and the tree edges between blocks (checked by the oracle)
    import oracle
    for seed in range(3):
        g = graphgen.planted(seed, k=16, vc=640, p=0.5, n_cross=2000, n_pend=10, cross_block=4)
        blk = np.where(g.cluster >= 0, g.cluster // 4, -1)
        e = g.edges
        cross = (g.cluster[e[:, 0]] >= 0) & (g.cluster[e[:, 1]] >= 0) & (g.cluster[e[:, 0]] != g.cluster[e[:, 1]])
        between = blk[e[:, 0]] != blk[e[:, 1]]
        assert (cross & between).sum() == 3                    # only the 3 tree edges between 4 blocks
        ct = g.cluster[g.tree]
        assert oracle.components(ct, 16) == 1 and ct.shape[0] == 15
        bt = blk[g.tree]
        inter = g.tree[bt[:, 0] != bt[:, 1]]
        assert inter.shape[0] == 3
        assert oracle.components(bt[bt[:, 0] != bt[:, 1]], 4) == 1   # the block tree spans the blocks
        want = np.sort(np.concatenate([g.pend, inter]), 1)
        want = want[np.lexsort((want[:, 1], want[:, 0]))]
        assert np.array_equal(oracle.bridges(e, g.V), want)
    with pytest.raises(ValueError):
        graphgen.planted(0, k=10, vc=100, p=0.5, n_cross=10, cross_block=4)      # 4 does not divide 10
