"""Pins of the CPU oracle against things other than itself.

* brute force over the definition of Section I (exhaustive for V <= 5,
  random multigraphs with loops and parallel edges for V <= 12);
* textbook closed forms (trees, cycles, complete graphs, ...);
* hand-worked cases in tests/golden/hand_examples.txt;
* networkx's bridge routine, run as an independent library;
* invariants of bridge sets (forest, b + c two-edge-connected classes,
  removal raises the component count by exactly one, relabel/permutation
  invariance);
* the generator's planted structure on the small and dense workloads.
"""
import itertools
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def canon(pairs):
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    if p.shape[0] == 0:
        return np.zeros((0, 2), dtype=np.int32)
    p = np.stack([p.min(1), p.max(1)], 1)
    p = np.unique(p, axis=0)
    return p.astype(np.int32)


def load_hand_examples():
    cases, cur = [], None
    for line in open(os.path.join(HERE, "golden", "hand_examples.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], V=0, e=[], b=[])
        elif tok[0] == "V":
            cur["V"] = int(tok[1])
        elif tok[0] == "e":
            cur["e"].append((int(tok[1]), int(tok[2])))
        elif tok[0] == "b":
            cur["b"].append((int(tok[1]), int(tok[2])))
        elif tok[0] == "end":
            cases.append(cur)
    return cases


HAND = load_hand_examples()


@pytest.mark.parametrize("case", HAND, ids=[c["name"] for c in HAND])
def test_hand_examples(case):
    got = oracle.bridges(np.array(case["e"], dtype=np.int32).reshape(-1, 2), case["V"])
    want = np.array(sorted(case["b"]), dtype=np.int32).reshape(-1, 2)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.brute_bridges(np.array(case["e"]).reshape(-1, 2), case["V"]), want)


# ---- closed forms --------------------------------------------------------------

def test_trees_all_edges():
    rng = np.random.default_rng(1)
    for V in [2, 3, 10, 257, 5000]:
        path = np.stack([np.arange(V - 1), np.arange(1, V)], 1)
        star = np.stack([np.zeros(V - 1, dtype=np.int64), np.arange(1, V)], 1)
        par = np.array([rng.integers(0, i) for i in range(1, V)])
        rnd = np.stack([par, np.arange(1, V)], 1)
        for t in (path, star, rnd):
            perm = rng.permutation(V)
            t2 = perm[t]
            assert np.array_equal(oracle.bridges(t2, V), canon(t2))


def test_cycles_and_complete_graphs_have_none():
    for n in [3, 4, 7, 100, 3000]:
        cyc = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
        assert oracle.bridges(cyc, n).shape[0] == 0
    for n in [3, 4, 9, 40]:
        kn = np.array(list(itertools.combinations(range(n), 2)))
        assert oracle.bridges(kn, n).shape[0] == 0
    assert np.array_equal(oracle.bridges([[0, 1]], 2), [[0, 1]])     # K2 is a tree


def test_double_edges_are_never_bridges():
    rng = np.random.default_rng(2)
    V = 300
    par = np.array([rng.integers(0, i) for i in range(1, V)])
    tree = np.stack([par, np.arange(1, V)], 1)
    doubled = tree[rng.random(V - 1) < 0.3]
    g = np.concatenate([tree, doubled[:, ::-1]])
    want = canon(np.array(sorted(set(map(tuple, canon(tree).tolist())) - set(map(tuple, canon(doubled).tolist())))))
    assert np.array_equal(oracle.bridges(g, V), want)


def test_disjoint_union_is_union_of_parts():
    a = np.array([[0, 1], [1, 2], [2, 0], [2, 3]])          # bridge 2-3
    b = np.array([[0, 1], [1, 2]])                           # two bridges
    g = np.concatenate([a, b + 4])
    assert np.array_equal(oracle.bridges(g, 10), canon([[2, 3], [4, 5], [5, 6]]))


def test_bad_ids_rejected():
    with pytest.raises(ValueError):
        oracle.bridges([[0, 5]], 5)
    with pytest.raises(ValueError):
        oracle.bridges([[-1, 0]], 5)


# ---- brute force ----------------------------------------------------------------

def test_exhaustive_small_graphs():
    for V in range(1, 6):
        pairs = list(itertools.combinations(range(V), 2))
        for mask in range(1 << len(pairs)):
            e = np.array([pairs[i] for i in range(len(pairs)) if mask >> i & 1], dtype=np.int32).reshape(-1, 2)
            assert np.array_equal(oracle.bridges(e, V), oracle.brute_bridges(e, V)), (V, e.tolist())


def test_random_multigraphs_vs_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(400):
        V = int(rng.integers(1, 13))
        E = int(rng.integers(0, 3 * V + 1))
        e = rng.integers(0, V, size=(E, 2)).astype(np.int32)
        assert np.array_equal(oracle.bridges(e, V), oracle.brute_bridges(e, V)), (V, e.tolist())


# ---- networkx, run as an independent library -------------------------------------

def test_against_networkx():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(4)
    for V, E in [(50, 60), (1000, 1100), (5000, 9000), (20000, 22000), (100000, 130000)]:
        e = rng.integers(0, V, size=(E, 2))
        G = nx.Graph()
        G.add_nodes_from(range(V))
        G.add_edges_from(map(tuple, e.tolist()))
        simple = np.array(list(G.edges()), dtype=np.int32).reshape(-1, 2)
        want = canon(np.array(list(nx.bridges(G)), dtype=np.int64).reshape(-1, 2))
        assert np.array_equal(oracle.bridges(simple, V), want)


# ---- invariants ------------------------------------------------------------------

def two_edge_classes(V, edges, bridges):
    bset = set(map(tuple, canon(bridges).tolist()))
    keep = [p for p in canon_rows(edges) if (min(p), max(p)) not in bset]
    return oracle.components(np.array(keep, dtype=np.int32).reshape(-1, 2), V)


def canon_rows(e):
    return [(int(a), int(b)) for a, b in np.asarray(e).reshape(-1, 2)]


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 40).flatmap(
    lambda V: st.tuples(st.just(V), st.lists(st.tuples(st.integers(0, V - 1), st.integers(0, V - 1)), max_size=80))))
def test_bridge_invariants(data):
    V, el = data
    e = np.array(el, dtype=np.int32).reshape(-1, 2)
    b = oracle.bridges(e, V)
    c = oracle.components(e, V)
    assert b.shape[0] <= max(V - 1, 0)
    # bridges form a forest
    assert b.shape[0] == V - oracle.components(b, V)
    # contracting the non-bridge edges leaves b + c classes
    assert two_edge_classes(V, e, b) == b.shape[0] + c
    # removing a bridge raises the component count by exactly one
    for u, v in b.tolist():
        idx = [i for i, (x, y) in enumerate(e.tolist()) if (min(x, y), max(x, y)) == (u, v)]
        assert len(idx) == 1
        rest = np.delete(e, idx[0], axis=0)
        assert oracle.components(rest, V) == c + 1
    # invariance under edge permutation, orientation flips and vertex relabelling
    rng = np.random.default_rng(len(el) * 7919 + V)
    perm = rng.permutation(V)
    e2 = perm[e[rng.permutation(e.shape[0])]] if e.shape[0] else e
    if e2.shape[0]:
        flip = rng.random(e2.shape[0]) < 0.5
        e2[flip] = e2[flip][:, ::-1]
    assert np.array_equal(oracle.bridges(e2, V), canon(perm[b]) if b.shape[0] else b)


# ---- the generator's planted structure ----------------------------------------

def cluster_tree_bridges(g):
    """Bridges expected from the planted structure alone, assuming every
    cluster is 2-edge-connected: the pendant edges, plus every tree edge that
    is a bridge of the cluster multigraph (tree + extra edges)."""
    k = g.params["k"]
    cl = g.cluster
    qe = np.concatenate([g.tree, g.extra])
    q = np.stack([cl[qe[:, 0]], cl[qe[:, 1]]], 1)
    qb = set(map(tuple, oracle.brute_bridges(q, k).tolist()))
    want = [tuple(t) for t, c in zip(g.tree.tolist(), q[:g.tree.shape[0]].tolist())
            if (min(c), max(c)) in qb]
    return canon(np.array(want + g.pend.tolist(), dtype=np.int64).reshape(-1, 2))


def test_dense_workload_equals_planted_expectation():
    g = graphgen.config("dense")
    got = oracle.bridges(g.edges, g.V)
    want = cluster_tree_bridges(g)
    assert got.shape[0] == want.shape[0] and np.array_equal(got, want)
    assert g.tree.shape[0] == 255 and g.pend.shape[0] == 1000


def test_small_workload_contains_planted_and_extras_are_real():
    g = graphgen.config("small")
    got = oracle.bridges(g.edges, g.V)
    planted = cluster_tree_bridges(g)
    gs = set(map(tuple, got.tolist()))
    assert set(map(tuple, planted.tolist())) <= gs
    # every reported bridge, planted or natural, is one by the definition
    c = oracle.components(g.edges, g.V)
    keys = g.edges.min(1).astype(np.int64) << 32 | g.edges.max(1)
    for u, v in got.tolist():
        rest = g.edges[keys != (u << 32 | v)]
        assert oracle.components(rest, g.V) == c + 1
    # and a sample of non-bridges is not
    rng = np.random.default_rng(5)
    for i in rng.choice(g.E, 60, replace=False):
        u, v = int(g.edges[i].min()), int(g.edges[i].max())
        if (u, v) in gs:
            continue
        assert oracle.components(np.delete(g.edges, i, axis=0), g.V) == c


# ---- 2-edge-connected classes (oracle side) ---------------------------------

def test_two_edge_labels_brute_force_and_invariants():
    rng = np.random.default_rng(41)
    for _ in range(150):
        V = int(rng.integers(1, 10))
        e = rng.integers(0, V, size=(int(rng.integers(0, 3 * V + 1)), 2)).astype(np.int32)
        lab = oracle.two_edge_labels(e, V)
        assert np.array_equal(lab, oracle.brute_two_edge_labels(e, V)), (V, e.tolist())
        assert np.unique(lab).shape[0] == oracle.bridges(e, V).shape[0] + oracle.components(e, V)
    # closed forms: a cycle is one class; a tree has V singleton classes
    cyc = np.stack([np.arange(6), (np.arange(6) + 1) % 6], 1)
    assert np.all(oracle.two_edge_labels(cyc, 6) == 0)
    tree = np.array([[0, 1], [1, 2], [1, 3]])
    assert np.array_equal(oracle.two_edge_labels(tree, 4), [0, 1, 2, 3])


def test_bridge_tree_definition_forest_and_closed_forms():
    # the bridge tree: classes contracted, bridges kept.  Pinned by the
    # brute-force definitions of classes and bridges on tiny multigraphs, by
    # the forest invariants (one tree per component of G, as many nodes as
    # classes, as many edges as bridges) and by closed forms.
    rng = np.random.default_rng(41)
    for _ in range(150):
        V = int(rng.integers(1, 11))
        e = rng.integers(0, V, size=(int(rng.integers(0, 16)), 2)).astype(np.int32)
        lab, t = oracle.bridge_tree(e, V)
        bl = oracle.brute_two_edge_labels(e, V)
        bb = oracle.brute_bridges(e, V)
        want = sorted(tuple(sorted((int(bl[a]), int(b)))) for a, b in
                      ((u, bl[v]) for u, v in bb.tolist()))
        assert np.array_equal(lab, bl)
        assert [tuple(x) for x in t.tolist()] == want
        nodes = np.unique(lab)
        assert t.shape[0] == bb.shape[0]
        assert np.all(t[:, 0] < t[:, 1]) if t.shape[0] else True
        # a forest over the classes with one tree per component of the graph
        idx = {int(c): k for k, c in enumerate(nodes)}
        tt = np.array([[idx[int(a)], idx[int(b)]] for a, b in t.tolist()], dtype=np.int32).reshape(-1, 2)
        assert oracle.components(tt, nodes.shape[0]) == nodes.shape[0] - t.shape[0]
        assert oracle.components(tt, nodes.shape[0]) == oracle.components(e, V)
    # k triangles in a row joined by single edges: a path of k classes
    k = 6
    tri = []
    for i in range(k):
        a, b, c = 3 * i, 3 * i + 1, 3 * i + 2
        tri += [[a, b], [b, c], [c, a]]
        if i:
            tri.append([3 * i - 1, a])
    lab, t = oracle.bridge_tree(np.array(tri, np.int32), 3 * k)
    assert np.array_equal(lab, np.repeat(np.arange(k) * 3, 3))
    assert t.tolist() == [[3 * i, 3 * i + 3] for i in range(k - 1)]
    # a tree graph is its own bridge tree; a cycle contracts to one node
    par = [[i, (i - 1) // 2] for i in range(1, 15)]
    lab, t = oracle.bridge_tree(np.array(par, np.int32), 15)
    assert np.array_equal(lab, np.arange(15)) and t.shape[0] == 14
    lab, t = oracle.bridge_tree(np.array([[i, (i + 1) % 7] for i in range(7)], np.int32), 7)
    assert np.all(lab == 0) and t.shape[0] == 0
