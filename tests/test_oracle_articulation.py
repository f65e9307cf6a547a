"""Pins of the articulation-point oracle ("failure points" of the abstract)
and of the scan-first certificate, against things other than themselves.

* hand-worked cases in tests/golden/hand_articulation.txt;
* the definition written out (remove each vertex, count components):
  exhaustive for V <= 5, random multigraphs for V <= 12;
* networkx's articulation-point routine, run as an independent library;
* textbook closed forms (paths, cycles, stars, trees, complete graphs, two
  cliques sharing a vertex);
* invariants (a bridge endpoint of degree >= 2 is a cut vertex; removing a
  cut vertex raises the component count, removing another vertex does not);
* the scan-first certificate keeps exactly the articulation points, which a
  certificate of two arbitrary (union-find) forests does not;
* planted mistakes in the oracle's source are caught by these pins.
"""
import ctypes
import itertools
import os
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def load_cases():
    cases, cur = [], None
    for line in open(os.path.join(HERE, "golden", "hand_articulation.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], V=0, e=[], a=[])
        elif tok[0] == "V":
            cur["V"] = int(tok[1])
        elif tok[0] == "e":
            cur["e"].append((int(tok[1]), int(tok[2])))
        elif tok[0] == "a":
            cur["a"].append(int(tok[1]))
        elif tok[0] == "end":
            cases.append(cur)
    return cases


CASES = load_cases()


def arr(e):
    return np.array(e, dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_examples(case):
    want = np.array(sorted(case["a"]), dtype=np.int32)
    assert np.array_equal(oracle.articulation_points(arr(case["e"]), case["V"]), want)
    assert np.array_equal(oracle.brute_articulation_points(arr(case["e"]), case["V"]), want)


def test_exhaustive_small_graphs():
    for V in range(1, 6):
        pairs = list(itertools.combinations(range(V), 2))
        for mask in range(1 << len(pairs)):
            e = arr([pairs[i] for i in range(len(pairs)) if mask >> i & 1])
            assert np.array_equal(oracle.articulation_points(e, V), oracle.brute_articulation_points(e, V)), \
                (V, e.tolist())


def test_random_multigraphs_vs_definition():
    rng = np.random.default_rng(51)
    for _ in range(400):
        V = int(rng.integers(1, 13))
        e = rng.integers(0, V, size=(int(rng.integers(0, 3 * V + 1)), 2)).astype(np.int32)
        assert np.array_equal(oracle.articulation_points(e, V), oracle.brute_articulation_points(e, V)), \
            (V, e.tolist())


def test_against_networkx():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(52)
    for V, E in [(50, 55), (1000, 1200), (5000, 6000), (20000, 30000), (100000, 120000)]:
        e = rng.integers(0, V, size=(E, 2))
        G = nx.Graph()
        G.add_nodes_from(range(V))
        G.add_edges_from([(int(a), int(b)) for a, b in e if a != b])
        want = np.array(sorted(nx.articulation_points(G)), dtype=np.int32)
        assert np.array_equal(oracle.articulation_points(e.astype(np.int32), V), want)


def test_closed_forms():
    for n in (3, 10, 1000):
        path = np.stack([np.arange(n - 1), np.arange(1, n)], 1)
        assert np.array_equal(oracle.articulation_points(path, n), np.arange(1, n - 1))
        cyc = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
        assert oracle.articulation_points(cyc, n).shape[0] == 0
        star = np.stack([np.full(n - 1, n // 2), np.delete(np.arange(n), n // 2)], 1)
        assert np.array_equal(oracle.articulation_points(star, n), [n // 2])
    for n in (3, 6, 30):
        kn = np.array(list(itertools.combinations(range(n), 2)))
        assert oracle.articulation_points(kn, n).shape[0] == 0
        # two copies of K_n glued at one vertex (vertex n-1 of the first is 0 of the second)
        two = np.concatenate([kn, kn + (n - 1)])
        assert np.array_equal(oracle.articulation_points(two, 2 * n - 1), [n - 1])
    rng = np.random.default_rng(53)
    V = 3000
    par = np.array([rng.integers(0, i) for i in range(1, V)])
    tree = np.stack([par, np.arange(1, V)], 1)
    deg = np.bincount(tree.ravel(), minlength=V)
    assert np.array_equal(oracle.articulation_points(tree, V), np.flatnonzero(deg >= 2))


def test_invariants():
    rng = np.random.default_rng(54)
    for _ in range(60):
        V = int(rng.integers(2, 60))
        e = rng.integers(0, V, size=(int(rng.integers(0, 2 * V)), 2)).astype(np.int32)
        ap = set(oracle.articulation_points(e, V).tolist())
        loopless = e[e[:, 0] != e[:, 1]]
        deg = np.bincount(loopless.ravel(), minlength=V)
        for u, v in oracle.bridges(e, V).tolist():
            for x in (u, v):
                if deg[x] >= 2:
                    assert x in ap
        c = oracle.components(e, V)
        for x in rng.choice(V, size=min(V, 10), replace=False).tolist():
            keep = e[(e[:, 0] != x) & (e[:, 1] != x)]
            relab = np.where(keep > x, keep - 1, keep)
            cx = oracle.components(relab, V - 1)
            assert (cx > c) == (x in ap)


def test_scan_first_certificate_keeps_articulation_points():
    rng = np.random.default_rng(55)
    survived_uf = 0
    for t in range(300):
        V = int(rng.integers(2, 40))
        e = rng.integers(0, V, size=(int(rng.integers(0, 4 * V)), 2)).astype(np.int32)
        f1, f2 = oracle.scan_first_certificate(e, V)
        s = np.concatenate([f1, f2])
        assert s.shape[0] <= 2 * max(V - 1, 0)
        assert f1.shape[0] == V - oracle.components(e, V)                 # spanning forest
        assert oracle.components(f1, V) == oracle.components(e, V)
        p1 = set(map(tuple, np.sort(f1, 1).tolist()))
        assert not (set(map(tuple, np.sort(f2, 1).tolist())) & p1)      # F' avoids F's pairs
        assert np.array_equal(oracle.articulation_points(s, V), oracle.articulation_points(e, V)), (V, e.tolist())
        # two arbitrary forests (Algorithm 2 on the list order) do not always keep them
        g1, g2 = oracle.certificate(e, V)
        if np.array_equal(oracle.articulation_points(np.concatenate([g1, g2]), V), oracle.articulation_points(e, V)):
            survived_uf += 1
    assert survived_uf < 300


def test_planted_workloads():
    for name in ("small", "dense"):
        g = graphgen.config(name)
        ap = set(oracle.articulation_points(g.edges, g.V).tolist())
        # every pendant edge's cluster endpoint (of degree >= 2) is a cut vertex
        deg = np.bincount(g.edges.ravel(), minlength=g.V)
        for _, inner in g.pend.tolist():
            assert inner in ap or deg[inner] == 1
        if name == "dense":
            f1, f2 = oracle.scan_first_certificate(g.edges[:200000], g.V)
            assert np.array_equal(oracle.articulation_points(np.concatenate([f1, f2]), g.V),
                                  oracle.articulation_points(g.edges[:200000], g.V))


# ---- planted mistakes in the oracle's source --------------------------------------

SRC = os.path.join(os.path.dirname(oracle.__file__), "articulation.c")
MUTANTS = {
    "strict_test": ("if (sp > 0 && low[x] >= disc[p]) cut[p] = 1;", "if (sp > 0 && low[x] > disc[p]) cut[p] = 1;"),
    "root_one_child": ("if (root_children >= 2) cut[s] = 1;", "if (root_children >= 1) cut[s] = 1;"),
    "root_as_inner": ("if (sp > 0 && low[x] >= disc[p]) cut[p] = 1;", "if (low[x] >= disc[p]) cut[p] = 1;"),
    "no_low_propagation": ("if (low[x] < low[p]) low[p] = low[x];", ";"),
    "back_edge_ignored": ("} else if (disc[y] < low[x]) {", "} else if (0) {"),
    "first_root_only": ("for (int64_t s = 0; s < V; s++) {\n        if (disc[s] != -1) continue;\n        int64_t sp = 0, root",
                        "for (int64_t s = 0; s < (V > 0 ? 1 : 0); s++) {\n        if (disc[s] != -1) continue;\n        int64_t sp = 0, root"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, name
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, name + ".c")
        open(path, "w").write(src.replace(old, new))
        so = os.path.join(tmp, name + ".so")
        subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", path, "-o", so])
        lib = ctypes.CDLL(so)
        lib.oracle_articulation_points.restype = ctypes.c_int
        lib.oracle_articulation_points.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]

        def run(e, V):
            e = np.ascontiguousarray(np.asarray(e, dtype=np.int32).reshape(-1, 2))
            out = np.zeros(max(V, 1), dtype=np.int32)
            n = ctypes.c_int64(0)
            lib.oracle_articulation_points(e.ctypes.data, e.shape[0], V, out.ctypes.data, out.shape[0], ctypes.byref(n))
            return out[:n.value].copy()

        caught = any(not np.array_equal(run(c["e"], c["V"]), np.array(sorted(c["a"]), dtype=np.int32)) for c in CASES)
        rng = np.random.default_rng(56)
        for _ in range(200):
            if caught:
                break
            V = int(rng.integers(1, 13))
            e = rng.integers(0, V, size=(int(rng.integers(0, 3 * V + 1)), 2)).astype(np.int32)
            caught = not np.array_equal(run(e, V), oracle.brute_articulation_points(e, V))
        assert caught, "mutant %s survived the pins" % name


def test_scan_first_certificates_through_the_phase_tree():
    # the merge rule of Section III (certificate of the union of two
    # certificates, pairwise in ceil(log2 M) rounds) with scan-first
    # certificates keeps the articulation points for any split
    rng = np.random.default_rng(57)

    def cert(e, V):
        f1, f2 = oracle.scan_first_certificate(e, V)
        return np.concatenate([f1, f2]).astype(np.int32).reshape(-1, 2)

    for t in range(200):
        V = int(rng.integers(2, 30))
        e = rng.integers(0, V, size=(int(rng.integers(0, 5 * V)), 2)).astype(np.int32)
        M = int(rng.integers(1, 9))
        E = e.shape[0]
        X = [cert(e[(i * E) // M:((i + 1) * E) // M], V) for i in range(M)]
        step = 1
        while step < M:
            for i in range(0, M, 2 * step):
                if i + step < M:
                    X[i] = cert(np.concatenate([X[i], X[i + step]]), V)
            step *= 2
        assert X[0].shape[0] <= 2 * (V - 1)
        assert np.array_equal(oracle.articulation_points(X[0], V), oracle.articulation_points(e, V)), (V, M, e.tolist())
