"""TEST INFRASTRUCTURE ONLY -- the CPU oracle for the bridge method.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2108_07346_amd``) never imports, links or calls it, and the two share
no code; both are fed by the seeded generator in ``graphgen``.

Contents
--------
``bridges(edges, V)``
    The oracle proper: a plain iterative low-link DFS over the whole graph
    (Algorithm 1 of Section IV-A, with the readings listed in ``tarjan.c``),
    returning the canonical bridge set: (min, max) pairs sorted ascending.
``brute_bridges(edges, V)``
    The definition of Section I written out for tiny graphs: an edge is a
    bridge iff removing it increases the number of connected components.
``certificate(edges, V)`` / ``phase_tree(edges, V, M)``
    Sequential Algorithm 2 and the Section III phase tree (``certificate.c``).
``check_certificate(f1, f2, edges, V)``
    The properties any valid certificate has (forests, disjointness, subset
    of the input, size bound of Lemma 1, same components and bridges), used
    to check certificates that are correct but not unique.
``components(edges, V)``
    Number of connected components (scipy's graph routine).
``articulation_points(edges, V)`` / ``brute_articulation_points(edges, V)``
    The abstract's "failure points": vertices whose removal increases the
    number of components -- by the low-link search (``articulation.c``) and
    by the definition written out for tiny graphs.
``scan_first_certificate(edges, V)``
    Two scan-first (breadth-first) forests, the second on the vertex pairs the
    first does not use: the certificate form under which articulation points
    survive (checked against the definition in the tests).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_DIR, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C oracle into liboracle.so (host C, gcc, no GPU code)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall",
                           os.path.join(_DIR, "tarjan.c"), os.path.join(_DIR, "certificate.c"),
                           os.path.join(_DIR, "articulation.c"), "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_bridges.restype = ctypes.c_int
    lib.oracle_bridges.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(i64)]
    lib.oracle_certificate.restype = ctypes.c_int
    lib.oracle_certificate.argtypes = [vp, i64, i64, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64)]
    lib.oracle_phase_tree.restype = ctypes.c_int
    lib.oracle_phase_tree.argtypes = [vp, i64, i64, i64, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
    lib.oracle_articulation_points.restype = ctypes.c_int
    lib.oracle_articulation_points.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(i64)]
    _lib = lib
    return lib


def _as_edges(edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    return e


_ERR = {-1: "bad arguments", -2: "vertex id out of range", -3: "out of host memory"}


def bridges(edges, V: int) -> np.ndarray:
    """Canonical bridge set of the multigraph (V, edges): int32 [B, 2], u < v, sorted."""
    e = _as_edges(edges)
    lib = _load()
    n = ctypes.c_int64(0)
    out = np.empty((max(int(V) - 1, 1), 2), dtype=np.int32)
    rc = lib.oracle_bridges(e.ctypes.data, e.shape[0], int(V), out.ctypes.data, out.shape[0], ctypes.byref(n))
    if rc:
        raise ValueError("oracle_bridges: " + _ERR.get(rc, str(rc)))
    return out[:n.value].copy()


def certificate(edges, V: int):
    """Sequential Algorithm 2 on the list order: returns (F, F') as int32 [n, 2] arrays."""
    e = _as_edges(edges)
    lib = _load()
    m = max(min(e.shape[0], int(V) - 1), 1)
    f1 = np.empty((m, 2), dtype=np.int32)
    f2 = np.empty((m, 2), dtype=np.int32)
    n1, n2 = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib.oracle_certificate(e.ctypes.data, e.shape[0], int(V), f1.ctypes.data, ctypes.byref(n1),
                                f2.ctypes.data, ctypes.byref(n2))
    if rc:
        raise ValueError("oracle_certificate: " + _ERR.get(rc, str(rc)))
    return f1[:n1.value].copy(), f2[:n2.value].copy()


def phase_tree(edges, V: int, M: int):
    """Section III phase tree over M contiguous chunks.

    Returns (F, F', sizes) where sizes[q] is the largest certificate after
    phase q (q = 0 is the per-chunk phase)."""
    e = _as_edges(edges)
    lib = _load()
    cap = max(min(e.shape[0], 2 * (int(V) - 1)), 1)
    x0 = np.empty((cap, 2), dtype=np.int32)
    n1, n2 = ctypes.c_int64(0), ctypes.c_int64(0)
    R = 0
    while (1 << R) < M:
        R += 1
    sizes = np.zeros(R + 1, dtype=np.int64)
    rc = lib.oracle_phase_tree(e.ctypes.data, e.shape[0], int(V), int(M), x0.ctypes.data, ctypes.byref(n1),
                               ctypes.byref(n2), sizes.ctypes.data)
    if rc:
        raise ValueError("oracle_phase_tree: " + _ERR.get(rc, str(rc)))
    return x0[:n1.value].copy(), x0[n1.value:n1.value + n2.value].copy(), sizes


def two_edge_labels(edges, V: int) -> np.ndarray:
    """2-edge-connected classes: the components of G without its bridges
    (Section I's bridges from the oracle above); label = smallest vertex of
    the class.  Plain sequential union-find."""
    e = _as_edges(edges)
    b = bridges(e, V)
    bset = set(map(tuple, b.tolist()))
    par = np.arange(V, dtype=np.int64)

    def find(x):
        r = x
        while par[r] != r:
            r = par[r]
        while par[x] != r:
            par[x], x = r, par[x]
        return r

    for u, v in e.tolist():
        if u == v or (min(u, v), max(u, v)) in bset:
            continue
        a, c = find(u), find(v)
        if a != c:
            par[max(a, c)] = min(a, c)
    return np.array([find(x) for x in range(V)], dtype=np.int32)


def bridge_tree(edges, V: int):
    """The bridge tree of Section I's bridges: the graph whose nodes are the
    2-edge-connected classes (labelled by their smallest vertex, as in
    two_edge_labels) and whose edges are the bridges, each joining the classes
    of its two endpoints.  Returns (labels int32 [V], tree edges int32 [B, 2]
    as (min, max) class labels, sorted).  A forest: one tree per connected
    component of the graph."""
    e = _as_edges(edges)
    lab = two_edge_labels(e, V)
    b = bridges(e, V)
    t = np.stack([lab[b[:, 0]], lab[b[:, 1]]], 1) if b.shape[0] else np.zeros((0, 2), np.int32)
    t = np.sort(t, 1).astype(np.int32)
    if t.shape[0]:
        t = t[np.lexsort((t[:, 1], t[:, 0]))]
    return lab, t


def brute_two_edge_labels(edges, V: int) -> np.ndarray:
    """The definition for tiny graphs: u and v share a class iff they stay
    connected after removing any single edge."""
    e = [(int(a), int(b)) for a, b in _as_edges(edges)]

    def comp(pairs):
        par = list(range(V))

        def f(x):
            while par[x] != x:
                x = par[x]
            return x
        for a, b in pairs:
            ra, rb = f(a), f(b)
            if ra != rb:
                par[ra] = rb
        return [f(x) for x in range(V)]

    cs = [comp(e)] + [comp(e[:i] + e[i + 1:]) for i in range(len(e))]
    lab = []
    for v in range(V):
        lab.append(min(u for u in range(V) if all(c[u] == c[v] for c in cs)))
    return np.array(lab, dtype=np.int32)


# ---- definitions written out for tiny graphs ---------------------------------

def _count_components_py(V: int, pairs) -> int:
    par = list(range(V))

    def find(x):
        while par[x] != x:
            x = par[x]
        return x

    c = V
    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra != rb:
            par[ra] = rb
            c -= 1
    return c


def brute_bridges(edges, V: int) -> np.ndarray:
    """Section I's definition, pure Python, for tiny graphs: remove each edge
    and count components; return the canonical bridge set."""
    e = [(int(a), int(b)) for a, b in _as_edges(edges)]
    base = _count_components_py(V, e)
    out = set()
    for i, (a, b) in enumerate(e):
        if _count_components_py(V, e[:i] + e[i + 1:]) > base:
            out.add((min(a, b), max(a, b)))
    return np.array(sorted(out), dtype=np.int32).reshape(-1, 2)


def components(edges, V: int) -> int:
    """Number of connected components of (V, edges)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    e = _as_edges(edges)
    if V == 0:
        return 0
    m = sp.coo_matrix((np.ones(e.shape[0], dtype=np.float32), (e[:, 0], e[:, 1])), shape=(V, V)).tocsr()
    return int(connected_components(m, directed=False)[0])


def _canon_keys(e: np.ndarray) -> np.ndarray:
    e = _as_edges(e).astype(np.int64)
    lo, hi = np.minimum(e[:, 0], e[:, 1]), np.maximum(e[:, 0], e[:, 1])
    return np.sort(lo * (1 << 32) + hi)


def _is_forest(f: np.ndarray, V: int) -> bool:
    # a multigraph is a forest iff it has no self-loop and |F| = V - c(F)
    f = _as_edges(f)
    if np.any(f[:, 0] == f[:, 1]):
        return False
    return f.shape[0] == V - components(f, V)


def _multiset_subset(sub: np.ndarray, sup: np.ndarray) -> bool:
    a, b = _canon_keys(sub), _canon_keys(sup)
    ua, ca = np.unique(a, return_counts=True)
    ub, cb = np.unique(b, return_counts=True)
    idx = np.searchsorted(ub, ua)
    if np.any(idx >= ub.shape[0]):
        return False
    return bool(np.all(ub[idx] == ua) and np.all(cb[idx] >= ca))


def check_certificate(f1, f2, edges, V: int, check_bridges: bool = True) -> list:
    """Properties of a valid certificate F u F' of the multigraph (V, edges).

    Returns a list of violated properties (empty when valid):
      * F and F' are forests (Algorithm 2's union-find keeps no cycle);
      * F is spanning: c(F) = c(G);
      * F u F' is a sub-multiset of the input (S is a subset of E);
      * |F u F'| <= 2(V-1) (Lemma 1);
      * c(S) = c(G) and bridges(S) = bridges(G) (the certificate property
        of Section III, restricted to bridges).
    """
    bad = []
    f1, f2, e = _as_edges(f1), _as_edges(f2), _as_edges(edges)
    if not _is_forest(f1, V):
        bad.append("F not a forest")
    if not _is_forest(f2, V):
        bad.append("F' not a forest")
    cG = components(e, V)
    if components(f1, V) != cG:
        bad.append("F not spanning")
    s = np.concatenate([f1, f2])
    if not _multiset_subset(s, e):
        bad.append("S not a sub-multiset of E")
    if s.shape[0] > 2 * (V - 1):
        bad.append("|S| > 2(V-1)")
    if components(s, V) != cG:
        bad.append("c(S) != c(G)")
    if check_bridges and not np.array_equal(bridges(s, V), bridges(e, V)):
        bad.append("bridges(S) != bridges(G)")
    return bad


# ---- articulation points ("failure points" of the abstract) -------------------

def articulation_points(edges, V: int) -> np.ndarray:
    """Articulation points of (V, edges): int32 vertex ids ascending."""
    e = _as_edges(edges)
    lib = _load()
    n = ctypes.c_int64(0)
    out = np.empty(max(int(V), 1), dtype=np.int32)
    rc = lib.oracle_articulation_points(e.ctypes.data, e.shape[0], int(V), out.ctypes.data, out.shape[0],
                                        ctypes.byref(n))
    if rc:
        raise ValueError("oracle_articulation_points: " + _ERR.get(rc, str(rc)))
    return out[:n.value].copy()


def brute_articulation_points(edges, V: int) -> np.ndarray:
    """The definition for tiny graphs: v is an articulation point iff the
    graph without v (and its edges) has more components than the graph."""
    e = [(int(a), int(b)) for a, b in _as_edges(edges)]
    base = _count_components_py(V, e)
    out = []
    for v in range(V):
        rest = [(a if a < v else a - 1, b if b < v else b - 1) for a, b in e if a != v and b != v]
        if _count_components_py(V - 1, rest) > base:
            out.append(v)
    return np.array(out, dtype=np.int32)


def scan_first_certificate(edges, V: int):
    """Two scan-first search forests (F, F'): F by breadth-first search from
    the smallest vertex of each component, a vertex's parent being its
    smallest-id neighbour one level up (scanning each level's vertices in id
    order makes this a scan-first search); F' the same on the edges whose
    vertex pair is not a pair of F (parallel copies of F's pairs excluded).
    Returns int32 [n, 2] arrays of the chosen edges (as listed in the input)."""
    e = _as_edges(edges)
    forests = []
    banned = set()
    for _ in range(2):
        adj = [[] for _ in range(int(V))]
        for i, (a, b) in enumerate(e.tolist()):
            if a == b or (min(a, b), max(a, b)) in banned:
                continue
            adj[a].append((b, i))
            adj[b].append((a, i))
        level = [-1] * int(V)
        chosen = []
        for r in range(int(V)):
            if level[r] != -1:
                continue
            level[r] = 0
            front = [r]
            while front:
                cand = {}
                for u in sorted(front):
                    for w, i in adj[u]:
                        if level[w] == -1 and (w not in cand or (u, i) < cand[w]):
                            cand[w] = (u, i)
                for w, (u, i) in cand.items():
                    level[w] = level[u] + 1
                    chosen.append(i)
                front = list(cand)
        f = e[np.array(sorted(chosen), dtype=np.int64)] if chosen else np.zeros((0, 2), np.int32)
        forests.append(f)
        banned = {(min(a, b), max(a, b)) for a, b in f.tolist()}
    return forests[0], forests[1]
