"""Seeded synthetic inputs: planted-cluster multigraphs as int32 edge lists.

This module produces inputs only.  It contains none of the bridge method's
arithmetic, so both the CPU oracle and the GPU library may be fed from it.
The generator itself is C (``graphgen.c``); this file marshals arguments and
holds the workload recipes:

* ``small``  -- 20 clusters x 100 vertices, p=0.1, random cluster tree,
  30 pendant vertices; simple graph; M=4.
* ``dense``  -- 256 clusters x 256 vertices, p=0.5, cluster tree plus
  round(0.02 * 255) = 5 extra inter-cluster edges, 1,000 pendant vertices;
  simple graph; M in {1, 16, 256, 1024}.
* ``large``  -- 1,024 clusters x 256 vertices, p=1.0 (complete clusters),
  262,144 * 7,600 / 2 i.i.d. uniform inter-cluster edges (drawn with
  replacement, so a few parallel copies occur), cluster tree,
  5,000 pendant vertices; M=4096.
* ``large_blocked`` -- as ``large`` with 262,144 * 1,300 / 2 cross edges,
  each inside one of 32 blocks of 32 clusters, and a cluster tree made of a
  tree per block plus a tree over the blocks: the 31 tree edges between
  blocks and the 5,000 pendant edges are the bridges.
* ``batched`` -- 4,096 graphs; graph g has V log-uniform in [64, 4096],
  k uniform in {2..16} near-equal clusters, p uniform in [0.05, 0.5], a
  cluster tree and stochastic round(f * (k-1)) extra edges, f ~ U[0, 0.03].
* ``served`` -- request r: V log-uniform in [256, 131072], average degree d
  log-uniform in [64, 2048]; clusters of s = min(V, max(256, 2d)) vertices
  with p = min(1, d/(s-1)), tree, round(0.02 (k-1)) extra edges and
  round(0.015 V) pendant vertices.

Every graph's vertex ids are relabelled by a keyed bijection, its edge list
is permuted by a keyed bijection and each pair's orientation is flipped with
probability 1/2.  Outputs are bit-identical on every host and thread count.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_DIR, "libgraphgen.so")
_lib = None


def build() -> str:
    """Compile graphgen.c into libgraphgen.so (host C, gcc)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-Wall",
                           os.path.join(_DIR, "graphgen.c"), "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    lib.gg_plan.restype = vp
    lib.gg_plan.argtypes = [u64, i32, i64, ctypes.c_double, i64, i64, i64, ctypes.c_int, ctypes.c_int, i32]
    lib.gg_V.restype = i64
    lib.gg_V.argtypes = [vp]
    lib.gg_E.restype = i64
    lib.gg_E.argtypes = [vp]
    lib.gg_n_intra.restype = i64
    lib.gg_n_intra.argtypes = [vp]
    lib.gg_fill.restype = ctypes.c_int
    lib.gg_fill.argtypes = [vp, vp]
    lib.gg_planted.restype = None
    lib.gg_planted.argtypes = [vp, vp, vp, vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_cluster_of.restype = None
    lib.gg_cluster_of.argtypes = [vp, vp]
    lib.gg_unit.restype = ctypes.c_double
    lib.gg_unit.argtypes = [u64, u64, u64]
    _lib = lib
    return lib


@dataclass
class Graph:
    """One generated graph.  ``edges`` is int32 [E, 2]; ids are in [0, V)."""
    edges: np.ndarray
    V: int
    tree: np.ndarray          # planted cluster-tree edges [k-1, 2]
    extra: np.ndarray         # extra inter-cluster edges [n_extra, 2]
    pend: np.ndarray          # pendant edges [n_pend, 2] (pendant vertex first)
    n_intra: int
    cluster: np.ndarray       # cluster index per vertex, -1 for pendant vertices
    params: dict = field(default_factory=dict)

    @property
    def E(self) -> int:
        return int(self.edges.shape[0])


def planted(seed: int, k: int, vc: int, p: float, n_extra: int = 0, n_cross: int = 0,
            n_pend: int = 0, relabel: bool = True, shuffle: bool = True, cross_block: int = 0) -> Graph:
    """Generate one planted-cluster graph (see the module docstring).  With
    cross_block = b > 0 (b >= 2 dividing k) the cross edges stay inside blocks
    of b consecutive clusters and the cluster tree is a tree per block plus a
    tree over the blocks."""
    lib = _load()
    h = lib.gg_plan(seed & (2**64 - 1), k, vc, float(p), n_extra, n_cross, n_pend, int(relabel), int(shuffle),
                    int(cross_block))
    if not h:
        raise ValueError("graphgen: invalid parameters k=%d vc=%d p=%g extra=%d cross=%d pend=%d block=%d"
                         % (k, vc, p, n_extra, n_cross, n_pend, cross_block))
    try:
        V, E = lib.gg_V(h), lib.gg_E(h)
        edges = np.empty((E, 2), dtype=np.int32)
        if lib.gg_fill(h, edges.ctypes.data) != 0:
            raise MemoryError("graphgen: out of host memory for %d edges" % E)
        tree = np.empty((max(k - 1, 0), 2), dtype=np.int32)
        extra = np.empty((n_extra, 2), dtype=np.int32)
        pend = np.empty((n_pend, 2), dtype=np.int32)
        lib.gg_planted(h, tree.ctypes.data, extra.ctypes.data, pend.ctypes.data)
        cluster = np.empty(V, dtype=np.int32)
        lib.gg_cluster_of(h, cluster.ctypes.data)
        n_intra = lib.gg_n_intra(h)
    finally:
        lib.gg_free(h)
    return Graph(edges, int(V), tree, extra, pend, int(n_intra), cluster,
                 dict(seed=seed, k=k, vc=vc, p=p, n_extra=n_extra, n_cross=n_cross, n_pend=n_pend,
                      cross_block=cross_block))


def unit(seed: int, tag: int, i: int) -> float:
    """Uniform double in [0, 1): draw i of stream `tag` under `seed`."""
    return _load().gg_unit(seed & (2**64 - 1), tag, i)


# ---- workload recipes -------------------------------------------------------

PLAIN = {
    "small": dict(k=20, vc=2000, p=0.1, n_extra=0, n_cross=0, n_pend=30, M=[4]),
    "dense": dict(k=256, vc=65536, p=0.5, n_extra=5, n_cross=0, n_pend=1000, M=[1, 16, 256, 1024]),
    "large": dict(k=1024, vc=262144, p=1.0, n_extra=0, n_cross=262144 * 7600 // 2, n_pend=5000, M=[4096]),
    # the large layout with the cross edges kept inside 32 blocks of 32
    # clusters (average cross degree 1,300: about 2.0e8 edges), so that the 31
    # tree edges between blocks stay bridges through every merge round
    "large_blocked": dict(k=1024, vc=262144, p=1.0, n_extra=0, n_cross=262144 * 1300 // 2, n_pend=5000,
                          cross_block=32, M=[4096, 512]),
}


def config(name: str, seed: int = 0) -> Graph:
    """One of the plain workloads: 'small', 'dense', 'large' or 'large_blocked'."""
    c = dict(PLAIN[name])
    c.pop("M")
    g = planted(seed, **c)
    g.params["name"] = name
    return g


def _key2(seed: int, idx: int) -> int:
    return (seed * 0x9E3779B97F4A7C15 + idx * 0xD1B54A32D192ED03 + 1) & (2**64 - 1)


def batched_params(seed: int, g: int) -> dict:
    """Recipe of graph g of the batched workload."""
    s = _key2(seed, g)
    V = int(round(math.exp(math.log(64) + unit(s, 1, 0) * (math.log(4096) - math.log(64)))))
    k = 2 + int(unit(s, 2, 0) * 15)
    p = 0.05 + unit(s, 3, 0) * 0.45
    f = unit(s, 4, 0) * 0.03
    x = f * (k - 1)
    n_extra = int(math.floor(x)) + (1 if unit(s, 5, 0) < x - math.floor(x) else 0)
    return dict(seed=s, k=k, vc=V, p=p, n_extra=n_extra, n_cross=0, n_pend=0)


@dataclass
class Batch:
    edges: np.ndarray      # int32 [sum E_g, 2], graph-local ids
    offsets: np.ndarray    # int64 [G+1]
    V: np.ndarray          # int32 [G]
    graphs: list           # per-graph params

    @property
    def G(self) -> int:
        return int(self.V.shape[0])

    def graph(self, g: int) -> np.ndarray:
        return self.edges[self.offsets[g]:self.offsets[g + 1]]


def batched(seed: int = 0, n_graphs: int = 4096, threads: int | None = None) -> Batch:
    """The batched workload: n_graphs independent graphs packed CSR-style."""
    params = [batched_params(seed, g) for g in range(n_graphs)]

    def one(pr):
        return planted(**pr)

    nt = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(nt) as ex:
        gs = list(ex.map(one, params))
    off = np.zeros(n_graphs + 1, dtype=np.int64)
    off[1:] = np.cumsum([x.E for x in gs])
    edges = np.empty((int(off[-1]), 2), dtype=np.int32)
    for i, x in enumerate(gs):
        edges[off[i]:off[i + 1]] = x.edges
    return Batch(edges, off, np.array([x.V for x in gs], dtype=np.int32), params)


def figure_params(V: int, E: int, seed: int = 0) -> dict:
    """Recipe of the paper's figure workloads (Figs. 2-4 give only |V| and |E|):
    clusters of 100 vertices holding about a tenth of the edges, the rest
    uniform between clusters, a cluster tree and V/1000 pendant vertices; V
    counts all vertices; E is met to within ~2% (the intra-cluster edges are Bernoulli draws)."""
    pend = max(1, V // 1000)
    vc = V - pend
    k = max(2, vc // 100)
    pairs = k * 100 * 99 / 2 if vc >= 200 else vc * (vc - 1) / 2
    intra = min(0.1 * E, pairs)
    p = min(1.0, intra / max(pairs, 1))
    cross = max(0, E - int(round(p * pairs)) - (k - 1) - pend)
    return dict(seed=(seed * 0x9E3779B97F4A7C15 + V * 31 + E) & (2**64 - 1), k=k, vc=vc, p=p, n_extra=0,
                n_cross=cross, n_pend=pend)


# Fig. 2: |E| = 10^7, |V| = 10^5, M swept; Fig. 3: |E| = 10^5, M = 10, |V| swept;
# Fig. 4: |V| = 10^5, M = 10, |E| swept.
FIGURES = {
    "fig2": [(100_000, 10_000_000, m) for m in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)],
    "fig3": [(v, 100_000, 10) for v in (1_000, 3_000, 10_000, 30_000, 100_000)],
    "fig4": [(100_000, e, 10) for e in (100_000, 300_000, 1_000_000, 3_000_000, 10_000_000)],
}


def figure(V: int, E: int, seed: int = 0) -> Graph:
    return planted(**figure_params(V, E, seed))


def served_params(seed: int, r: int) -> dict:
    """Recipe of request r of the served workload."""
    s = _key2(seed ^ 0x5E77ED, r)
    V = int(round(math.exp(math.log(256) + unit(s, 1, 0) * (math.log(131072) - math.log(256)))))
    d = math.exp(math.log(64) + unit(s, 2, 0) * (math.log(2048) - math.log(64)))
    size = min(V, max(256, int(round(2 * d))))
    p = min(1.0, d / (size - 1))
    k = max(1, int(round(V / size)))
    return dict(seed=s, k=k, vc=V, p=p, n_extra=int(round(0.02 * (k - 1))), n_cross=0,
                n_pend=int(round(0.015 * V)))


def served_request(seed: int, r: int) -> Graph:
    return planted(**served_params(seed, r))
