"""CPU checks of the certificate properties the hot path relies on.

The sequential reference (Algorithm 2 and the Section III phase tree in
oracle/certificate.c) must produce certificates that pass the property
checker, for any chunk count M; and the checker must flag broken
certificates.  These pin the properties before any GPU code exists.
"""
import numpy as np
import pytest

import graphgen
import oracle


def rand_multigraph(rng, V, E):
    return rng.integers(0, V, size=(E, 2)).astype(np.int32)


@pytest.mark.parametrize("seed", range(6))
def test_certificate_properties_random(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 300))
    e = rand_multigraph(rng, V, int(rng.integers(0, 8 * V)))
    f1, f2 = oracle.certificate(e, V)
    assert oracle.check_certificate(f1, f2, e, V) == []
    # Algorithm 2: F is a maximal spanning forest of G
    assert f1.shape[0] == V - oracle.components(e, V)


def test_certificate_of_small_workload():
    g = graphgen.config("small")
    f1, f2 = oracle.certificate(g.edges, g.V)
    assert oracle.check_certificate(f1, f2, g.edges, g.V) == []
    assert f1.shape[0] + f2.shape[0] <= 2 * (g.V - 1)


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 16, 100, 9949, 10051, 10058, 20000])
def test_phase_tree_m_invariance_small(M):
    g = graphgen.config("small")
    f1, f2, sizes = oracle.phase_tree(g.edges, g.V, M)
    assert np.all(sizes <= 2 * (g.V - 1))
    assert oracle.check_certificate(f1, f2, g.edges, g.V) == []
    assert len(sizes) == 1 + int(np.ceil(np.log2(M))) if M > 1 else len(sizes) == 1


@pytest.mark.parametrize("M", [1, 16, 256, 1024])
def test_phase_tree_dense_sweep(M):
    g = graphgen.config("dense")
    f1, f2, sizes = oracle.phase_tree(g.edges, g.V, M)
    assert np.all(sizes <= 2 * (g.V - 1))
    s = np.concatenate([f1, f2])
    assert np.array_equal(oracle.bridges(s, g.V), oracle.bridges(g.edges, g.V))
    assert f1.shape[0] == g.V - oracle.components(g.edges, g.V)


def test_phase_tree_empty_chunks_and_tiny():
    e = np.array([[0, 1], [1, 2], [2, 0], [2, 3]], dtype=np.int32)
    for M in [1, 2, 3, 4, 5, 7, 64]:
        f1, f2, _ = oracle.phase_tree(e, 4, M)
        assert oracle.check_certificate(f1, f2, e, 4) == []
    f1, f2, _ = oracle.phase_tree(np.zeros((0, 2), np.int32), 5, 3)
    assert f1.shape[0] == 0 and f2.shape[0] == 0
    f1, f2, _ = oracle.phase_tree(np.array([[0, 0], [0, 0]], np.int32), 1, 2)
    assert f1.shape[0] == 0 and f2.shape[0] == 0


def test_checker_flags_broken_certificates():
    rng = np.random.default_rng(9)
    V = 60
    e = rand_multigraph(rng, V, 400)
    f1, f2 = oracle.certificate(e, V)
    assert oracle.check_certificate(f1, f2, e, V) == []
    # a dropped F edge: F no longer spans
    assert "F not spanning" in oracle.check_certificate(f1[1:], f2, e, V)
    # F' edge that closes a cycle inside F'
    cyc = np.concatenate([f2, f2[:1]])
    assert "F' not a forest" in oracle.check_certificate(f1, cyc, e, V)
    # an edge that is not in the input
    keys = set(map(tuple, np.sort(e, 1).tolist()))
    fake = next((a, b) for a in range(V) for b in range(a + 1, V) if (a, b) not in keys)
    assert "S not a sub-multiset of E" in oracle.check_certificate(f1, np.concatenate([f2, [fake]]), e, V)
    # dropping all of F' changes the bridges of a 2-edge-connected graph
    cyc_g = np.stack([np.arange(V), (np.arange(V) + 1) % V], 1).astype(np.int32)
    g1, g2 = oracle.certificate(cyc_g, V)
    assert "bridges(S) != bridges(G)" in oracle.check_certificate(g1, g2[:0], cyc_g, V)
