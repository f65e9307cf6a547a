"""The C-ABI library on a machine without a GPU: it builds, loads, exports
every entry point that include/bridges.h declares, and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2108_07346_amd as br

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bridges.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(br_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(br.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = br.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_null_and_bad_arguments_rejected_without_a_device():
    lib = br.load()
    n = ctypes.c_int64(0)
    assert lib.br_bridges_find(None, None, 0, 1, 1, None, 0, ctypes.byref(n), None) == br.BR_EINVAL
    assert b"null" in lib.br_last_error()
    assert lib.br_cert_build(None, None, 0, 1, 1, None, 0, None, None) == br.BR_EINVAL
    assert lib.br_cert_merge(None, None, 0, None, 0, 1, None, 0, None, None) == br.BR_EINVAL
    assert lib.br_bridges_find_batched(None, None, None, None, 0, 0, None, 0, None, None) == br.BR_EINVAL
    assert lib.br_set_profiling(None, 1) == br.BR_EINVAL
    assert lib.br_destroy(None) == br.BR_OK


def test_final_step_v_limit_is_two_to_the_29():
    # the calls that run a final step refuse V above 2^29 before touching the
    # context (so the check is visible without a device); at 2^29 itself the
    # next check (the null context) is the one that fires
    lib = br.load()
    n = ctypes.c_int64(0)
    for V, word in (((1 << 29) + 1, b"2^29"), (1 << 29, b"null"), (2147483647, b"2^29")):
        assert lib.br_bridges_find(None, None, 0, V, 1, None, 0, ctypes.byref(n), None) == br.BR_EINVAL
        assert word in lib.br_last_error()
        assert lib.br_two_edge_components(None, None, 0, V, 1, None, None, None) == br.BR_EINVAL
        assert word in lib.br_last_error()
        assert lib.br_bridge_tree(None, None, 0, V, 1, None, None, 0, None, None, None) == br.BR_EINVAL
        assert word in lib.br_last_error()
        assert lib.br_articulation_points(None, None, 0, V, None, 0, ctypes.byref(n), None) == br.BR_EINVAL
        assert word in lib.br_last_error()
    # the certificate calls take any V up to 2^31 - 1 (null context here)
    assert lib.br_cert_build(None, None, 0, 2147483647, 1, None, 0, None, None) == br.BR_EINVAL
    assert b"null" in lib.br_last_error()


def test_create_fails_cleanly_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = br.load().br_create(ctypes.byref(h), 0)
    assert rc in (br.BR_EHIP, br.BR_EINVAL) and not h


def test_max_v_limit():
    assert br.batched_max_v() >= 64


def test_server_create_fails_cleanly_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert br.load().br_server_create(ctypes.byref(h), 0, 1 << 30, 4) in (br.BR_EHIP, br.BR_EINVAL)
    assert br.load().br_server_create(ctypes.byref(h), 0, 0, 4) == br.BR_EINVAL
    t = ctypes.c_uint64(0)
    assert br.load().br_submit(None, None, 0, 1, ctypes.byref(t)) == br.BR_EINVAL


def test_certificate_bridges_host_entry_matches_oracle():
    import numpy as np
    import graphgen
    import oracle
    g = graphgen.config("small")
    for M in (1, 4, 33):
        f1, f2, _ = oracle.phase_tree(g.edges, g.V, M)
        assert np.array_equal(br.certificate_bridges(f1, f2, g.V), oracle.bridges(g.edges, g.V))
    rng = np.random.default_rng(0)
    for _ in range(200):
        V = int(rng.integers(1, 30))
        e = rng.integers(0, V, size=(int(rng.integers(0, 60)), 2)).astype(np.int32)
        k = int(rng.integers(0, e.shape[0] + 1))
        assert np.array_equal(br.certificate_bridges(e[:k], e[k:], V), oracle.bridges(e, V))
    with pytest.raises(br.BridgeError):
        br.certificate_bridges(np.array([[0, 3]]), np.zeros((0, 2)), 3)


def test_certificate_bridges_many_keys():
    # relabelled random recursive trees: every edge is a bridge, so the
    # canonical ordering of many keys (the radix path) is checked against
    # numpy's lexicographic sort; a chord per tree makes some edges non-bridges
    import numpy as np
    import oracle
    rng = np.random.default_rng(1)
    for V in (65, 1000, 70000, 300000):
        i = np.arange(1, V, dtype=np.int64)
        par = (rng.random(V - 1) * i).astype(np.int64)
        relabel = rng.permutation(V).astype(np.int32)
        e = relabel[np.stack([par, i], 1)]
        s = np.sort(e, 1)
        want = s[np.lexsort((s[:, 1], s[:, 0]))]
        assert np.array_equal(br.certificate_bridges(e, np.zeros((0, 2), np.int32), V), want)
        chord = np.array([[relabel[0], relabel[V - 1]]], dtype=np.int32)
        if V <= 70000:
            assert np.array_equal(br.certificate_bridges(e, chord, V), oracle.bridges(np.concatenate([e, chord]), V))
