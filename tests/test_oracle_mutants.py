"""The oracle pins must reject plausible mistakes in the oracle.

Each mutant is a copy of oracle/tarjan.c with one planted mistake, built on
the CPU into a temporary library; the brute-force and hand-worked pins must
fail for every mutant.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from test_oracle import HAND

SRC = os.path.join(os.path.dirname(oracle.__file__), "tarjan.c")

MUTANTS = {
    "bridge_test_ge": ("if (low[x] > disc[p]) {", "if (low[x] >= disc[p]) {"),
    "parent_by_vertex": ("if ((int64_t)eid[a] == st_pe[sp]) continue;",
                         "if (sp > 0 && y == st_v[sp - 1]) continue;"),
    "no_low_propagation": ("if (low[x] < low[p]) low[p] = low[x];", ";"),
    "first_root_only": ("for (int64_t s = 0; s < V; s++) {", "for (int64_t s = 0; s < (V > 0 ? 1 : 0); s++) {"),
    "back_edge_ignored": ("} else if (disc[y] < low[x]) {", "} else if (0) {"),
    "pair_order_swapped": ("br[nb++] = (a << 32) | b;", "br[nb++] = (b << 32) | a;"),
}


def build_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, name
    path = os.path.join(tmp, name + ".c")
    open(path, "w").write(src.replace(old, new))
    so = os.path.join(tmp, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", path, "-o", so])
    lib = ctypes.CDLL(so)
    lib.oracle_bridges.restype = ctypes.c_int
    lib.oracle_bridges.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    return lib


def run(lib, e, V):
    e = np.ascontiguousarray(np.asarray(e, dtype=np.int32).reshape(-1, 2))
    out = np.zeros((max(V - 1, 1), 2), dtype=np.int32)
    n = ctypes.c_int64(0)
    lib.oracle_bridges(e.ctypes.data, e.shape[0], V, out.ctypes.data, out.shape[0], ctypes.byref(n))
    return out[:n.value].copy()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_mutant(name, tmp)
        caught = False
        for c in HAND:
            want = np.array(sorted(c["b"]), dtype=np.int32).reshape(-1, 2)
            if not np.array_equal(run(lib, c["e"], c["V"]), want):
                caught = True
                break
        rng = np.random.default_rng(11)
        for _ in range(200):
            if caught:
                break
            V = int(rng.integers(1, 13))
            e = rng.integers(0, V, size=(int(rng.integers(0, 3 * V + 1)), 2)).astype(np.int32)
            if not np.array_equal(run(lib, e, V), oracle.brute_bridges(e, V)):
                caught = True
        assert caught, "mutant %s survived the pins" % name
