"""Writes the stored expected bridge sets used by the GPU tests.

Calls only the input generator (graphgen) and the CPU oracle (oracle): no
value here comes from the GPU path.  Run from the repository root:

    python tests/golden/make_golden.py large          # ~1.03e9 edges, ~45 GB host RAM
    python tests/golden/make_golden.py large_blocked  # ~2.0e8 edges

Each output file lists one bridge "u v" per line (u < v, ascending) after a
header naming the workload, V, E and a SHA-256 of the edge bytes.
"""
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def edge_digest(e):
    h = hashlib.sha256()
    step = 1 << 24
    for i in range(0, e.shape[0], step):
        h.update(e[i:i + step].tobytes())
    return h.hexdigest()


def write(name):
    t0 = time.time()
    g = graphgen.config(name)
    t1 = time.time()
    digest = edge_digest(g.edges)
    b = oracle.bridges(g.edges, g.V)
    t2 = time.time()
    path = os.path.join(HERE, "%s_bridges.txt" % name)
    with open(path, "w") as f:
        f.write("# workload %s seed 0: V %d E %d edges_sha256 %s\n" % (name, g.V, g.E, digest))
        f.write("# written by tests/golden/make_golden.py from the CPU oracle (generation %.1f s, oracle %.1f s)\n"
                % (t1 - t0, t2 - t1))
        for u, v in b.tolist():
            f.write("%d %d\n" % (u, v))
    print("%s: %d bridges -> %s" % (name, b.shape[0], path), flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["small", "dense"]:
        write(n)
