"""Full-size parity on the large workload (1,024 complete clusters of 256
vertices, 996,147,200 uniform inter-cluster edges, cluster tree, 5,000 pendant
vertices: V = 267,144, E = 1,029,576,583, 8.2 GB of edges) at M = 4096, the
configuration bench.py times with --workload large.

The expected bridge set was written by tests/golden/make_golden.py from the
CPU oracle (no GPU value is stored); the test also re-derives its planted
structure: the uniform cross edges cover every tree edge, so the bridges are
exactly the 5,000 pendant edges.
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import graphgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_bridges.txt")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def read_golden():
    head, rows = "", []
    for line in open(GOLDEN):
        if line.startswith("#"):
            head += line
        else:
            u, v = line.split()
            rows.append((int(u), int(v)))
    return head, np.array(rows, dtype=np.int32).reshape(-1, 2)


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated (tests/golden/make_golden.py large)")
def test_large_workload_bit_exact():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    head, want = read_golden()
    import time
    t0 = time.time()
    say("large: generating")
    g = graphgen.config("large")
    say("large: generated in %.1f s" % (time.time() - t0))
    assert ("V %d E %d" % (g.V, g.E)) in head
    h = hashlib.sha256()
    for i in range(0, g.E, 1 << 24):
        h.update(g.edges[i:i + (1 << 24)].tobytes())
    assert h.hexdigest() in head, "generated edges differ from the ones the golden file was written for"
    say("large: edge digest matches (%.1f s)" % (time.time() - t0))
    pend = np.sort(np.stack([g.pend.min(1), g.pend.max(1)], 1).astype(np.int64) @ np.array([1 << 32, 1]))
    keys = want.astype(np.int64) @ np.array([1 << 32, 1])
    assert np.array_equal(np.sort(keys), pend)          # planted: exactly the pendant edges
    say("large: uploading %d edges" % g.E)
    d = torch.from_numpy(g.edges).cuda()
    del g
    ctx = br.Context(0)
    for mode in (0, 1):
        ctx.set_final_step(mode)
        say("large: M=4096 final step %d" % mode)
        got = ctx.find(d, 267144, 4096)
        assert np.array_equal(got, want)
    ctx.close()
