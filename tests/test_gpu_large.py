"""Full-size parity on the large workloads, in the configuration bench.py
times (M = 4096 chunks: 12 merge rounds).

* ``large``: 1,024 complete clusters of 256 vertices, 996,147,200 uniform
  inter-cluster edges, cluster tree, 5,000 pendant vertices: V = 267,144,
  E = 1,029,576,583 (8.2 GB of edges).  The uniform cross edges cover every
  tree edge, so the bridges are exactly the 5,000 pendant edges.
* ``large_blocked``: the same clusters with 170,393,600 cross edges kept
  inside 32 blocks of 32 clusters and a block-structured cluster tree
  (E = 203,822,983): the 31 tree edges between blocks survive every merge
  round as bridges, next to the 5,000 pendant edges.

The expected bridge sets were written by tests/golden/make_golden.py from the
CPU oracle (no GPU value is stored); each test also re-derives them from the
planted structure before comparing.
"""
import hashlib
import os
import sys
import time

import numpy as np
import pytest

import graphgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def read_golden(name):
    head, rows = "", []
    for line in open(os.path.join(HERE, "%s_bridges.txt" % name)):
        if line.startswith("#"):
            head += line
        else:
            u, v = line.split()
            rows.append((int(u), int(v)))
    return head, np.array(rows, dtype=np.int32).reshape(-1, 2)


def keys_of(e):
    e = np.sort(np.asarray(e, dtype=np.int64), 1)
    return np.sort(e[:, 0] << 32 | e[:, 1])


def generate_checked(name, head):
    t0 = time.time()
    say("%s: generating" % name)
    g = graphgen.config(name)
    say("%s: generated in %.1f s" % (name, time.time() - t0))
    assert ("V %d E %d" % (g.V, g.E)) in head
    h = hashlib.sha256()
    for i in range(0, g.E, 1 << 24):
        h.update(g.edges[i:i + (1 << 24)].tobytes())
    assert h.hexdigest() in head, "generated edges differ from the ones the golden file was written for"
    say("%s: edge digest matches (%.1f s)" % (name, time.time() - t0))
    return g


def run_both_final_steps(name, d, V, Ms, want, tuned=False):
    # the plan the size rules give, then (tuned) the one the tuner picks for
    # this shape -- the launch configuration bench.py times
    import paper_2108_07346_amd as br
    ctx = br.Context(0)
    for M in Ms:
        for plan in (("size rules", "tuned") if tuned else ("size rules",)):
            if plan == "tuned":
                say("%s: M=%d tuner %s" % (name, M, ctx.autotune(d, V, M)))
            for mode in (1, 0):
                ctx.set_final_step(mode)
                say("%s: M=%d %s, final step %d" % (name, M, plan, mode))
                got = ctx.find(d, V, M)
                assert np.array_equal(got, want), (M, plan, mode)
    ctx.close()


@pytest.mark.skipif(not os.path.exists(os.path.join(HERE, "large_bridges.txt")),
                    reason="golden file not generated (tests/golden/make_golden.py large)")
def test_large_workload_bit_exact():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    head, want = read_golden("large")
    g = generate_checked("large", head)
    assert np.array_equal(keys_of(want), keys_of(g.pend))          # planted: exactly the pendant edges
    say("large: uploading %d edges" % g.E)
    d = torch.from_numpy(g.edges).cuda()
    V = g.V
    del g
    run_both_final_steps("large", d, V, (4096,), want, tuned=True)


@pytest.mark.skipif(not os.path.exists(os.path.join(HERE, "large_blocked_bridges.txt")),
                    reason="golden file not generated (tests/golden/make_golden.py large_blocked)")
def test_large_blocked_tree_bridges_survive_every_merge_round():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    head, want = read_golden("large_blocked")
    g = generate_checked("large_blocked", head)
    blk = g.cluster[g.tree] // 32
    between = g.tree[blk[:, 0] != blk[:, 1]]
    assert between.shape[0] == 31
    planted = np.concatenate([g.pend, between])
    assert np.array_equal(keys_of(want), keys_of(planted))         # pendant edges + the block tree's edges
    d = torch.from_numpy(g.edges).cuda()
    V = g.V
    del g
    run_both_final_steps("large_blocked", d, V, (4096, 512, 1), want)
