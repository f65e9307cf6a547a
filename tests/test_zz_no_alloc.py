"""br_cert_build_static (the certificate in the library's fixed device array,
for callers that cannot allocate) against br_cert_build on the same inputs.

Certificates are not unique (any maximal forests do), so the two outputs are
compared by what every valid certificate of the input shares: |F| = V - c(G)
exactly, the certificate properties (forests, F spanning, sub-multiset of the
input, Lemma 1's size bound) and the bridge set, bit for bit.  Two calls in a
row, the second with a smaller input, so that stale contents of the array
would show."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_same_as_cert_build(ctx, g, M):
    d = torch.from_numpy(g.edges).cuda()
    cap = max(min(g.E, 2 * (g.V - 1)), 1)
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    s1, s2 = ctx.cert_build_static(d, g.V, M, out=out, counts=counts)
    a1, a2 = ctx.cert_build(d, g.V, M)
    s1, s2, a1, a2 = (x.cpu().numpy() for x in (s1, s2, a1, a2))
    say("V=%d E=%d M=%d: static |F|=%d |F'|=%d, workspace |F|=%d |F'|=%d" %
        (g.V, g.E, M, s1.shape[0], s2.shape[0], a1.shape[0], a2.shape[0]))
    assert s1.shape[0] == a1.shape[0] == g.V - oracle.components(g.edges, g.V)
    assert oracle.check_certificate(s1, s2, g.edges, g.V) == []
    assert oracle.check_certificate(a1, a2, g.edges, g.V) == []
    want = oracle.bridges(g.edges, g.V)
    assert np.array_equal(oracle.bridges(np.concatenate([s1, s2]), g.V), want)
    assert np.array_equal(oracle.bridges(np.concatenate([a1, a2]), g.V), want)


def test_static_scratch_matches_workspace_path_twice_then_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    ctx = br.Context(0)
    check_same_as_cert_build(ctx, graphgen.config("dense"), 16)     # fills much of the array
    check_same_as_cert_build(ctx, graphgen.config("small"), 4)      # smaller: stale contents must not leak
    check_same_as_cert_build(ctx, graphgen.config("small"), 100)
    e = np.zeros((0, 2), np.int32)
    s1, s2 = ctx.cert_build_static(torch.zeros((0, 2), dtype=torch.int32, device="cuda"), 5, 3)
    assert s1.shape[0] == 0 and s2.shape[0] == 0
    # beyond the array: a clear error before any device work
    big = torch.zeros((1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(br.BridgeError) as ei:
        ctx.cert_build_static(big, 8 << 20, 4)
    assert ei.value.code == br.BR_ENOMEM and "scratch" in str(ei.value)
    ctx.close()
