"""Parity on the paper's figure workloads (Figs. 2-4 give |V|, |E| and M only;
graphgen.figure supplies a planted-cluster graph of that size): bit-exact
bridge sets against the CPU oracle at every point of the three sweeps, with
both final steps."""
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


@pytest.mark.parametrize("fig", sorted(graphgen.FIGURES))
def test_figure_sweep_bit_exact(fig):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_07346_amd as br
    ctx = br.Context(0)
    last = None
    for V, E, M in graphgen.FIGURES[fig]:
        if last is None or last[0] != (V, E):
            g = graphgen.figure(V, E)
            last = ((V, E), g, torch.from_numpy(g.edges).cuda(), oracle.bridges(g.edges, g.V))
        _, g, d, want = last
        for mode in (0, 1):
            ctx.set_final_step(mode)
            say("%s V=%d E=%d M=%d final step %d" % (fig, g.V, g.E, M, mode))
            assert np.array_equal(ctx.find(d, g.V, M), want)
    ctx.close()
