"""The tuner: a choice measured in one process is kept in the file that
BR_AUTOTUNE_CACHE names and used, without measuring again, by a later
process; results stay bit-exact whatever plan the tuner picks."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, %r)
import numpy as np, torch, graphgen, oracle
import paper_2108_07346_amd as br
ctx = br.Context(0)
out = {}
g = graphgen.config("dense")
d = torch.from_numpy(g.edges).cuda()
out["plain"] = ctx.autotune(d, g.V, 16)
out["plain_ok"] = bool(np.array_equal(ctx.find(d, g.V, 16), oracle.bridges(g.edges, g.V)))
b = graphgen.batched(0, n_graphs=48)
db = torch.from_numpy(b.edges).cuda()
pairs, boff = ctx.find_batched(db, b.offsets, b.V, 0)
out["batched_chunk"] = int(ctx.profile()["rounds"])
out["batched_ok"] = all(np.array_equal(pairs[boff[i]:boff[i + 1]], oracle.bridges(b.graph(i), int(b.V[i])))
                        for i in range(b.G))
print("RESULT " + json.dumps(out), flush=True)
""" % ROOT


def run_child(cache):
    env = dict(os.environ, BR_AUTOTUNE_CACHE=cache)
    r = subprocess.run([sys.executable, "-u", "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    return json.loads(line[7:])


def test_tuned_choice_reloaded_by_a_later_process(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cache = str(tmp_path / "tune.json")
    first = run_child(cache)
    print("first process:", first, flush=True)
    assert first["plain"]["source"] == "measured" and first["plain_ok"] and first["batched_ok"]
    saved = json.load(open(cache))
    assert first["plain"]["key"] in saved
    bkeys = [k for k in saved if "|batched|" in k]
    assert len(bkeys) == 1 and {"chunk_edges", "blocks_per_cu"} <= set(saved[bkeys[0]])
    assert first["batched_chunk"] == int(saved[bkeys[0]]["chunk_edges"])
    second = run_child(cache)
    print("second process:", second, flush=True)
    assert second["plain"]["source"] == "cache"
    assert {k: v for k, v in second["plain"].items() if k != "source"} == \
           {k: v for k, v in first["plain"].items() if k != "source"}
    assert second["plain_ok"] and second["batched_ok"]
    assert second["batched_chunk"] == first["batched_chunk"]
    assert json.load(open(cache)) == saved            # nothing measured again


def test_every_tuner_candidate_is_exact():
    # each plan the tuner may pick gives the oracle's bridges (dense, large-state
    # random graph); the second graph has more vertices than the solo kernel's
    # claim tables have bits, so roots share claim bits
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(31)
    cases = []
    V = 150_000
    e = rng.integers(0, V, size=(600_000, 2)).astype(np.int32)
    cases.append((e, V, 256, [{"BR_SOLO": "0", "BR_TILE0": "1024"}, {"BR_SOLO": "0", "BR_PREM": "1"},
                              {"BR_SOLO": "1", "BR_SOLO_TOP": "1", "BR_PREM": "1"},
                              {"BR_SOLO": "1", "BR_SOLO_NBK": "0"}, {"BR_SOLO": "1", "BR_SOLO_NBK": "16", "BR_SOLO_NBK2": "1"},
                              {"BR_SOLO": "1", "BR_SOLO_TOP": "2", "BR_SOLO_MBK": "1"},
                              {"BR_SOLO": "1", "BR_SOLO_TOP": "2", "BR_SOLO_WM": "0"}] +
                  [{"BR_SOLO": "1", "BR_SOLO_VARIANT": str(v), "BR_SOLO_TOP": str(t)} for v in range(5) for t in (0, 3)]))
    V2 = 700_000
    e2 = rng.integers(0, V2, size=(1_400_000, 2)).astype(np.int32)
    cases.append((e2, V2, 512, [{"BR_SOLO": "1", "BR_SOLO_VARIANT": str(v), "BR_SOLO_TOP": str(t)}
                                for v in (0, 2, 4) for t in (0, 2)]))
    code = r"""
import os, sys
sys.path.insert(0, %r)
import numpy as np, torch
import paper_2108_07346_amd as br
e = np.load(sys.argv[1])
ctx = br.Context(0)
got = ctx.find(torch.from_numpy(e).cuda(), int(sys.argv[3]), int(sys.argv[4]))
np.save(sys.argv[2], got)
""" % (ROOT,)
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        for ci, (e, V, M, envs) in enumerate(cases):
            want = oracle.bridges(e, V)
            ein = os.path.join(td, "e%d.npy" % ci)
            np.save(ein, e)
            for k, env in enumerate(envs):
                out = os.path.join(td, "o%d_%d.npy" % (ci, k))
                r = subprocess.run([sys.executable, "-u", "-c", code, ein, out, str(V), str(M)],
                                   env=dict(os.environ, **env), capture_output=True, text=True, timeout=300)
                assert r.returncode == 0, (env, r.stderr[-1500:])
                assert np.array_equal(np.load(out), want), (V, env)
                print("V", V, "candidate", env, "exact", flush=True)
