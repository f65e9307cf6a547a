"""Benchmark of the bridge path on one MI355X.

One step = one br_bridges_find call: per-chunk certificates (phase 0), the
merge rounds, the bridges of the merged certificate (the library's default
bridge step on the GPU), the copy of the bridges to the host and the
canonical sort -- every step of the path, on input already resident in HBM.
The same steps with Algorithm 1's depth-first search on the host as the final
step are reported under "detail".  Prints one JSON line (rank 0, N = 1).

Default workload: the large configuration (V = 267,144 as 1,024 complete
clusters of 256 vertices, 996,147,200 uniform inter-cluster edges, cluster
tree, 5,000 pendant vertices; E = 1,029,576,583, 8.2 GB of int32 pairs) at
M = 4096 chunks -- the largest configuration that fits one GPU; a sweep over
M and the dense configuration (V = 66,536, E = 4,178,013, M = 16) are
reported under "detail".  "achievable" is the read bandwidth a plain
16-byte-load stream over the same edge list reaches on this device.

Before timing, the library's tuner measures the certificate plans for the
workload's shape and keeps the fastest (outside the timed region; every plan
gives the same bridges).

Roofline: the dominant kernel is the certificate kernel that streams the edge
list -- phase 0 of the plan that ran (for the one-workgroup-per-node plan,
k_solo, which also runs the lower merge levels); its algorithmic traffic is
counted as 8 bytes per input edge (one read of the int32 pair; the
certificates it writes and re-reads are left out, so the fraction is a lower
bound), divided by its duration from HIP events recorded on the call's stream
during the timed steps, against the 8 TB/s HBM3E peak.  "traffic" is the
counter-measured HBM bytes per launch from the committed rocprofv3 summary,
when that summary was taken from the current kernel source (else null).
"method_bytes_at_M" is the method's own traffic at the configured M -- the
edge list read once, every certificate edge written to its node's region and
read once more by its merge, from the library's per-node counts -- over the
timed certificate phases (phase 0 and every merge).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0
# certificate plans the library reports (br_profile.plan_kind) and the unit
# the roofline line times for each: the launches from the first certificate
# kernel to the end of phase 0 (of the merge levels inside the kernel, for the
# one-workgroup-per-node plan)
PLAN_NAMES = {0: "many workgroups per chunk", 1: "one workgroup per node", 2: "whole tree in LDS"}
UNIT_NAMES = {0: "phase 0 per query (k_phase0 stages and the compressions between them)",
              1: "k_solo per query (phase 0 and the merge levels it runs, one workgroup per node)",
              2: "k_batched per query (phase 0 and every merge, in LDS)"}
CSRC = os.path.join(ROOT, "paper_2108_07346_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def load_traffic(workload, M, plan_kind=0):
    """Counter-measured HBM bytes per launch of the dominant kernel, from the
    committed rocprofv3 summary -- only if it was taken for the same plan and
    the kernel source is unchanged since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    rec = t.get("%s_M%d" % (workload, M))
    if not rec or rec.get("plan_kind", 0) != plan_kind:
        return None
    try:
        sha = hashlib.sha256(open(os.path.join(CSRC, rec["kernel_file"]), "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return rec.get("bytes_per_launch") if sha == rec.get("kernel_sha") else None


def host_info():
    """The host the CPU numbers come from: CPU model and core counts."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu": model, "nproc": os.cpu_count(), "usable_cores": usable}


def achievable_read(d, stream, reps=5):
    """Read bandwidth of one pass of br_probe_read (16-byte loads) over the
    edge list, timed with events on the launch stream (GB/s)."""
    import torch
    import paper_2108_07346_amd as br
    for _ in range(2):
        br.probe_read(d, stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        br.probe_read(d, stream)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    return d.numel() * d.element_size() / (ms / 1000) / 1e9


def cpu_baseline(g, budget_s):
    """The oracle as it stands, single-threaded, on the host."""
    import oracle
    import numpy as np
    if g.E > 60_000_000:      # bounded sample: a prefix of the shuffled list
        n = 60_000_000
        e = np.ascontiguousarray(g.edges[:n])
        sample = "first %d edges of the shuffled list (uniform sample), full V" % n
    else:
        e = g.edges
        sample = "whole workload"
    oracle.bridges(e[:1000], g.V)          # load
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.bridges(e, g.V)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or (dt > 0 and reps >= 50):
            break
    h = host_info()
    return {"value": e.shape[0] * reps / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "%s, %d repetition(s) in %.1f s, one thread of %s (nproc %d)" %
                      (sample, reps, dt, h["cpu"], h["nproc"]),
            "host": h}


def bench_batched(args):
    """Batched workload: one br_bridges_find_batched call per step, against the
    plain path called once per graph on the same GPU."""
    import numpy as np
    import torch
    import graphgen
    import paper_2108_07346_amd as br
    t0 = time.perf_counter()
    b = graphgen.batched(0, n_graphs=args.graphs)
    E = int(b.edges.shape[0])
    d = torch.from_numpy(b.edges).cuda()
    torch.cuda.synchronize()
    print("bench: batched %d graphs, E=%d (generated in %.1f s)" % (b.G, E, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    ctx = br.Context(0)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):          # the first call tunes chunk_edges when --chunk 0
        ctx.find_batched(d, b.offsets, b.V, args.chunk, stream)
    ctx.set_profiling(True)
    acc = {"ms_phase0": 0.0, "ms_cert": 0.0, "ms_dfs": 0.0, "ms_canon": 0.0}
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        pairs, boff = ctx.find_batched(d, b.offsets, b.V, args.chunk, stream)
        p = ctx.profile()
        for k in acc:
            acc[k] += p[k]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    chunk = int(ctx.profile()["rounds"])
    phases = {k: v / args.steps for k, v in acc.items()}
    ms_step = 1000 * dt / args.steps
    # the same batch with Algorithm 1's search per graph on the host instead of
    # the default bridge step on the GPU (one launch sequence over all certificates)
    ctx.set_final_step(0)
    ctx.set_profiling(True)
    ctx.find_batched(d, b.offsets, b.V, args.chunk, stream)
    acch = {"ms_phase0": 0.0, "ms_cert": 0.0, "ms_dfs": 0.0}
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(args.steps):
        ph_, bh_ = ctx.find_batched(d, b.offsets, b.V, args.chunk, stream)
        p = ctx.profile()
        for k in acch:
            acch[k] += p[k]
    torch.cuda.synchronize()
    dth = time.perf_counter() - th
    ctx.set_final_step(1)
    assert np.array_equal(ph_, pairs) and np.array_equal(bh_, boff)
    host_search = {"edges_per_s": E * args.steps / dth, "ms_per_step": 1000 * dth / args.steps,
                   "ms_host_search": round(acch["ms_dfs"] / args.steps, 4)}
    print("bench: batched, host search %s" % json.dumps(host_search), file=sys.stderr, flush=True)
    # baseline: the plain path, one call (certificate kernels + bridge step) per graph
    ctx.set_profiling(False)
    views = [d[b.offsets[g]:b.offsets[g + 1]] for g in range(b.G)]
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for g in range(b.G):
        ctx.find(views[g], int(b.V[g]), 1, stream)
    torch.cuda.synchronize()
    t_base = time.perf_counter() - tb
    t_k = phases["ms_phase0"] / 1000
    achieved = 8.0 * E / t_k / 1e9 if t_k > 0 else 0.0
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        reps, tc = 0, time.perf_counter()
        ng = 0
        while time.perf_counter() - tc < args.cpu_budget and ng < b.G:
            oracle.bridges(b.graph(ng), int(b.V[ng]))
            reps += int(b.offsets[ng + 1] - b.offsets[ng])
            ng += 1
        dtc = time.perf_counter() - tc
        cpu = {"value": reps / dtc, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "first %d of %d graphs (%d edges) in %.1f s, one host core" % (ng, b.G, reps, dtc)}
    line = {
        "metric": "edges/sec certified+bridged at 1 GPU (% HBM roofline)",
        "value": E * args.steps / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic (seeded planted-cluster generator)",
        "config": {"workload": "batched", "graphs": b.G, "E": E, "chunk_edges": chunk, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_GBS, "traffic": load_traffic("batched", 0),
                     "kernel": "k_batched (persistent, all graphs)", "algorithmic_bytes_per_launch": 8 * E},
        "cpu_baseline": cpu,
        "detail": {"phases_ms": {k: round(v, 4) for k, v in phases.items()},
                   "one_call_per_graph": {"ms": 1000 * t_base, "edges_per_s": E / t_base,
                                          "speedup_of_batched": t_base / (dt / args.steps)},
                   "host_search": host_search,
                   "bridges": int(boff[-1])},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_figures(args):
    """The paper's figure experiments (Figs. 2-4) as synthetic sweeps: the
    whole path per point, both final steps, with the paper's complexity
    O(E/M + V log M) printed beside each point (no numbers exist in the paper)."""
    import numpy as np
    import torch
    import graphgen
    import paper_2108_07346_amd as br
    ctx = br.Context(0)
    stream = torch.cuda.current_stream()
    out = {}
    for fig, points in graphgen.FIGURES.items():
        rows = []
        cache = {}
        for V, E, M in points:
            if (V, E) not in cache:
                cache.clear()
                g = graphgen.figure(V, E)
                cache[(V, E)] = (g, torch.from_numpy(g.edges).cuda())
            g, d = cache[(V, E)]
            row = {"V": g.V, "E": g.E, "M": M, "model_E_over_M_plus_V_log2M": g.E / M + g.V * np.log2(max(M, 2))}
            for mode in (0, 1):
                ctx.set_final_step(mode)
                ctx.set_profiling(False)
                for _ in range(2):
                    ctx.find(d, g.V, M, stream)
                ctx.set_profiling(True)
                reps = 5
                acc = 0.0
                ph = {"ms_phase0": 0.0, "ms_merge": 0.0}
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(reps):
                    ctx.find(d, g.V, M, stream)
                    p = ctx.profile()
                    for k in ph:
                        ph[k] += p[k] / reps
                torch.cuda.synchronize()
                ms = 1000 * (time.perf_counter() - t) / reps
                row["ms_host_search" if mode == 0 else "ms_gpu_final_step"] = round(ms, 4)
                row.update({k: round(v, 4) for k, v in ph.items()})
            ctx.set_final_step(1)
            rows.append(row)
            print("bench: %s %s" % (fig, json.dumps(row)), file=sys.stderr, flush=True)
        out[fig] = rows
    line = {"metric": "paper figures 2-4 as synthetic sweeps (ms per bridge query)", "value": None, "unit": "ms",
            "n_gpus": 1, "steps": 5, "warmup": 2, "ms_per_step": None, "higher_is_better": False,
            "scaling": "strong", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic (seeded planted-cluster generator)", "config": {"workload": "figures"},
            "roofline": None, "cpu_baseline": None, "detail": out}
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_articulation(args):
    """Articulation points of the dense workload: the scan-first certificate and
    the cut-vertex test on it, both on the GPU (the default final step); the
    host low-link search over the copied certificate (final step 0) timed as a
    detail; the oracle (the low-link search on the whole graph) beside it."""
    import numpy as np
    import torch
    import graphgen
    import paper_2108_07346_amd as br
    g = graphgen.config("dense")
    d = torch.from_numpy(g.edges).cuda()
    ctx = br.Context(0)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        out = ctx.articulation_points(d, g.V, stream)
    acc = {"ms_cert": 0.0, "ms_dfs": 0.0}
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.articulation_points(d, g.V, stream)
        p = ctx.profile()
        for k in acc:
            acc[k] += p[k] / args.steps
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # detail: the host low-link search as the final step
    ctx.set_final_step(0)
    out0 = ctx.articulation_points(d, g.V, stream)
    nh = max(1, min(args.steps, 5))
    th = time.perf_counter()
    for _ in range(nh):
        out0 = ctx.articulation_points(d, g.V, stream)
    ms_host = 1000 * (time.perf_counter() - th) / nh
    ctx.set_final_step(1)
    assert np.array_equal(out0, out)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        reps, tc = 0, time.perf_counter()
        while True:
            want = oracle.articulation_points(g.edges, g.V)
            reps += 1
            if time.perf_counter() - tc >= min(args.cpu_budget, 10.0):
                break
        dtc = time.perf_counter() - tc
        assert np.array_equal(want, out)
        cpu = {"value": g.E * reps / dtc, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "whole dense workload, %d repetition(s) in %.1f s, one host core" % (reps, dtc)}
    line = {"metric": "articulation points: edges/s (scan-first certificate and cut-vertex test on the GPU)",
            "value": g.E * args.steps / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1000 * dt / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "int32", "data": "synthetic (seeded planted-cluster generator)",
            "config": {"workload": "dense", "V": g.V, "E": g.E, "parallelism": "single GPU"},
            "roofline": None, "cpu_baseline": cpu,
            "detail": {"phases_ms": {k: round(v, 4) for k, v in acc.items()}, "articulation_points": int(out.shape[0]),
                       "certificate_edges": int(p["cert_f1"] + p["cert_f2"]), "bfs_levels": int(p["rounds"]),
                       "ms_per_step_host_search": round(ms_host, 4)}}
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_classes(args):
    """2-edge-connected classes of the dense workload (labels = smallest vertex
    of each class): the certificate, the bridge test and the union of the
    non-bridge certificate edges, all on the GPU (the default final step); the
    oracle (its own low-link search and union on the whole graph) timed beside
    it."""
    import numpy as np
    import torch
    import graphgen
    import paper_2108_07346_amd as br
    g = graphgen.config("dense")
    M = args.M or 16
    d = torch.from_numpy(g.edges).cuda()
    ctx = br.Context(0)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        lab, n = ctx.two_edge_components(d, g.V, M, stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        lab, n = ctx.two_edge_components(d, g.V, M, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        reps, tc = 0, time.perf_counter()
        while True:
            want = oracle.two_edge_labels(g.edges, g.V)
            reps += 1
            if time.perf_counter() - tc >= min(args.cpu_budget, 10.0):
                break
        dtc = time.perf_counter() - tc
        assert np.array_equal(want, lab)
        cpu = {"value": g.E * reps / dtc, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "whole dense workload, %d repetition(s) in %.1f s, one host core" % (reps, dtc)}
    line = {"metric": "2-edge-connected classes: edges/s (certificate, bridges and class union on the GPU)",
            "value": g.E * args.steps / dt, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1000 * dt / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "int32", "data": "synthetic (seeded planted-cluster generator)",
            "config": {"workload": "dense", "V": g.V, "E": g.E, "M": M, "parallelism": "single GPU"},
            "roofline": None, "cpu_baseline": cpu, "detail": {"classes": int(n)}}
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_served(args):
    """Served workload: open-loop Poisson arrivals at fixed QPS; latency from
    each request's scheduled arrival to the moment its answer is back on the
    host.  Three servers over the same arrival sequence: the batch lane (the
    requests within the LDS kernels' limit certified together, one batched
    call per tick; the rest on slots), slots only (every request runs the
    plain path on one of the slots, concurrently), and one slot (the plain
    per-request path, serialised)."""
    import threading
    import numpy as np
    import torch
    import graphgen
    import paper_2108_07346_amd as br
    t0 = time.perf_counter()
    if args.mix == "small":
        # requests drawn like the batched workload's graphs (V 64..4096)
        pool = [graphgen.planted(**graphgen.batched_params(1, r)) for r in range(args.pool)]
    else:
        pool = [graphgen.served_request(0, r) for r in range(args.pool)]
    Es = np.array([g.E for g in pool])
    print("bench: %s pool of %d requests, mean E %.3g, max E %d (generated in %.1f s)" %
          (args.mix, len(pool), Es.mean(), Es.max(), time.perf_counter() - t0), file=sys.stderr, flush=True)
    dev = [torch.from_numpy(g.edges).cuda() for g in pool] if args.resident else None
    torch.cuda.synchronize()
    results = {}
    qps = args.qps or ("100,200,500,1000,2000,5000" if args.mix == "served" else "1000,5000,20000,50000")
    qps_list = [float(x) for x in qps.split(",")]
    servers = (("batch_lane", args.slots, True), ("slots_only", args.slots, False), ("per_request", 1, False))

    def run(qps, slots, lane, resident, seed):
        srv = br.Server(0, mem_budget=64 << 30, max_slots=slots)
        srv.set_final_step(args.final_step)
        if not lane:
            srv.set_batching(0)
        else:
            srv.set_batching(args.lane_max_v or br.lds_max_v(), args.lane_max_e)
        rng = np.random.default_rng(seed)          # the same arrivals for every server
        n = args.requests
        sched = np.cumsum(rng.exponential(1.0 / qps, size=n))
        pick = rng.integers(0, len(pool), size=n)
        tickets = [None] * n
        done_t = [0.0] * n
        ready = threading.Semaphore(0)

        def collector():
            for i in range(n):
                ready.acquire()
                srv.wait(tickets[i], pool[pick[i]].V)
                done_t[i] = time.perf_counter()

        th = threading.Thread(target=collector)
        th.start()
        start = time.perf_counter() + 0.05
        for i in range(n):
            while True:
                now = time.perf_counter()
                if now >= start + sched[i]:
                    break
                time.sleep(min(0.0005, start + sched[i] - now))
            g = pool[pick[i]]
            tickets[i] = srv.submit(dev[pick[i]] if resident else g.edges, g.V)
            ready.release()
        th.join()
        end = max(done_t)
        st = srv.stats()
        srv.close()
        lat = np.array([done_t[i] - (start + sched[i]) for i in range(n)]) * 1000
        edges = int(sum(pool[pick[i]].E for i in range(n)))
        return {"requests": n, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "achieved_qps": n / (end - start), "edges_per_s": edges / (end - start),
                "batched_ticks": int(st["batched_ticks"]), "batched_requests": int(st["batched_requests"]),
                "peak_inflight": int(st["peak_inflight"])}

    mode = "resident" if args.resident else "host"
    for k, qps in enumerate(qps_list):
        for name, slots, lane in servers:
            key = "%s_%s_qps%d" % (mode, name, qps)
            results[key] = run(qps, slots, lane, args.resident, seed=k)
            print("bench: %s %s" % (key, json.dumps(results[key])), file=sys.stderr, flush=True)
    head = results["%s_batch_lane_qps%d" % (mode, qps_list[0])]
    line = {
        "metric": "served p50/p99 latency (ms) and edges/s at fixed QPS, 1 GPU",
        "value": head["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": head["requests"], "warmup": 0,
        "ms_per_step": head["p50_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic (seeded planted-cluster generator)",
        "config": {"workload": "served" if args.mix == "served" else "served_small", "pool": len(pool),
                   "slots": args.slots, "qps": qps_list,
                   "requests_per_point": args.requests, "edges": mode,
                   "lane_limits": [args.lane_max_v or None, args.lane_max_e],
                   "final_step": "gpu" if args.final_step else "host search",
                   "parallelism": "single GPU"},
        "roofline": None, "cpu_baseline": None, "detail": results,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["small", "dense", "large", "large_blocked", "batched", "served",
                                                            "figures", "articulation", "classes"])
    ap.add_argument("--qps", default=None, help="served: comma-separated QPS (default by mix)")
    ap.add_argument("--mix", default="served", choices=["served", "small"],
                    help="served: request sizes of the served workload, or small graphs like the batched workload's")
    ap.add_argument("--requests", type=int, default=2000, help="served: requests per QPS point and server")
    ap.add_argument("--pool", type=int, default=32, help="served: distinct requests generated")
    ap.add_argument("--lane-max-v", type=int, default=0, help="served: batch lane V limit (0: the LDS kernels' limit)")
    ap.add_argument("--lane-max-e", type=int, default=1 << 21, help="served: batch lane edge limit")
    ap.add_argument("--slots", type=int, default=8, help="served: device slots")
    ap.add_argument("--resident", action="store_true", help="served: submit edge lists already on the GPU")
    ap.add_argument("--final-step", type=int, default=1, help="served: 1 bridge step on the GPU (default), 0 host search")
    ap.add_argument("--graphs", type=int, default=4096, help="batched: number of graphs")
    ap.add_argument("--chunk", type=int, default=0, help="batched: chunk_edges (0 = tuned)")
    ap.add_argument("--M", type=int, default=None)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="plain workloads: skip the tuner (size rules only)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, help="run a plain device copy of this many MiB")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the path runs on one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import graphgen
    import paper_2108_07346_amd as br

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n}), flush=True)
        return

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "figures":
        return bench_figures(args)
    if args.workload == "articulation":
        return bench_articulation(args)
    if args.workload == "classes":
        return bench_classes(args)
    M = args.M or {"small": 4, "dense": 16, "large": 4096, "large_blocked": 4096}[args.workload]
    t0 = time.perf_counter()
    g = graphgen.config(args.workload)
    t_gen = time.perf_counter() - t0
    d = torch.from_numpy(g.edges).cuda()
    torch.cuda.synchronize()
    print("bench: workload %s V=%d E=%d M=%d (generated in %.1f s)" % (args.workload, g.V, g.E, M, t_gen),
          file=sys.stderr, flush=True)

    ctx = br.Context(0)
    stream = torch.cuda.current_stream()

    def run_steps(Mx, n, prof):
        ctx.set_profiling(prof)
        acc = {"ms_phase0": 0.0, "ms_merge": 0.0, "ms_cert": 0.0, "ms_d2h": 0.0, "ms_dfs": 0.0, "ms_canon": 0.0,
               "ms_bridge_dev": 0.0}
        out = None
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            out = ctx.find(d, g.V, Mx, stream)
            if prof:
                p = ctx.profile()
                for k in acc:
                    acc[k] += p[k]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        return dt, {k: v / max(n, 1) for k, v in acc.items()}, out

    tuned = None
    if not args.no_tune:
        # the library's tuner picks the certificate plan for this shape (kept
        # in BR_AUTOTUNE_CACHE when set); outside the timed region
        t0 = time.perf_counter()
        tuned = ctx.autotune(d, g.V, M, stream)
        print("bench: tuner %s (%.1f s)" % (json.dumps(tuned), time.perf_counter() - t0), file=sys.stderr, flush=True)
    run_steps(M, args.warmup, False)
    dt, phases, out = run_steps(M, args.steps, True)
    prof = ctx.profile()
    plan_kind = int(prof["plan_kind"])
    ms_step = 1000.0 * dt / args.steps
    value = g.E * args.steps / dt
    t_k = phases["ms_phase0"] / 1000.0
    achieved = 8.0 * g.E / t_k / 1e9 if t_k > 0 else 0.0
    traffic = load_traffic(args.workload, M, plan_kind)
    print("bench: %d steps, %.3f ms/step, %.3e edges/s, phases %s, bridges %d" %
          (args.steps, ms_step, value, json.dumps({k: round(v, 4) for k, v in phases.items()}), out.shape[0]),
          file=sys.stderr, flush=True)

    # the method's own bytes at this M (edge list, certificates written and
    # read by the merges), over the timed certificate phases
    ctx.set_profiling(2)
    ctx.find(d, g.V, M, stream)
    alg_m = int(ctx.profile()["alg_bytes"])
    ctx.set_profiling(1)
    method_at_m = None
    if alg_m > 0 and phases["ms_cert"] > 0:
        gbs = alg_m / (phases["ms_cert"] / 1000) / 1e9
        method_at_m = {"bytes": alg_m, "ms_cert": round(phases["ms_cert"], 4), "GBs": gbs, "frac": gbs / PEAK_GBS}
    detail = {"phases_ms": {k: round(v, 5) for k, v in phases.items()}, "bridges": int(out.shape[0]),
              "certificate_edges": int(prof["cert_f1"] + prof["cert_f2"]), "merge_rounds": int(prof["rounds"]),
              "plan": PLAN_NAMES[plan_kind], "tuner": tuned,
              "complexity_claim": "O(E/M + V log M) on M machines (paper, Section V)"}
    # the same step with Algorithm 1's depth-first search on the host (after
    # copying the certificate) instead of the default bridge step on the GPU
    ctx.set_final_step(0)
    run_steps(M, 2, False)
    hdt, hph, hout = run_steps(M, args.steps, True)
    ctx.set_final_step(1)
    assert hout.shape == out.shape and (hout == out).all()
    detail["host_search"] = {"edges_per_s": g.E * args.steps / hdt, "ms_per_step": 1000 * hdt / args.steps,
                             "ms_d2h": round(hph["ms_d2h"], 5), "ms_dfs": round(hph["ms_dfs"], 5)}
    print("bench: host search %s" % json.dumps(detail["host_search"]), file=sys.stderr, flush=True)
    sweep_ms = {"dense": (1, 16, 256, 1024), "large": (64, 256, 1024, 4096)}.get(args.workload)
    achievable = achievable_read(d, stream)
    print("bench: read stream over the edge list %.0f GB/s" % achievable, file=sys.stderr, flush=True)
    if sweep_ms and not args.no_sweep:
        sweep = {}
        reps = 10 if args.workload == "dense" else 2
        for Mx in sweep_ms:
            tuned_x = ctx.autotune(d, g.V, Mx, stream) if not args.no_tune else None   # each M its own plan
            run_steps(Mx, 1, False)
            sdt, sph, _ = run_steps(Mx, reps, True)
            sweep[str(Mx)] = {"edges_per_s": g.E * reps / sdt, "ms_per_step": 1000 * sdt / reps,
                              "plan": PLAN_NAMES[int(ctx.profile()["plan_kind"])],
                              "tuner": {k: v for k, v in (tuned_x or {}).items() if k not in ("key", "source")},
                              "ms_phase0": round(sph["ms_phase0"], 5), "ms_merge": round(sph["ms_merge"], 5),
                              "ms_bridge_step": round(sph["ms_bridge_dev"], 5),
                              "phase0_frac_hbm": (8.0 * g.E / (sph["ms_phase0"] / 1000) / 1e9) / PEAK_GBS
                              if sph["ms_phase0"] > 0 else None}
            print("bench: sweep M=%d %s" % (Mx, json.dumps(sweep[str(Mx)])), file=sys.stderr, flush=True)
        detail["m_sweep"] = sweep

    if args.workload == "large" and not args.no_sweep:
        # the dense configuration beside it (M = 16), whole query
        gd = graphgen.config("dense")
        dd = torch.from_numpy(gd.edges).cuda()
        if not args.no_tune:
            ctx.autotune(dd, gd.V, 16, stream)
        for _ in range(3):
            ctx.find(dd, gd.V, 16, stream)
        ctx.set_profiling(True)
        accd = {"ms_phase0": 0.0, "ms_merge": 0.0, "ms_bridge_dev": 0.0}
        torch.cuda.synchronize()
        td = time.perf_counter()
        for _ in range(20):
            ctx.find(dd, gd.V, 16, stream)
            p = ctx.profile()
            for k in accd:
                accd[k] += p[k] / 20
        torch.cuda.synchronize()
        dtd = (time.perf_counter() - td) / 20
        detail["dense_M16"] = {"V": gd.V, "E": gd.E, "edges_per_s": gd.E / dtd, "ms_per_step": 1000 * dtd,
                               **{k: round(v, 5) for k, v in accd.items()},
                               "phase0_frac_hbm": 8.0 * gd.E / (accd["ms_phase0"] / 1000) / 1e9 / PEAK_GBS}
        print("bench: dense M=16 %s" % json.dumps(detail["dense_M16"]), file=sys.stderr, flush=True)
        del dd

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, args.cpu_budget)
        print("bench: cpu baseline %s" % json.dumps(cpu), file=sys.stderr, flush=True)

    line = {
        "metric": "edges/sec certified+bridged at 1 GPU (% HBM roofline)",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded planted-cluster generator)",
        "config": {"workload": args.workload, "V": g.V, "E": g.E, "M": M, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_GBS, "traffic": traffic,
                     "kernel": UNIT_NAMES[plan_kind],
                     "algorithmic_bytes_per_launch": 8 * g.E,
                     "achievable_read_GBs": achievable,
                     "method_bytes_at_M": method_at_m},
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
