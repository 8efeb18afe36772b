#!/usr/bin/env python3
"""Benchmark of the CentRA hot path on one MI355X.

Workload (default, the large sparse configuration): undirected
Barabasi-Albert graph n = 1,000,000, attachment 5 (seed 1), uint32 CSR
resident in HBM; Algorithm 1 with a schedule starting at 100,000 samples and
doubling up to 4,000,000, k = 50, t = 64, eps = 0.01, delta = 0.1.  One step
= one complete run of Algorithm 1 from an empty sample (sampling, greedy
cover, AMCERA and bound at every iteration) until the stopping condition
holds or the cap is reached.  value = shortest paths sampled per second of
whole-job time.

Other workloads (`--workload`):
  skewed     the skewed directed configuration: R-MAT scale 22 (edge factor
             16, a/b/c/d = .57/.19/.19/.05, seed 1, duplicates and self loops
             dropped) with its reverse CSR; 2,000,000 samples doubling to
             8,000,000, k = 100, t = 128, eps = 0.01, delta = 0.1;
  small      the small configuration: Barabasi-Albert n = 2,000, attachment
             5; one iteration at 10,000 samples, k = 10, t = 10,
             eps = 0.05, delta = 0.1;
  triangles  Algorithm 1 on the triangle hyperedge space (the triangle
             centrality) of the R-MAT scale 20 graph above, symmetrised
             (1,048,576 nodes, 31.4M arcs, 424M triangles); 1,000,000
             samples doubling to 8,000,000, k = 50, t = 64, eps = 0.01,
             delta = 0.1; the per-graph triangle index is built once before
             the timed steps and its time is reported as index_s;
  kpaths     Algorithm 1 on the kappa-path hyperedge space (the kappa-path
             centrality; random simple walks of length at most kappa = 5) of
             the Barabasi-Albert n = 1,000,000 graph above; 1,000,000
             samples doubling to 8,000,000, k = 50, t = 64, eps = 0.05,
             delta = 0.1 (the top-50 cover about 2% of the walks, so
             eps = 0.01 would not certify below 64M samples).

Also reported:
  - roofline: the sampling kernel's algorithmic bytes per launch over its
    average launch time, measured with HIP events recorded on the launch
    stream around every launch in the timed region.  Shortest paths: 4 B
    per CSR entry scanned + 28 B per node given a level, counted exactly by
    the kernel.  Triangles: 56 B per sample (20 B written; the bracketing
    prefix pair, the arc's source and target, its list offset and the
    listed node read).  kappa-paths: the walk pass reads 12 B per step (the
    row bounds and the chosen entry) and stages the node (4 B), the gather
    reads and writes it (8 B): 24 B per walk node, plus 12 B per walk (its
    length written, its offset read).  `traffic` comes from
    the committed rocprofv3
    counter summary when it was taken on the current kernel source, else
    null;
  - cpu_baseline: the oracle (plain C, single thread) on a bounded sample
    of the same workload on this host: the first sample indices for a
    fixed time (shortest paths), or its triangle enumeration over seeded
    uniformly drawn rows, extrapolated to all rows (triangles);
    cpu_baseline_all_cores: the same path sampling split over the host's
    cores (at most 16 threads), results unchanged by construction.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SAMPLER_SRC = os.path.join(ROOT, "paper_2306_03651_amd", "csrc", "sample.hip")

WORKLOADS = {
    "sparse": dict(graph="barabasi_albert", n=1_000_000, m0=5, graph_seed=1, seed=1, instance=0,
                   m_init=100_000, m_max=4_000_000, growth=2, k=50, t=64, eps=0.01, delta=0.1,
                   traffic="sample_paths_ba1e6_traffic.txt",
                   label="CentRA (Algorithm 1) on Barabasi-Albert n=1e6, attachment 5, seed 1; samples 100k "
                         "doubling to 4M, k=50, t=64, eps=0.01, delta=0.1"),
    "skewed": dict(graph="rmat", scale=22, edge_factor=16, graph_seed=1, seed=1, instance=0,
                   m_init=2_000_000, m_max=8_000_000, growth=2, k=100, t=128, eps=0.01, delta=0.1,
                   traffic="sample_paths_rmat22_traffic.txt",
                   label="CentRA (Algorithm 1) on R-MAT scale 22 (edge factor 16, .57/.19/.19/.05, seed 1, "
                         "directed); samples 2M doubling to 8M, k=100, t=128, eps=0.01, delta=0.1"),
    "small": dict(graph="barabasi_albert", n=2000, m0=5, graph_seed=1, seed=1, instance=0,
                  m_init=10_000, m_max=10_000, growth=2, k=10, t=10, eps=0.05, delta=0.1, traffic=None,
                  label="CentRA (Algorithm 1) on Barabasi-Albert n=2,000, attachment 5, seed 1; one iteration at "
                        "10,000 samples, k=10, t=10, eps=0.05, delta=0.1"),
    "kpaths": dict(graph="barabasi_albert", n=1_000_000, m0=5, graph_seed=1, seed=1, instance=0,
                   m_init=1_000_000, m_max=8_000_000, growth=2, k=50, t=64, eps=0.05, delta=0.1,
                   space="kpaths", kappa=5, traffic="sample_kpaths_ba1e6_traffic.txt",
                   label="CentRA (Algorithm 1) on the kappa-path hyperedge space (kappa=5) of Barabasi-Albert "
                         "n=1e6, attachment 5, seed 1; samples 1M doubling to 8M, k=50, t=64, eps=0.05, "
                         "delta=0.1"),
    "triangles": dict(graph="rmat_undirected", scale=20, edge_factor=16, graph_seed=1, seed=1, instance=0,
                      m_init=1_000_000, m_max=8_000_000, growth=2, k=50, t=64, eps=0.01, delta=0.1,
                      space="triangles", traffic="sample_triangles_rmat20u_traffic.txt",
                      label="CentRA (Algorithm 1) on the triangle hyperedge space of R-MAT scale 20 (edge factor "
                            "16, .57/.19/.19/.05, seed 1, symmetrised); samples 1M doubling to 8M, k=50, t=64, "
                            "eps=0.01, delta=0.1"),
}
# Workloads of the batching and serving engine (one JSON line each, not the
# default benchmark line).
ENGINE_WORKLOADS = {
    "batched": dict(count=256, mix_seed=1, ba_n=(1_000, 100_000), grid_side=(32, 128), k=(5, 50), t=32,
                    m_init=50_000, m_max=50_000, eps=0.05, delta=0.1, seed=1,
                    label="uneven instances: 256 graphs, each Barabasi-Albert n~U[1e3,1e5] (attachment 5) or an L x L "
                          "grid L~U[32,128] (Bernoulli 1/2, numpy seed 1), 50k shortest-path samples each, "
                          "k~U[5,50], t=32, eps=0.05, delta=0.1 (one iteration of Algorithm 1 per instance)"),
    "serving": dict(rate=200.0, duration=2.0, arrival_seed=1, t=100, delta=0.1, eps=(0.05, 0.02, 0.01), k=(10, 500),
                    seed=1,
                    label="serving: 8 resident graphs (4 Barabasi-Albert n=1e6, 2 R-MAT scale 20 directed, 2 grids "
                          "2048x2048); Poisson arrivals at 200 queries/s for 2 s, each (graph~U{0..7}, k~U[10,500], "
                          "eps~U{0.05,0.02,0.01}, delta=0.1, t=100); pools 100k doubling to 6.4M samples "
                          "(grids: 1k doubling to 16k), drawn and built before the stream starts"),
}
TRIANGLE_SAMPLE_BYTES = 56
KPATH_NODE_BYTES, KPATH_SAMPLE_BYTES = 24, 12
WORKLOAD = WORKLOADS["sparse"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(src: str = SAMPLER_SRC) -> str:
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def read_traffic(name=WORKLOAD["traffic"]):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current source of its kernel (sample.hip unless the summary
    names another)."""
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip()
    if "kernel_source" in vals:
        src = os.path.join(ROOT, "paper_2306_03651_amd", "csrc", os.path.basename(vals["kernel_source"]))
        if not os.path.exists(src) or vals.get("kernel_source_sha256_16") != kernel_source_hash(src):
            return None
    elif vals.get("sampler_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_desc():
    return f"host {platform.processor() or platform.machine()}, {os.cpu_count()} logical CPUs"


def oracle_sampler(graph, W):
    """(draw(first, count), batch, unit, description) of the oracle's sampler
    for W's space; kappa-path walks are drawn by the oracle's own batch loop
    (a walk takes about a microsecond, less than a Python call)."""
    import oracle
    og = oracle.OracleGraph(graph)
    if W.get("space") == "kpaths":
        kappa = W["kappa"]
        lib = oracle._load()

        def draw(first, count):
            import numpy as np
            off = np.zeros(count + 1, dtype=np.uint64)
            nodes = np.zeros(count * kappa, dtype=np.uint32)
            lib.orc_sample_kpaths(ctypes.byref(og.c), kappa, W["seed"], W["instance"], first, count, off, nodes)
        return (draw, 20000, "walks/s",
                f"the oracle's kappa-path sampler (random simple walk, kappa={kappa}, rows scanned per step)")
    c_bits = oracle._load().orc_count_bits(ctypes.byref(og.c))
    return ((lambda first, count: oracle.sample_path(graph, W["seed"], W["instance"], first, c_bits=c_bits, og=og)),
            1, "paths/s", "the oracle's sampler (full-level BFS with normalised counts + backtrack)")


def cpu_baseline(graph, seconds: float, W):
    draw, batch, unit, what = oracle_sampler(graph, W)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        draw(done, batch)
        done += batch
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": unit, "cores": 1, "kind": "oracle",
            "sample": f"sample indices 0..{done - 1} of the benchmark workload (seed 1, instance 0) drawn by "
                      f"{what}, one thread, {dt:.1f} s; greedy cover and AMCERA excluded; {host_desc()}"}


def cpu_baseline_all_cores(graph, seconds: float, W):
    """The oracle's sampler with the independent per-sample loop split over
    threads (the C calls release the GIL); each thread draws the indices
    congruent to its number modulo the thread count."""
    from concurrent.futures import ThreadPoolExecutor
    draw, batch, unit, what = oracle_sampler(graph, W)
    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()

    def work(j):
        done = 0   # batches of this thread: thread j draws batches j, j + threads, ...
        while time.perf_counter() - t0 < seconds:
            draw((j + threads * done) * batch, batch)
            done += 1
        return done * batch

    with ThreadPoolExecutor(threads) as ex:
        counts = list(ex.map(work, range(threads)))
    dt = time.perf_counter() - t0
    return {"value": sum(counts) / dt, "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"{sum(counts)} sample indices (thread j draws batch j, j + {threads}, ... of {batch}) of the benchmark "
                      f"workload drawn by {what} on {threads} threads for {dt:.1f} s; {host_desc()}"}


def cpu_baseline_triangles(graph, seconds: float, m_final: int):
    """The oracle's triangle space: its cost is the enumeration of every
    triangle (the draws after it are a table lookup each).  Rows a (the
    smallest node of their triangles) are drawn uniformly with a fixed seed
    and enumerated for a bounded time; n times the mean time per row
    estimates the enumeration of all rows."""
    import numpy as np
    import oracle
    og = oracle.OracleGraph(graph)
    rng = np.random.default_rng(1)
    rows = 0
    found = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        found += oracle.row_triangle_count(graph, int(rng.integers(graph.n)), og=og)
        rows += 1
    dt = time.perf_counter() - t0
    est = dt / rows * graph.n
    return {"value": m_final / est, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"the oracle's triangle enumeration on {rows} uniformly drawn rows (seed 1; {found} "
                      f"triangles) in {dt:.1f} s, one thread, extrapolated to all {graph.n} rows: {est:.0f} s "
                      f"before its first draw; value = the workload's {m_final} samples over that time; "
                      f"greedy cover and AMCERA excluded; {host_desc()}"}


def copy_probe():
    import torch
    x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")   # 1 GiB
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(8):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_probe_bytes_read_per_launch": 1 << 30, "copy_probe_bytes_written_per_launch": 1 << 30,
                      "launches": 8, "GBps_read_plus_write": round(8 * 2 * (1 << 30) / dt / 1e9, 1)}), flush=True)


def sweeps():
    """Synthetic analogues of the paper's experiments on t and m (Section 5):
    the fixed-size bound (one iteration, delta itself) on the sparse
    workload's graph, k = 50, delta = 0.05; eta, AMCERA and phase times
    against t at m = 500,000, and eta against m at t = 100.  Prints one
    JSON line."""
    import torch
    from paper_2306_03651_amd import binding, inputs
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    W = WORKLOADS["sparse"]
    g = inputs.ba_graph(W["n"], W["m0"], W["graph_seed"])
    ctx = binding.centra_create(0, 0)
    dg = binding.DeviceGraph(ctx, g)
    stream = torch.cuda.current_stream()

    def fixed(m, t):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, picks, res, _ = binding.centra_progressive(ctx, dg.handle, 50, t, 0.01, 0.05, W["seed"], W["instance"],
                                                       m, m, 2, 1, stream=stream,
                                                       schedule=binding.CENTRA_SCHEDULE_FIXED)
        torch.cuda.synchronize()
        return {"m": m, "t": t, "eta": res.eta, "amcera": res.amcera, "c_hat": res.c_hat, "r": res.r,
                "ms_total": round(1e3 * (time.perf_counter() - t0), 2),
                "phase_ms": {"sample": round(res.ms_sample, 2), "cover": round(res.ms_cover, 2),
                             "mcera": round(res.ms_mcera, 2)}}

    fixed(100_000, 10)   # warm-up
    over_t = []
    for t in [1, 10, 50, 100, 200, 500, 1000]:
        over_t.append(fixed(500_000, t))
        log(f"t sweep: {over_t[-1]}")
    over_m = []
    for m in [50_000, 100_000, 200_000, 500_000, 1_000_000]:
        over_m.append(fixed(m, 100))
        log(f"m sweep: {over_m[-1]}")
    dg.release()
    binding.centra_destroy(ctx)
    print(json.dumps({"sweep": "fixed-size bound on " + W["label"].split(";")[0] + "; k=50, delta=0.05",
                      "over_t": over_t, "over_m": over_m}), flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def batched_bench(args):
    """Plain (one centra_progressive call per instance, one after the
    other) against the engine (every instance a pool with one query, run
    together), on the same instances; results must be identical."""
    import numpy as np
    import torch
    from paper_2306_03651_amd import binding, inputs
    W = ENGINE_WORKLOADS["batched"]
    mix = inputs.uneven_instances(W["count"], W["mix_seed"], W["ba_n"], W["grid_side"], W["k"])
    t0 = time.time()
    graphs = [inputs.instance_graph(kind, size, gs) for kind, size, gs, _ in mix]
    log(f"{len(graphs)} graphs built in {time.time() - t0:.1f}s "
        f"({sum(1 for m in mix if m[0] == 'ba')} BA, {sum(1 for m in mix if m[0] == 'grid')} grids)")
    ctx = binding.centra_create(0, 0)
    dgs = [binding.DeviceGraph(ctx, g) for g in graphs]
    stream = torch.cuda.current_stream()

    def plain():
        out = []
        for i, (dg, (_, _, _, k)) in enumerate(zip(dgs, mix)):
            out.append(binding.centra_progressive(ctx, dg.handle, k, W["t"], W["eps"], W["delta"], W["seed"], i,
                                                  W["m_init"], W["m_max"], stream=stream))
        torch.cuda.synchronize()
        return out

    def batched(flags=0):
        eng = binding.Engine(ctx, 0, flags)
        try:
            qs = []
            for i, (dg, (_, _, _, k)) in enumerate(zip(dgs, mix)):
                pid = eng.add_pool(dg.handle, W["seed"], i, W["t"], W["m_init"], W["m_max"])
                qs.append(eng.submit(pid, k, W["t"], W["eps"], W["delta"]))
            eng.run(stream=stream)
            torch.cuda.synchronize()
            return [eng.result(q) for q in qs], eng.stats(), eng.log()
        finally:
            eng.destroy()

    for i in range(args.warmup):
        batched()
        plain()
        log(f"warmup {i} done")
    tp, tb = [], []
    for i in range(args.steps):
        ts = time.perf_counter()
        res_p = plain()
        tp.append(time.perf_counter() - ts)
        ts = time.perf_counter()
        res_b, st, tune_log = batched()
        tb.append(time.perf_counter() - ts)
        log(f"step {i}: plain {tp[-1]:.3f}s, batched {tb[-1]:.3f}s")
    same = all(a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2].coverage == b[2].coverage and
               a[2].eta == b[2].eta for a, b in zip(res_p, res_b))
    paths = sum(int(r[2].m_final) for r in res_b)
    mp, mb = sum(tp) / len(tp), sum(tb) / len(tb)
    for dg in dgs:
        dg.release()
    binding.centra_destroy(ctx)
    out = {"metric": "time to certified top-k over 256 uneven instances (batched vs plain)", "value": round(mb, 4),
           "unit": "s", "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "dtype": "u64", "data": "synthetic", "config": {"workload": W["label"]},
           "batched_s": round(mb, 4), "plain_s": round(mp, 4), "speedup_vs_plain": round(mp / mb, 3),
           "paths_per_s_batched": round(paths / mb, 1), "paths_per_s_plain": round(paths / mp, 1),
           "certified": sum(int(r[2].certified) for r in res_b), "instances": len(res_b),
           "results_identical": bool(same),
           "engine": {"ticks": st.ticks, "sampler_launches": st.sampler_launches, "graph_replays": st.graph_replays,
                      "graphs_captured": st.graphs_captured, "tuned_block": st.tuned_block,
                      "ms_sample": round(st.ms_sample, 2), "ms_levels": round(st.ms_levels, 2),
                      "ms_greedy": round(st.ms_greedy, 2), "ms_select": round(st.ms_select, 2),
                      "peak_bytes": st.peak_bytes, "autotune": tune_log.strip()},
           "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)


def serving_bench(args):
    """A Poisson stream of queries over 8 resident graphs, served by the
    engine in real time (continuous batching); latency = completion time -
    arrival time of each query."""
    import numpy as np
    import torch
    from paper_2306_03651_amd import binding, inputs
    W = ENGINE_WORKLOADS["serving"]
    t0 = time.time()
    spec = [("ba", 1), ("ba", 2), ("ba", 3), ("ba", 4), ("rmat", 1), ("rmat", 2), ("grid", 0), ("grid", 0)]
    graphs = []
    for kind, gs in spec:
        if kind == "ba":
            graphs.append(inputs.ba_graph(1_000_000, 5, gs))
        elif kind == "rmat":
            graphs.append(inputs.rmat_graph(20, 16, seed=gs))
        else:
            graphs.append(inputs.grid_graph(2048))
    log(f"8 graphs built in {time.time() - t0:.1f}s")
    ctx = binding.centra_create(0, 0)
    dgs = [binding.DeviceGraph(ctx, g) for g in graphs]
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(W["arrival_seed"])
    queries = []
    tarr = 0.0
    while True:
        tarr += float(rng.exponential(1.0 / W["rate"]))
        if tarr > W["duration"]:
            break
        queries.append((int(rng.integers(8)), int(rng.integers(W["k"][0], W["k"][1] + 1)),
                        float(rng.choice(W["eps"])), tarr))
    eng = binding.Engine(ctx, 0)
    try:
        for i, (kind, _) in enumerate(spec):
            m_init, m_max = (1_000, 16_000) if kind == "grid" else (100_000, 6_400_000)
            eng.add_pool(dgs[i].handle, W["seed"], i, W["t"], m_init, m_max)
        qids = [eng.submit(gi, k, W["t"], eps, W["delta"], a) for gi, k, eps, a in queries]
        # resident sample sets: every pool drawn and built to its cap before
        # the stream starts
        tp = time.perf_counter()
        for i, (kind, _) in enumerate(spec):
            eng.prefill(i, 16_000 if kind == "grid" else 6_400_000, stream=stream)
        torch.cuda.synchronize()
        prefill_s = time.perf_counter() - tp
        log(f"pools prefilled in {prefill_s:.1f}s; {len(queries)} queries over {W['duration']} s")
        ts = time.perf_counter()
        eng.run(realtime=True, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - ts
        res = [eng.result(q) for q in qids]
        st = eng.stats()
        tune_log = eng.log()
    finally:
        eng.destroy()
    lat = [r[3].finished_s - r[3].arrival_s for r in res]
    waits = [r[3].admitted_s - r[3].arrival_s for r in res]
    last = max(r[3].finished_s for r in res)
    by_graph = {}
    for (gi, k, eps, a), r, l in zip(queries, res, lat):
        by_graph.setdefault(spec[gi][0], []).append(l)
    # the same query alone (a fresh engine) equals its result in the mix
    alone_same = True
    for idx in range(min(3, len(queries))):
        gi, k, eps, a = queries[idx]
        e1 = binding.Engine(ctx, 0, binding.CENTRA_ENGINE_NO_TUNE)
        try:
            kind = spec[gi][0]
            m_init, m_max = (1_000, 16_000) if kind == "grid" else (100_000, 6_400_000)
            e1.add_pool(dgs[gi].handle, W["seed"], gi, W["t"], m_init, m_max)
            q = e1.submit(0, k, W["t"], eps, W["delta"], 0.0)
            e1.run(stream=stream)
            r1 = e1.result(q)
        finally:
            e1.destroy()
        alone_same &= bool(r1[0] == res[idx][0] and np.array_equal(r1[1], res[idx][1]) and
                           r1[2].eta == res[idx][2].eta)
    # the plain form on the first queries: each query alone, one after the
    # other, with centra_progressive (no shared samples): its service time
    plain_times = []
    for gi, k, eps, a in queries[:args.plain_queries]:
        kind = spec[gi][0]
        m_init, m_max = (1_000, 16_000) if kind == "grid" else (100_000, 6_400_000)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        binding.centra_progressive(ctx, dgs[gi].handle, k, W["t"], eps, W["delta"], W["seed"], gi, m_init, m_max,
                                   stream=stream)
        torch.cuda.synchronize()
        plain_times.append(time.perf_counter() - tq)
    for dg in dgs:
        dg.release()
    binding.centra_destroy(ctx)
    served = len(res) / last if last > 0 else None
    out = {"metric": "serving latency and throughput (continuous batching)", "value": round(served, 2),
           "unit": "queries/s", "higher_is_better": True, "n_gpus": 1, "steps": 1, "warmup": 0, "dtype": "u64",
           "data": "synthetic", "config": {"workload": W["label"]},
           "queries": len(res), "offered_qps": W["rate"], "served_qps": round(served, 2),
           "wall_s": round(wall, 3), "prefill_s": round(prefill_s, 2),
           "latency_p50_s": round(percentile(lat, 50), 4), "latency_p99_s": round(percentile(lat, 99), 4),
           "latency_max_s": round(max(lat), 4), "queue_wait_p50_s": round(percentile(waits, 50), 4),
           "latency_p50_by_graph_s": {k: round(percentile(v, 50), 4) for k, v in by_graph.items()},
           "certified": sum(int(r[2].certified) for r in res),
           "alone_equals_mix": alone_same,
           "plain_service_s": [round(x, 3) for x in plain_times],
           "plain_qps_estimate": round(len(plain_times) / sum(plain_times), 3) if plain_times else None,
           "plain_note": f"the first {len(plain_times)} queries served one at a time by centra_progressive "
                         "(no shared samples); plain_qps_estimate = queries / their summed service time",
           "engine": {"ticks": st.ticks, "peak_active": st.peak_active, "greedy_runs": st.greedy_runs,
                      "sampler_launches": st.sampler_launches,
                      "samples": st.samples, "graph_replays": st.graph_replays, "tuned_block": st.tuned_block,
                      "ms_sample": round(st.ms_sample, 1), "ms_levels": round(st.ms_levels, 1),
                      "ms_greedy": round(st.ms_greedy, 1), "ms_select": round(st.ms_select, 1),
                      "peak_bytes": st.peak_bytes, "autotune": tune_log.strip()},
           "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="time budget of the oracle CPU baseline")
    ap.add_argument("--m-max", type=int, default=WORKLOAD["m_max"], help=argparse.SUPPRESS)
    ap.add_argument("--uncapped-max", type=int, default=None,
                    help="sample cap of the extra runs that measure time to certified (0 = skip; default 128M for "
                         "the sparse workload, 32M for the skewed one, 64M for triangles, 10M for small)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + sorted(ENGINE_WORKLOADS), default="sparse",
                    help="sparse (default): BA n=1e6; skewed: R-MAT scale 22, directed; small: BA n=2,000; "
                         "triangles: the triangle space of R-MAT scale 20, undirected")
    ap.add_argument("--sweep", action="store_true",
                    help="run only the t and m sweeps of the fixed-size bound (one JSON line)")
    ap.add_argument("--hedge", action="store_true",
                    help="also run HEDGE-P (union bound, same schedule) to certification, outside the timed steps")
    ap.add_argument("--sampler", choices=["single", "bidir"], default="single",
                    help="shortest-path workloads: the single-source sampler (default) or the balanced "
                         "bidirectional one (centra_sample_paths_bidir)")
    ap.add_argument("--plain-queries", type=int, default=8,
                    help="serving workload: queries also served one at a time by centra_progressive")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy 8 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.sweep:
        sweeps()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the hot path is single-GPU here); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_03651_amd import binding, inputs

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.workload == "batched":
        batched_bench(args)
        return
    if args.workload == "serving":
        serving_bench(args)
        return
    W = dict(WORKLOADS[args.workload])
    tri = W.get("space") == "triangles"
    kp = W.get("space") == "kpaths"
    bidir = args.sampler == "bidir" and not (tri or kp)
    space = (binding.CENTRA_SPACE_TRIANGLES if tri else binding.CENTRA_SPACE_KPATHS if kp
             else binding.CENTRA_SPACE_PATHS_BIDIR if bidir else binding.CENTRA_SPACE_SHORTEST_PATHS)
    kappa = W.get("kappa", 0)
    if args.uncapped_max is None:
        args.uncapped_max = {"sparse": 128_000_000, "skewed": 32_000_000, "triangles": 64_000_000,
                             "kpaths": 64_000_000, "small": 10_000_000}[args.workload]
    if args.workload == "sparse":
        W["m_max"] = args.m_max
    t0 = time.time()
    if W["graph"] == "rmat":
        g = inputs.rmat_graph(W["scale"], W["edge_factor"], seed=W["graph_seed"])
    elif W["graph"] == "rmat_undirected":
        import numpy as np
        d = inputs.rmat_graph(W["scale"], W["edge_factor"], seed=W["graph_seed"])
        src = np.repeat(np.arange(d.n), np.diff(d.row_ptr.astype(np.int64)))
        g = inputs.from_edges(d.n, src, d.col_idx, directed=False)
        del d, src
    else:
        g = inputs.ba_graph(W["n"], W["m0"], W["graph_seed"])
    log(f"graph: n={g.n} arcs={g.n_arcs} ({time.time() - t0:.1f}s)")
    ctx = binding.centra_create(0, 0)
    dg = binding.DeviceGraph(ctx, g)
    stream = torch.cuda.current_stream()
    index_s = None
    n_triangles = None
    if tri:
        torch.cuda.synchronize()
        ti = time.perf_counter()
        n_triangles = binding.centra_triangle_count(ctx, dg.handle, stream=stream)
        torch.cuda.synchronize()
        index_s = time.perf_counter() - ti
        log(f"triangle index: T={n_triangles} in {index_s:.3f}s")

    def step():
        return binding.centra_progressive(ctx, dg.handle, W["k"], W["t"], W["eps"], W["delta"], W["seed"],
                                          W["instance"], W["m_init"], W["m_max"], W["growth"], 1,
                                          stream=stream, space=space, kappa=kappa)

    for i in range(args.warmup):
        rc, picks, res, itlog = step()
        log(f"warmup {i}: m={res.m_final} iters={res.iterations} certified={res.certified} "
            f"eta={res.eta:.5f} ms={res.ms_total:.0f}")
    binding.centra_sampler_stats_get(ctx, reset=True)
    torch.cuda.synchronize()
    paths = 0
    times = []
    results = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        rc, picks, res, itlog = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        paths += res.m_final
        results.append((rc, picks, res, itlog))
        log(f"step {i}: {times[-1]:.3f}s m={res.m_final} iters={res.iterations} certified={res.certified} "
            f"eta={res.eta:.5f} c_hat={res.c_hat:.4f}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    st = binding.centra_sampler_stats_get(ctx)
    rc, picks, res, itlog = results[-1]
    # time to certified (outside the timed steps): the same doubling schedule
    # without the 4M cap, and the paper's own schedule (growth 1.2 with the
    # optimistic guess)
    def uncapped_run(num, den, schedule, method=binding.CENTRA_METHOD_CENTRA):
        torch.cuda.synchronize()
        tu = time.perf_counter()
        urc, upicks, ures, ulog = binding.centra_progressive(
            ctx, dg.handle, W["k"], W["t"], W["eps"], W["delta"], W["seed"], W["instance"], W["m_init"],
            args.uncapped_max, num, den, stream=stream, schedule=schedule, space=space, kappa=kappa, method=method)
        torch.cuda.synchronize()
        return {"time_s": round(time.perf_counter() - tu, 3), "certified": bool(ures.certified),
                "m_final": int(ures.m_final), "iterations": int(ures.iterations),
                "m_schedule": [int(it.m) for it in ulog], "eta": ures.eta, "c_hat": ures.c_hat,
                "picks_head": [int(x) for x in upicks[:10]]}

    uncapped = adaptive = None
    if args.uncapped_max > 0:
        uncapped = uncapped_run(W["growth"], 1, binding.CENTRA_SCHEDULE_GEOMETRIC)
        log(f"uncapped: {uncapped}")
        adaptive = uncapped_run(6, 5, binding.CENTRA_SCHEDULE_ADAPTIVE)
        log(f"adaptive: {adaptive}")
    hedge = None
    if args.hedge:
        # HEDGE-P (Sec. 5's comparison method): the same doubling schedule
        # and sampler with the union bound in place of the AMCERA
        hedge = uncapped_run(W["growth"], 1, binding.CENTRA_SCHEDULE_GEOMETRIC, binding.CENTRA_METHOD_HEDGE_P)
        log(f"hedge-p: {hedge}")
    ctx_log = binding.centra_context_log(ctx).strip()
    dg.release()
    binding.centra_destroy(ctx)

    launches = max(1, st.launches)
    if tri:
        bytes_per_launch = TRIANGLE_SAMPLE_BYTES * st.samples / launches
    elif kp:
        bytes_per_launch = (KPATH_NODE_BYTES * st.hyperedge_nodes + KPATH_SAMPLE_BYTES * st.samples) / launches
    else:
        bytes_per_launch = (4.0 * st.arcs + 28.0 * st.nodes) / launches
    sec_per_launch = st.kernel_ms / 1e3 / launches
    achieved = bytes_per_launch / sec_per_launch / 1e9
    traffic = None if bidir else read_traffic(W["traffic"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_tri_sample" if tri else "k_kpath + k_kpath_gather" if kp else
                "k_sample_bidir" if bidir else "k_sample_paths",
                "launches": st.launches,
                "avg_launch_ms": round(st.kernel_ms / launches, 3),
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
                "kernel_share_of_steps": round(st.kernel_ms / 1e3 / total, 4)}
    if not tri and not kp:
        roofline.update({"arcs_per_path": round(st.arcs / max(1, st.samples), 1),
                         "nodes_per_path": round(st.nodes / max(1, st.samples), 1),
                         "entries_per_path": round(st.hyperedge_nodes / max(1, st.samples), 3),
                         "visited_set": "lds bitmap" if st.lds_bitmap else "lds bloom filter + hbm records",
                         "concurrent_bfs": st.slots, "wide_samples": st.wide,
                         "wide_ms_per_step": round(st.wide_ms / max(1, args.steps), 2),
                         "wide_arcs_per_wide_sample": round(st.wide_arcs / max(1, st.wide))})

    cpu = cpu_all = None
    if args.cpu_seconds > 0:
        if tri:
            cpu = cpu_baseline_triangles(g, args.cpu_seconds, int(res.m_final))
        else:
            cpu = cpu_baseline(g, args.cpu_seconds, W)
            cpu_all = cpu_baseline_all_cores(g, args.cpu_seconds, W)
        log(f"cpu baseline: {cpu}")
    value = paths / total
    out = {
        "metric": "triangles sampled/s" if tri else "kappa-path walks sampled/s" if kp else "shortest paths sampled/s",
        "value": round(value, 1),
        "unit": "triangles/s" if tri else "walks/s" if kp else "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if (tri or kp) else "u64",
        "data": "synthetic",
        "config": {"workload": W["label"] + ("; balanced bidirectional sampler" if bidir else ""),
                   "n": int(g.n), "arcs": int(g.n_arcs), "m_init": W["m_init"], "m_max": W["m_max"],
                   "k": W["k"], "t": W["t"], "eps": W["eps"], "delta": W["delta"]},
        "triangles": n_triangles,
        "index_s": round(index_s, 4) if index_s is not None else None,
        "time_to_certified_s": round(sum(times) / len(times), 3) if res.certified else
        (uncapped["time_s"] if uncapped and uncapped["certified"] else None),
        "time_to_cap_s": None if res.certified else round(sum(times) / len(times), 3),
        "uncapped_run": uncapped,
        "time_to_certified_adaptive_s": adaptive["time_s"] if adaptive and adaptive["certified"] else None,
        "uncapped_adaptive_run": adaptive,
        "hedge_p_run": hedge,
        "certified": bool(res.certified),
        "m_final": int(res.m_final),
        "iterations": int(res.iterations),
        "eta": res.eta,
        "c_hat": res.c_hat,
        "stop_lhs_over_rhs": (1 - 1 / 2.718281828459045) * ((1 - 1 / 2.718281828459045 - W["eps"]) * res.xi + res.eta)
        / (W["eps"] * res.c_hat) if res.c_hat > 0 else None,
        "phase_ms": {"sample": round(res.ms_sample, 1), "cover": round(res.ms_cover, 1),
                     "mcera": round(res.ms_mcera, 1)},
        "roofline": roofline,
        "slot_placement": ctx_log or None,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
