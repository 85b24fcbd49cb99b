"""Benchmark: SPC label index build + batched SPC queries on one MI355X.

Default line (the largest single-GPU workload): R-MAT scale 21 (2,097,152
vertices, edge factor 16, a,b,c,d = 0.57,0.19,0.19,0.05, seed 5), degree
order.  The index is built once, timed (host clock around the build call,
CSR resident in HBM); then each step is one batch of 10M uniform SPC queries
on the resident index (HIP events around the launch); then the served
level at 1.0x saturation (Poisson arrivals, batch sizes log-uniform in
1..65536) gives p50/p99 latency beside a one-request-at-a-time FIFO.
`value` is label entries built per second; `queries_per_s` and p50/p99 sit
beside it.  A side object repeats the Chung-Lu n = 2^20 build (where the
oracle's byte model of the build exists) with its own roofline.

Other workloads (--workload): chunglu (the Chung-Lu line on its own),
rmat_batch (512 R-MAT graphs, batched vs plain), rmat_served (offered-load
sweep), grid (k x k grid, round cap or ordering variants).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "label entries built/sec + SPC queries/sec (bit-exact); p50/p99 query latency"
PROFILES = os.path.join(ROOT, "profiles")


def source_hash(src: str = "build.hip") -> str:
    h = hashlib.sha256()
    p = os.path.join(ROOT, "paper_2212_00977_amd", "csrc", src)
    h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name: str, src: str = "build.hip"):
    """HBM bytes per launch of a kernel on a workload from the committed
    rocprofv3 counter summary profiles/<name>_traffic.json, if it was taken
    on the current source of the kernel (else None)."""
    path = os.path.join(PROFILES, f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_hash") != source_hash(src):
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(g, seconds: float):
    """The oracle (sequential pruned BFS, hubs in rank order) on the same
    graph, stopped after `seconds`: entries it produced per second."""
    import oracle

    order = oracle.degree_order(g.off)
    roff, radj = oracle.relabel(g.off, g.adj, order)
    lib = oracle.lib()
    t0 = time.perf_counter()
    h = lib.oracle_build_pruned(g.n, roff, radj, 0, 0, seconds)
    dt = time.perf_counter() - t0
    e = lib.oracle_index_entries(h)
    hubs = lib.oracle_index_hubs_done(h)
    lib.oracle_index_free(h)
    return {"value": e / dt, "unit": "label entries/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential pruned BFS over the first {hubs} hubs in rank order "
                      f"({e} entries, {dt:.1f} s) of the same graph"}


def serve_runs(ix, n, args, sat_qps, log):
    import numpy as np

    """Open-loop served load on the resident index: Poisson request arrivals,
    batch sizes log-uniform in [1, 65536], offered at a fraction of the
    measured batch query rate; continuous batching vs one-at-a-time FIFO."""
    from paper_2212_00977_amd import inputs, serve

    mean_batch = 65536 / np.log(65537) - 0.5  # E[floor(exp(U[0, ln 65537)))]
    levels = [0.25, 0.5, 0.75, 1.0, 1.25] if args.serve_sweep else [0.5]
    res = []
    for lv in levels:
        rate = lv * sat_qps / mean_batch
        count = min(2000, max(20, int(rate * max(args.serve_seconds, 1.0))))
        reqs = serve.requests_from(inputs.poisson_requests(n, rate, count, seed=7 + int(100 * lv)))
        srv = serve.Server(ix, io_budget_bytes=1 << 30, streams=4, max_batch=1 << 18)
        srv.run(reqs[: min(10, len(reqs))])  # warm the streams and host buffers
        st = srv.run(reqs).summary()
        base = serve.fifo_baseline(ix, reqs).summary()
        entry = {"offered_fraction": lv, "offered_requests_per_s": rate,
                 "served": st, "fifo": base}
        log(f"serve {lv:.2f}x: {st['queries_per_s']:.3g} q/s p50 {st['p50_ms']:.2f} ms "
            f"p99 {st['p99_ms']:.2f} ms | fifo p50 {base['p50_ms']:.2f} p99 {base['p99_ms']:.2f}")
        if args.serve_sweep:
            print(json.dumps({"serve_level": entry}), flush=True)
        res.append(entry)
    r0 = res[0]
    return {"offered_fraction": r0["offered_fraction"], "queries_per_s": r0["served"]["queries_per_s"],
            "p50_ms": r0["served"]["p50_ms"], "p99_ms": r0["served"]["p99_ms"],
            "fifo_p50_ms": r0["fifo"]["p50_ms"], "fifo_p99_ms": r0["fifo"]["p99_ms"],
            "requests": r0["served"]["requests"], "deferred": r0["served"]["deferred"],
            "launches": r0["served"]["launches"]}


def bench_served(args, dev, log):
    """Served load on a resident index: R-MAT scale 21 (a,b,c,d = 0.57,0.19,
    0.19,0.05, edge factor 16, seed 5).  Saturation = served throughput of a
    burst of requests all arriving at once; then Poisson arrivals at 0.25 ..
    1.25 x saturation (batch sizes log-uniform in [1, 65536], uniform pairs),
    continuous batching vs one request at a time (FIFO), latency from each
    request's scheduled arrival."""
    import numpy as np
    import torch

    from paper_2212_00977_amd import inputs, serve, spc

    scale = 21 - args.scale_down
    log(f"generating R-MAT scale {scale}")
    g = inputs.rmat(scale, 16, seed=5)
    off_d = torch.from_numpy(g.off.view(np.int64)).to(dev)
    adj_d = torch.from_numpy(g.adj.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    ix = spc.build_index(off_d, adj_d, device=dev, stream=stream,
                         opts=spc.BuildOptions(one_shell=args.one_shell, equivalence=args.equivalence))
    build_ms = (time.perf_counter() - t0) * 1e3
    st = ix.stats()
    log(f"build {build_ms:.0f} ms, {st['entries']} entries, fringe {st['fringe_vertices']}, "
        f"twins {st['twin_vertices']}, peak {st['peak_build_bytes'] / 2**30:.1f} GiB")
    del off_d, adj_d
    spc.release_cached_memory()
    torch.cuda.empty_cache()
    ts, tt = inputs.queries(g.n, 1_000_000, seed=3)
    qcfg = ix.tune_queries(ts, tt, stream=stream)
    log(f"query autotuner: configuration {qcfg} {spc.query_configs()[qcfg]}")

    mean_batch = 65536 / np.log(65537) - 0.5
    srv_kw = dict(io_budget_bytes=1 << 30, streams=args.serve_streams, max_batch=args.serve_max_batch)
    # saturation: a burst (every request at t = 0)
    burst = serve.requests_from(inputs.poisson_requests(g.n, 1e9, args.serve_requests // 2, seed=6))
    for r in burst:
        r.arrival = 0.0
    srv = serve.Server(ix, **srv_kw)
    srv.run(burst[:20])  # warm the streams and pinned host buffers
    serve.fifo_baseline(ix, burst[:20])
    sat = srv.run(burst).summary()
    sat_qps = sat["queries_per_s"]
    log(f"saturation: {sat_qps:.3g} q/s over {sat['requests']} requests")
    levels = []
    for lv in (0.25, 0.5, 0.75, 1.0, 1.25):
        rate = lv * sat_qps / mean_batch
        reqs = serve.requests_from(inputs.poisson_requests(g.n, rate, args.serve_requests,
                                                           seed=7 + int(100 * lv)))
        served = srv.run(reqs).summary()
        fifo = serve.fifo_baseline(ix, reqs).summary()
        log(f"{lv:.2f}x: served {served['queries_per_s']:.3g} q/s p50 {served['p50_ms']:.2f} ms "
            f"p99 {served['p99_ms']:.2f} ms deferred {served['deferred']} | fifo p50 "
            f"{fifo['p50_ms']:.2f} p99 {fifo['p99_ms']:.2f}")
        levels.append({"offered_fraction": lv, "offered_requests_per_s": rate, "served": served,
                       "fifo": fifo})
    ix.free()
    one = levels[3]["served"]
    out = {"metric": METRIC, "value": one["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
           "steps": len(levels), "warmup": 1, "ms_per_step": one["makespan_s"] * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic",
           "config": {"workload": f"served SPC queries on a resident R-MAT scale {scale} index "
                                  "(ef 16, seed 5); Poisson requests, batch sizes log-uniform "
                                  "in 1..65536; value = served q/s at 1.0x saturation",
                      "n": g.n, "m": g.m, "entries": st["entries"], "rounds": st["rounds"],
                      "requests_per_level": args.serve_requests, "max_batch": args.serve_max_batch,
                      "streams": args.serve_streams, "one_shell": args.one_shell,
                      "equivalence": args.equivalence, "fringe_vertices": st["fringe_vertices"],
                      "twin_vertices": st["twin_vertices"], "parallelism": "single-gpu"},
           "p50_ms": one["p50_ms"], "p99_ms": one["p99_ms"],
           "build_ms": build_ms, "build_entries_per_s": st["entries"] / (build_ms * 1e-3),
           "query_config": dict(zip(("stage", "tiles"), spc.query_configs()[qcfg])),
           "index_bytes": st["index_bytes"], "peak_build_bytes": st["peak_build_bytes"],
           "saturation": sat, "levels": levels}
    print(json.dumps(out), flush=True)


def bench_grid(args, dev, log):
    """High-diameter workload: k x k 4-neighbour grid, 5% of edges deleted
    uniformly (seed 3), largest component, degree order with seeded random
    ties.  With a round cap D the index is L_{<=D}: answers up to D are
    exact, longer ones carry the horizon flag."""
    import numpy as np
    import torch

    from paper_2212_00977_amd import inputs, spc

    k = args.grid_k
    log(f"generating grid {k}x{k}")
    g = inputs.grid_lcc(k, 0.05, seed=3)
    off_d = torch.from_numpy(g.off.view(np.int64)).to(dev)
    adj_d = torch.from_numpy(g.adj.view(np.int32)).to(dev)
    tie_d = torch.from_numpy(g.tie_key.view(np.int64)).to(dev)
    order_d, order_ms, core = None, 0.0, None
    if args.order != "degree":  # host-side hybrid / tree-decomposition order
        delta = 0xFFFFFFFF if args.order == "td" else args.delta
        t0 = time.perf_counter()
        order_np, core = spc.hybrid_order(g.off, g.adj, delta)
        order_ms = (time.perf_counter() - t0) * 1e3
        order_d = torch.from_numpy(order_np.view(np.int32)).to(dev)
        tie_d = None
        log(f"{args.order} order on the host: {order_ms:.0f} ms, core {core}")
    s_np, t_np = inputs.queries(g.n, args.queries, seed=3)
    s_d = torch.from_numpy(s_np.view(np.int32)).to(dev)
    t_d = torch.from_numpy(t_np.view(np.int32)).to(dev)
    stream = torch.cuda.current_stream()
    opts = spc.BuildOptions(round_cap=args.round_cap)
    torch.cuda.synchronize()
    runs = []
    for i in range(args.warmup + args.steps):
        t0 = time.perf_counter()
        ix = spc.build_index(off_d, adj_d, order=order_d, tie_key=tie_d, opts=opts, device=dev,
                             stream=stream)
        bms = (time.perf_counter() - t0) * 1e3
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        dist, cnt, flg = ix.query(s_d, t_d, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        qms = ev0.elapsed_time(ev1)
        st = ix.stats()
        log(f"{'warmup' if i < args.warmup else 'step'} {i}: build {bms:.0f} ms, query {qms:.1f} ms, "
            f"entries {st['entries']}, rounds {st['rounds']}")
        if i >= args.warmup:
            runs.append((bms, qms))
        f = flg.cpu().numpy()
        ix.free()
    bms = float(np.mean([r[0] for r in runs]))
    qms = float(np.mean([r[1] for r in runs]))
    horizon = int(((f & spc.FLAG_HORIZON) != 0).sum())
    # the paper counts ordering in indexing time: a host-side order is part
    # of every build's time (the degree order runs inside the build)
    out = {"metric": METRIC, "value": st["entries"] / ((order_ms + bms) * 1e-3), "unit": "label entries/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": order_ms + bms + qms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic",
           "config": {"workload": f"grid {k}x{k}, 5% edges deleted, LCC, seed 3, "
                                  f"{'degree order, random ties' if args.order == 'degree' else args.order + ' order'}, "
                                  f"round cap {args.round_cap or 'none'}, {args.queries} queries",
                      "order": args.order, "order_host_ms": order_ms, "core": core,
                      "n": g.n, "m": g.m, "entries": st["entries"], "rounds": st["rounds"],
                      "truncated": bool(st["truncated"]), "dist_bits": st["dist_bits"],
                      "parallelism": "single-gpu"},
           "build_ms": order_ms + bms, "build_ms_device": bms,
           "device_entries_per_s": st["entries"] / (bms * 1e-3),
           "query_ms": qms, "queries_per_s": args.queries / (qms * 1e-3),
           "queries_beyond_horizon": horizon, "index_bytes": st["index_bytes"],
           "peak_build_bytes": st["peak_build_bytes"]}
    print(json.dumps(out), flush=True)


def bench_batch(args, dev, log):
    """512 independent R-MAT graphs (a,b,c,d = 0.57,0.19,0.19,0.05, edge factor
    8, scales uniform in 10..16, seed 4): one batched build vs one plain build
    per graph; then 10,000 queries per graph (uneven label lengths)."""
    import numpy as np
    import torch

    from paper_2212_00977_amd import inputs, spc

    log("generating graphs")
    graphs = inputs.rmat_batch(args.batch_graphs, seed=4)
    N = sum(g.n for g in graphs)
    M = sum(g.m for g in graphs)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # inputs resident in HBM before timing
    dev_graphs = []
    for g in graphs:
        dev_graphs.append(inputs.Graph(g.n, torch.from_numpy(g.off.view(np.int64)).to(dev),
                                       torch.from_numpy(g.adj.view(np.int32)).to(dev), g.name))
    qs = [inputs.queries(g.n, 10000, seed=1000 + i) for i, g in enumerate(graphs)]
    s_d = [torch.from_numpy(s.view(np.int32)).to(dev) for s, _ in qs]
    t_d = [torch.from_numpy(t.view(np.int32)).to(dev) for _, t in qs]
    torch.cuda.synchronize()

    opts = spc.BuildOptions(one_shell=args.one_shell, equivalence=args.equivalence)

    def batched():
        t0 = time.perf_counter()
        ix = spc.build_index_batch(dev_graphs, device=dev, stream=stream, opts=opts)
        t1 = time.perf_counter()
        return ix, (t1 - t0) * 1e3

    def plain():
        # each form starts from the same memory state: the cache keeps freed
        # blocks by size, and blocks given back to the runtime are cleared by
        # the driver before their next use (seconds per 100 GB)
        spc.release_cached_memory()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        entries = 0
        for g in dev_graphs:
            ix = spc.build_index(g.off, g.adj, device=dev, stream=stream, opts=opts)
            entries += ix.stats()["entries"]
            ix.free()
        return entries, (time.perf_counter() - t0) * 1e3

    spc.release_cached_memory()
    for _ in range(args.warmup):
        ix, _ = batched()
        ix.free()
    runs = []
    for i in range(args.steps):
        ix, ms = batched()
        runs.append(ms)
        log(f"batched build {i}: {ms:.1f} ms")
        if i < args.steps - 1:
            ix.free()
    st = ix.stats()
    entries = st["entries"]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # every graph's queries in one bucketed call (threshold tuned on a sample
    # of the same mix), against one launch per graph
    gid_d = torch.cat([torch.full((10000,), gi, dtype=torch.int32, device=dev) for gi in range(len(graphs))])
    sa_d, ta_d = torch.cat(s_d), torch.cat(t_d)
    samp = torch.randperm(gid_d.shape[0], device=dev)[:200000]
    small = ix.tune_query_buckets(gid_d[samp], sa_d[samp], ta_d[samp], stream=stream)
    ix.query_multi(gid_d, sa_d, ta_d, stream=stream)  # warm
    torch.cuda.synchronize()
    ev0.record(stream)
    ix.query_multi(gid_d, sa_d, ta_d, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    qms = ev0.elapsed_time(ev1)
    ev0.record(stream)
    for gi in range(len(graphs)):
        ix.query(s_d[gi], t_d[gi], graph_id=gi, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    qms_each = ev0.elapsed_time(ev1)
    log(f"queries: one bucketed call {qms:.1f} ms (threshold {small}), one launch per graph {qms_each:.1f} ms")
    ix.free()
    pe, pms = plain()
    log(f"plain per-graph builds: {pms:.1f} ms ({pe} entries)")
    bms = float(np.mean(runs))
    out = {"metric": METRIC, "value": entries / (bms * 1e-3), "unit": "label entries/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": bms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic",
           "config": {"workload": f"{len(graphs)} R-MAT graphs, scales 10..16, ef 8, seed 4, "
                                  "one batched build + 10,000 queries per graph",
                      "graphs": len(graphs), "n": N, "m": M, "entries": entries,
                      "rounds": st["rounds"], "one_shell": args.one_shell,
                      "equivalence": args.equivalence, "fringe_vertices": st["fringe_vertices"],
                      "twin_vertices": st["twin_vertices"], "parallelism": "single-gpu"},
           "batched_build_ms": bms, "plain_build_ms": pms,
           "plain_entries_per_s": pe / (pms * 1e-3), "batched_speedup": pms / bms,
           "batched_breakdown_ms": {"device_total": st["ms_total"], "round_kernel": st["ms_round_kernel"],
                                    "host_and_launch": bms - st["ms_total"],
                                    "round_kernel_launches": st["round_kernel_launches"]},
           "query_ms": qms, "queries_per_s": 10000 * len(graphs) / (qms * 1e-3),
           "query_bucket_threshold": small, "query_ms_one_launch_per_graph": qms_each}
    print(json.dumps(out), flush=True)


def reduced_side(kind, off_d, adj_d, s_d, t_d, dev, stream, cfg, ref_d, ref_c, log, reps=2):
    """The same workload built with an index reduction -- kind "one_shell"
    (Section "Reduction by 1-Shell") or "equivalence" (Section "Reduction
    by Equivalence Relation"): build time, vertices cut off or merged, index
    size and query rate of the reduced index, and how many answers differ
    from the full index's (the last timed step's outputs).  Not part of the
    headline value."""
    import torch

    from paper_2212_00977_amd import spc

    nq = int(s_d.shape[0])
    opts = spc.BuildOptions(**{kind: True})
    builds, queries = [], []
    for i in range(reps):  # the first build warms the block cache
        t0 = time.perf_counter()
        ix = spc.build_index(off_d, adj_d, device=dev, stream=stream, opts=opts)
        builds.append((time.perf_counter() - t0) * 1e3)
        ix.set_query_config(cfg)
        bits = ix.dist_bits
        d = torch.empty(nq, dtype=torch.uint8 if bits == 8 else torch.int16, device=dev)
        c = torch.empty(nq, dtype=torch.int64, device=dev)
        f = torch.empty(nq, dtype=torch.uint8, device=dev)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        ix.query(s_d, t_d, stream=stream, out=(d, c, f))
        ev1.record(stream)
        torch.cuda.synchronize()
        queries.append(ev0.elapsed_time(ev1))
        st = ix.stats()
        if i < reps - 1:
            ix.free()
    same_bits = bits == 8
    diff = int(((d.to(torch.int32) != ref_d.to(torch.int32)) | (c != ref_c)).sum()) if same_bits else -1
    ix.free()
    out = {"build_ms": builds[-1], "query_ms": queries[-1], "queries_per_s": nq / (queries[-1] * 1e-3),
           "fringe_vertices": st["fringe_vertices"], "fringe_depth": st["fringe_depth"],
           "twin_vertices": st["twin_vertices"], "core_vertices": st["n"], "entries": st["entries"], "index_bytes": st["index_bytes"],
           "peak_build_bytes": st["peak_build_bytes"], "dist_bits": bits,
           "answers_differing_from_full_index": diff}
    log(f"{kind}: build {builds[-1]:.1f} ms, fringe {st['fringe_vertices']}, twins {st['twin_vertices']}, "
        f"entries {st['entries']}, queries {queries[-1]:.1f} ms, differing answers {diff}")
    return out


def _profile_json(name):
    """A committed summary under profiles/ (None if absent)."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    try:
        return json.load(open(path))
    except Exception:
        return None


def _roofline(kernel, bytes_total, ms_total, launches, model, traffic=None, **extra):
    """Roofline object of one kernel: algorithmic bytes per launch over the
    average launch duration (HIP events on the kernel's stream)."""
    avg_ms = ms_total / max(launches, 1)
    per_launch = bytes_total / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "launches": launches, "avg_launch_ms": avg_ms, "alg_bytes_per_launch": per_launch,
            "bytes_model": model, **extra}


def _s8d_round_kernel_bytes(prof, rounds_from=2):
    """The oracle's byte model summed over the rounds the round kernel runs
    (round 1 of a simple graph takes the sort path, not the round kernel)."""
    return sum(r["total"] for r in prof["rounds"] if r["round"] >= rounds_from)


def cpu_baselines(g_main, log, threads_sample_scale=17):
    """The oracle on the host cores, same run: (1) the threaded PULL build
    (all host threads) of R-MAT scale `threads_sample_scale`, edge factor
    16, seed 5 (the main workload's generator at a size the oracle finishes
    in seconds), and its threaded merge-join over 1M uniform queries; (2) the
    sequential pruned BFS on the main workload's graph itself for 10 s."""
    import oracle
    from paper_2212_00977_amd import inputs

    threads = oracle.host_threads()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    gs = inputs.rmat(threads_sample_scale, 16, seed=5)
    t0 = time.perf_counter()
    L = oracle.build_graph(gs, method="pull", threads=threads)
    bt = time.perf_counter() - t0
    s, t = inputs.queries(gs.n, 1_000_000, seed=2)
    rk = L.rank_of()
    rs, rt = rk[s], rk[t]
    t0 = time.perf_counter()
    oracle.query_arrays(L.off, L.hub, L.dist, L.count, rs, rt, threads=threads)
    qt = time.perf_counter() - t0
    log(f"cpu oracle: threaded PULL {L.entries} entries in {bt:.1f} s, 1M queries in {qt:.2f} s "
        f"({threads} threads)")
    one = cpu_baseline(g_main, 10.0)
    return {"value": L.entries / bt, "unit": "label entries/s", "cores": threads, "kind": "oracle",
            "sample": f"the oracle's threaded PULL build on {threads} host threads of R-MAT scale "
                      f"{threads_sample_scale}, edge factor 16, seed 5 (the workload's generator at "
                      f"1/{1 << (21 - threads_sample_scale)} of its vertices; {L.entries} entries, "
                      f"{bt:.1f} s): the full index of the workload is beyond the oracle",
            "queries_per_s": 1_000_000 / qt,
            "query_sample": f"the oracle's merge-join on {threads} threads, 1M uniform pairs over "
                            f"that index ({qt:.2f} s)",
            "single_core": one, "nproc": os.cpu_count(), "cpu_model": model}


def bench_rmat21(args, dev, log):
    """The default line: R-MAT scale 21, edge factor 16, seed 5.  One timed
    build; K steps of one 10M-query batch each on the resident index; the
    served level at 1.0x saturation against FIFO; the Chung-Lu build as a
    side object; the oracle on the host cores."""
    import numpy as np
    import torch

    from paper_2212_00977_amd import inputs, serve, spc

    scale = 21 - args.scale_down
    log(f"generating R-MAT scale {scale}")
    g = inputs.rmat(scale, 16, seed=5)
    off_d = torch.from_numpy(g.off.view(np.int64)).to(dev)
    adj_d = torch.from_numpy(g.adj.view(np.int32)).to(dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    # freed device memory stays with the library between builds: memory the
    # runtime takes back is cleared by the driver before its next use
    spc.set_cache_limit(None)
    first_ms = None
    if args.warmup > 0:  # an untimed build first (the memory of earlier processes is cleared here)
        t0 = time.perf_counter()
        ix0 = spc.build_index(off_d, adj_d, device=dev, stream=stream)
        first_ms = (time.perf_counter() - t0) * 1e3
        ix0.free()
        log(f"warmup build {first_ms:.0f} ms")
    t0 = time.perf_counter()
    ix = spc.build_index(off_d, adj_d, device=dev, stream=stream)
    build_ms = (time.perf_counter() - t0) * 1e3
    st = ix.stats()
    rs = {k: v.tolist() for k, v in {**ix.round_stats(), **ix.round_profile()}.items()}
    log(f"build {build_ms:.0f} ms, {st['entries']} entries, {st['rounds']} rounds, "
        f"{st['round_kernel_launches']} round-kernel launches, "
        f"peak {st['peak_build_bytes'] / 2**30:.1f} GiB")
    for r in range(len(rs["kept"])):
        log("round %d: raw %d merged %d kept %d  %.1f ms" % (r, rs["raw"][r], rs["merged"][r], rs["kept"][r],
                                                             rs["kernel_ms"][r]))
    del off_d, adj_d
    spc.release_cached_memory()
    torch.cuda.empty_cache()
    nq = args.queries
    # the tuner times every launch configuration on a batch of the timed
    # batch's size (another seed): the grouping of a large batch by staged
    # label changes which configuration is fastest
    ts, tt = inputs.queries(g.n, nq, seed=3)
    qcfg = ix.tune_queries(ts, tt, stream=stream)
    log(f"query autotuner: configuration {qcfg} {spc.query_configs()[qcfg]}")
    s_np, t_np = inputs.queries(g.n, nq, seed=2)
    s_d = torch.from_numpy(s_np.view(np.int32)).to(dev)
    t_d = torch.from_numpy(t_np.view(np.int32)).to(dev)
    dist_o = torch.empty(nq, dtype=torch.uint8 if ix.dist_bits == 8 else torch.int16, device=dev)
    cnt_o = torch.empty(nq, dtype=torch.int64, device=dev)
    flg_o = torch.empty(nq, dtype=torch.uint8, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    qms = []
    for i in range(args.warmup + args.steps):
        ev0.record(stream)
        ix.query(s_d, t_d, stream=stream, out=(dist_o, cnt_o, flg_o))
        ev1.record(stream)
        torch.cuda.synchronize()
        if i >= args.warmup:
            qms.append(ev0.elapsed_time(ev1))
    query_ms = float(np.mean(qms))
    log(f"{args.steps} query steps: {query_ms:.1f} ms per 10M-query batch")

    # served: saturation (a burst), then Poisson arrivals at 1.0x of it
    mean_batch = 65536 / np.log(65537) - 0.5
    srv_kw = dict(io_budget_bytes=1 << 30, streams=4, max_batch=1 << 18)
    burst = serve.requests_from(inputs.poisson_requests(g.n, 1e9, args.serve_requests, seed=6))
    for r in burst:
        r.arrival = 0.0
    srv = serve.Server(ix, **srv_kw)
    srv.run(burst[:20])  # warm the streams and pinned host buffers
    serve.fifo_baseline(ix, burst[:20])
    sat = srv.run(burst).summary()
    rate = sat["queries_per_s"] / mean_batch
    reqs = serve.requests_from(inputs.poisson_requests(g.n, rate, args.serve_requests, seed=107))
    served = srv.run(reqs).summary()
    fifo = serve.fifo_baseline(ix, reqs).summary()
    log(f"served 1.0x: {served['queries_per_s']:.3g} q/s p50 {served['p50_ms']:.2f} ms p99 "
        f"{served['p99_ms']:.2f} ms | fifo p50 {fifo['p50_ms']:.2f} p99 {fifo['p99_ms']:.2f}")
    ix.free()
    spc.release_cached_memory()

    # rooflines: the round kernel (the build's dominant kernel) and the query kernel
    rk = _roofline("k_round", st["alg_bytes_round_kernel"], st["ms_round_kernel"],
                   st["round_kernel_launches"],
                   "kernel-counted: pulled entries (12 B), u's label entries staged, landmark "
                   "masks or row slices read, filter words looked up, label entries the probe "
                   "searches read, label offsets, survivors written; the oracle cannot rebuild "
                   "this index, so the byte model from the definitions is reported for the same "
                   "kernel on the Chung-Lu side line",
                   traffic=measured_traffic("k_round_rmat21"))
    qb = _profile_json("oracle_bytes_k_query_rmat21.json")
    q_roof = None
    if qb and qb.get("n") == g.n and qb.get("m") == g.m:
        q_roof = _roofline("k_query", qb["mean_bytes"] * nq, query_ms, 1,
                           "oracle: (|L(s)|+|L(t)|)(4+delta) + 16 k* + 8 + (delta+8+1) per query, "
                           f"mean over {qb['queries']} sampled pairs of the query stream "
                           f"(standard error {qb['stderr_bytes']:.0f} B)",
                           traffic=measured_traffic("k_query_rmat21", "query.hip"),
                           bytes_per_query=qb["mean_bytes"])
    out = {
        "metric": METRIC,
        "value": st["entries"] / (build_ms * 1e-3),
        "unit": "label entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": query_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {scale}, edge factor 16, a,b,c,d = 0.57,0.19,0.19,0.05, "
                               f"seed 5, degree order: one index build (value; after one untimed "
                               f"warmup build when warmup > 0), then steps of {nq} "
                               "uniform SPC queries on the resident index, then Poisson requests "
                               "at 1.0x saturation (p50/p99)",
                   "step": f"one batch of {nq} uniform queries on the resident index "
                           "(the build is timed once, before the steps)",
                   "n": g.n, "m": g.m, "entries": st["entries"], "rounds": st["rounds"],
                   "max_dist": st["max_dist"], "queries": nq, "parallelism": "single-gpu"},
        "build_ms": build_ms,
        "warmup_build_ms": first_ms,
        "build_entries_per_s": st["entries"] / (build_ms * 1e-3),
        "queries_per_s": nq / (query_ms * 1e-3),
        "query_ms": query_ms,
        "p50_ms": served["p50_ms"],
        "p99_ms": served["p99_ms"],
        "served_1x": {"queries_per_s": served["queries_per_s"], "p50_ms": served["p50_ms"],
                      "p99_ms": served["p99_ms"], "requests": served["requests"],
                      "deferred": served["deferred"], "launches": served["launches"],
                      "offered_queries_per_s": sat["queries_per_s"],
                      "fifo_queries_per_s": fifo["queries_per_s"], "fifo_p50_ms": fifo["p50_ms"],
                      "fifo_p99_ms": fifo["p99_ms"], "saturation_queries_per_s": sat["queries_per_s"]},
        "query_config": dict(zip(("stage", "tiles"), spc.query_configs()[qcfg])),
        "build_breakdown_ms": {"order": st["ms_order"], "rounds": st["ms_rounds"],
                               "finalize": st["ms_finalize"], "device_total": st["ms_total"],
                               "round_kernel": st["ms_round_kernel"]},
        "round_kernel_launches": st["round_kernel_launches"],
        "rounds": {k: rs[k] for k in ("raw", "merged", "kept", "kernel_ms")},
        "roofline": rk,
        "query_roofline": q_roof,
        "index_bytes": st["index_bytes"],
        "peak_build_bytes": st["peak_build_bytes"],
    }
    if not args.no_side:
        log("side line: Chung-Lu n=2^20")
        out["chunglu"] = bench_chunglu(args, dev, log, steps=2, warmup=1, side=True)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baselines(g, log)
    if args.scale_down:
        out["note"] = "scaled-down smoke run, not the benchmark workload"
    print(json.dumps(out), flush=True)


def bench_chunglu(args, dev, log, steps, warmup, side=False):
    """Chung-Lu n = 2^20 (power law 2.1 clipped to [2, 20000], mean degree
    10, seed 2), degree order: each step builds the index and answers 10M
    uniform queries.  Returns the JSON object (its roofline uses the oracle's
    byte model of the build when profiles/ holds it)."""
    import numpy as np
    import torch

    from paper_2212_00977_amd import inputs, spc

    log("generating Chung-Lu graph")
    g = inputs.workload("chunglu", scale_down=args.scale_down)
    nq = args.queries
    s_np, t_np = inputs.queries(g.n, nq, seed=2)
    off_d = torch.from_numpy(g.off.view(np.int64)).to(dev)
    adj_d = torch.from_numpy(g.adj.view(np.int32)).to(dev)
    s_d = torch.from_numpy(s_np.view(np.int32)).to(dev)
    t_d = torch.from_numpy(t_np.view(np.int32)).to(dev)
    dist_o = torch.empty(nq, dtype=torch.uint8, device=dev)
    cnt_o = torch.empty(nq, dtype=torch.int64, device=dev)
    flg_o = torch.empty(nq, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts_np, tt_np = inputs.queries(g.n, nq, seed=3)
    torch.cuda.synchronize()
    qcfg = [None]
    bopts = spc.BuildOptions(propagation=args.propagation)

    def step(keep=False):
        t0 = time.perf_counter()
        ix = spc.build_index(off_d, adj_d, device=dev, stream=stream, opts=bopts)
        t1 = time.perf_counter()
        ix.set_query_config(qcfg[0])
        if ix.dist_bits != 8:
            raise RuntimeError("Chung-Lu index with 16-bit outputs: outputs sized for 8 bits")
        ev0.record(stream)
        ix.query(s_d, t_d, stream=stream, out=(dist_o, cnt_o, flg_o))
        ev1.record(stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = ix.stats()
        st["_rounds"] = {k: v.tolist() for k, v in {**ix.round_stats(), **ix.round_profile()}.items()}
        if not keep:
            ix.free()
            ix = None
        return dict(build_ms=(t1 - t0) * 1e3, query_ms=ev0.elapsed_time(ev1),
                    step_ms=(t2 - t0) * 1e3, stats=st, index=ix)

    # query autotuner, before any timed work: one build, every launch
    # configuration timed on a separate sample
    ix = spc.build_index(off_d, adj_d, device=dev, stream=stream)
    qcfg[0] = ix.tune_queries(ts_np, tt_np, stream=stream)
    ix.free()
    log(f"query autotuner: configuration {qcfg[0]} {spc.query_configs()[qcfg[0]]}")
    for i in range(warmup):
        r = step()
        log(f"warmup {i}: build {r['build_ms']:.1f} ms, query {r['query_ms']:.1f} ms, "
            f"entries {r['stats']['entries']}")
    torch.cuda.synchronize()
    runs = []
    tt0 = time.perf_counter()
    for i in range(steps):
        r = step(keep=(i == steps - 1))
        runs.append(r)
        log(f"step {i}: build {r['build_ms']:.1f} ms, query {r['query_ms']:.1f} ms")
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - tt0) * 1e3

    st = runs[-1]["stats"]
    rs = st["_rounds"]
    for r in range(len(rs["kept"])):
        log("round %d: raw %d merged %d kept %d tail %d staged %d rowB %d hdr %d  %.1f ms" % (
            r, rs["raw"][r], rs["merged"][r], rs["kept"][r], rs["scanned"][r], rs["staged"][r],
            rs["row_bytes"][r], rs["headers"][r], rs["kernel_ms"][r]))
    entries = st["entries"]
    build_ms = float(np.mean([r["build_ms"] for r in runs]))
    query_ms = float(np.mean([r["query_ms"] for r in runs]))
    rk_ms = float(np.mean([r["stats"]["ms_round_kernel"] for r in runs]))
    launches = st["round_kernel_launches"]
    traffic = measured_traffic("k_round_chunglu_n2e20")
    kc = _roofline("k_round", st["alg_bytes_round_kernel"], rk_ms, launches,
                   "kernel-counted (the kernel's own count of what it must read and write)",
                   traffic=traffic)
    prof = _profile_json("oracle_bytes_k_round_chunglu_n2e20.json")
    defn = None
    if prof and prof.get("n") == g.n and prof.get("m") == g.m and prof.get("entries") == entries:
        # the byte model written from the definitions (its probes consume the
        # candidate's label in hub order: 80-95% of its bytes); the kernel's
        # membership filter and landmark masks skip most of those bytes, so
        # this is an effective rate, not a bandwidth, and may exceed the peak
        b_rk = _s8d_round_kernel_bytes(prof)
        m = _roofline("k_round", b_rk, rk_ms, launches, "definitions")
        defn = {"round_kernel_bytes": b_rk, "round_kernel_effective_GBps": m["achieved"],
                "round_kernel_effective_frac": m["frac"], "build_bytes": prof["total"],
                "build_effective_GBps": prof["total"] / (build_ms * 1e-3) / 1e9,
                "build_effective_frac": prof["total"] / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "bytes_model": "oracle byte model (B_csr + B_expand + B_stage + B_probe + B_write, "
                               "from the oracle's threaded PULL build; round kernel: rounds 2..)",
                "note": "bytes the definitions' merge-join probes read, over the measured time: "
                        "an effective rate (the kernel skips most of them), not a bandwidth"}
    qb = _profile_json("oracle_bytes_k_query_chunglu_n2e20.json")
    q_roof = None
    if qb and qb.get("n") == g.n and qb.get("m") == g.m:
        q_roof = _roofline("k_query", qb["mean_bytes"] * nq, query_ms, 1,
                           f"oracle: B_q, mean over {qb['queries']} sampled pairs of the query stream",
                           bytes_per_query=qb["mean_bytes"])
    out = {
        "metric": METRIC,
        "value": entries / (build_ms * 1e-3),
        "unit": "label entries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": total_ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"chung-lu n=2^{20 - args.scale_down} exp 2.1 clip [2,20000] "
                               f"mean deg 10 seed 2, degree order, {args.propagation} propagation, "
                               f"{nq} uniform queries",
                   "n": g.n, "m": g.m, "entries": entries, "rounds": st["rounds"],
                   "max_dist": st["max_dist"], "queries": nq, "parallelism": "single-gpu"},
        "build_ms": build_ms,
        "query_ms": query_ms,
        "query_config": dict(zip(("stage", "tiles"), spc.query_configs()[qcfg[0]])),
        "queries_per_s": nq / (query_ms * 1e-3),
        "build_breakdown_ms": {"order": st["ms_order"], "rounds": st["ms_rounds"],
                               "finalize": st["ms_finalize"], "device_total": st["ms_total"],
                               "round_kernel": rk_ms},
        "roofline": kc,
        "definition_byte_model": defn,
        "query_roofline": q_roof,
        "index_bytes": st["index_bytes"],
        "peak_build_bytes": st["peak_build_bytes"],
    }
    last_ix = runs[-1]["index"]
    if not side and not args.no_reductions:
        for kind in ("one_shell", "equivalence"):
            out[kind] = reduced_side(kind, off_d, adj_d, s_d, t_d, dev, stream, qcfg[0], dist_o, cnt_o, log)
    if not side and (args.serve_seconds > 0 or args.serve_sweep):
        out["serve"] = serve_runs(last_ix, g.n, args, out["queries_per_s"], log)
    last_ix.free()
    if not side and not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
    if side:
        for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            out.pop(k)
    del off_d, adj_d, s_d, t_d, dist_o, cnt_o, flg_o
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=10_000_000)
    ap.add_argument("--scale-down", type=int, default=0,
                    help="shrink n by 2^k (smoke runs only; not the benchmark workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="default line: skip the Chung-Lu side line")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="chunglu: length of the served-load run on the last index (0 = skip)")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="chunglu: after the steps, sweep the offered load (0.25..1.25 x saturation) "
                         "and print one JSON line per level")
    ap.add_argument("--workload", default="rmat21",
                    choices=["rmat21", "chunglu", "rmat_batch", "rmat_served", "grid"],
                    help="rmat21: the benchmark line; chunglu: the Chung-Lu build line alone; "
                         "rmat_batch: 512 R-MAT graphs built as one batch vs one build per graph; "
                         "rmat_served: offered-load sweep on a resident R-MAT scale-21 index; "
                         "grid: k x k grid with a round cap (separate JSON lines)")
    ap.add_argument("--grid-k", type=int, default=2048, help="grid side (grid workload)")
    ap.add_argument("--round-cap", type=int, default=64,
                    help="round cap D for the grid workload (0 = complete index)")
    ap.add_argument("--order", default="degree", choices=["degree", "hybrid", "td"],
                    help="vertex order of the grid workload: degree (random ties), hybrid "
                         "(--delta), td (tree decomposition: no degree bound)")
    ap.add_argument("--delta", type=int, default=5, help="hybrid order degree threshold")
    ap.add_argument("--serve-max-batch", type=int, default=1 << 18,
                    help="queries per coalesced launch (rmat_served)")
    ap.add_argument("--serve-streams", type=int, default=4, help="streams of the server (rmat_served)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per offered-load level (rmat21, rmat_served)")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--no-reductions", action="store_true",
                    help="skip the side measurements of the reduced builds")
    ap.add_argument("--one-shell", action="store_true",
                    help="build with the 1-shell reduction (rmat_served, rmat_batch)")
    ap.add_argument("--propagation", default="pull", choices=["pull", "push", "auto"],
                    help="propagation paradigm of the chunglu workload's timed builds")
    ap.add_argument("--equivalence", action="store_true",
                    help="build with the neighbourhood-equivalence reduction (rmat_served, rmat_batch)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU "
                                   "sharding of the build is a design note, not built"}))
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)  # noqa: E731

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": args.copy_calibration, "copies": 3}))
        return

    if args.workload == "rmat_batch":
        return bench_batch(args, dev, log)
    if args.workload == "rmat_served":
        return bench_served(args, dev, log)
    if args.workload == "grid":
        return bench_grid(args, dev, log)
    if args.workload == "chunglu":
        out = bench_chunglu(args, dev, log, args.steps, args.warmup)
        if args.scale_down:
            out["note"] = "scaled-down smoke run, not the benchmark workload"
        print(json.dumps(out), flush=True)
        return
    return bench_rmat21(args, dev, log)


if __name__ == "__main__":
    main()
