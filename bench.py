"""Benchmark of the RS scoring pass on one MI355X.

One step = one full scoring pass (rs_score: border detection, interaction
matrix, weights, w_max, type-II aggregate, Eq. RSI scores) plus rs_topk(K) on a
graph already resident in HBM.  Prints ONE JSON line (rank 0, N=1).

  python bench.py [--steps K] [--warmup W] [--workload lfr_20m|lfr_1m|sbm_2k|batch|served|robustness]
                  [--no-cpu-baseline] [--copy-calibration]

--workload batch scores many small graphs as one batch (one pass over their
disjoint union, per-graph w_max and top-k) and times the same graphs scored
one by one as separate resident graphs beside it; --workload served drives the
request server.

--copy-calibration runs only a plain device copy of known size, for scaling the
FETCH_SIZE / WRITE_SIZE counters of rocprofv3 runs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RS-scored edges/sec on 1 MI355X (% HBM roofline); p50/p99 re-score latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "sbm_2k": ("SBM n=2,000, 20 communities of 100, p_in=0.05, p_out=0.001, seed 0", 20),
    "lfr_1m": ("LFR-style n=1,000,000, degree exponent 2.5 mean 20 max 5,000, community sizes "
               "exponent 1.5 on [50, 20,000], mixing 0.1, seed 0", 1000),
    "lfr_20m": ("LFR-style n=20,000,000, mean degree 30, max 100,000, mixing 0.15, seed 0", 10000),
    "batch": ("graphs g = 0..G-1 (seed 1000+g): n log-uniform on [200, 50,000], mean degree U[8, 40], "
              "U{5..500} communities (at most n/10), mixing U[0.05, 0.3], SBM or LFR-style (max degree "
              "min(1,000, n/4)) with probability 1/2; scored as one batch, per-graph w_max and top-20", 20),
    "robustness": ("LFR-style n=100,000, mean degree 20, max 1,000, community sizes on [50, 5,000], mixing 0.1, "
                   "seed 0; 5% of the edges (or vertices) removed per step up to 75%", 25),
    "served": ("resident LFR-style graphs (seeds 5000+g), n log-uniform on [1e5, nmax], mean degree 20, "
               "max 5,000, mixing 0.1; Poisson removal requests, each followed by a top-100 query", 100),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_graph(name):
    """The workload's seeded graph (cached in $RS_GRAPH_CACHE when that is set)."""
    from rsgen import cached, cfg_lfr_1m, cfg_lfr_20m, cfg_sbm_small
    if name == "sbm_2k":
        return cfg_sbm_small(0)
    make = {"lfr_1m": cfg_lfr_1m, "lfr_20m": cfg_lfr_20m}[name]
    return cached(f"{name}_seed0", lambda: make(0, log=log), log=log)


def kernel_bytes(c, n, nnz, s_off, k_top):
    """Algorithmic bytes of one pass (B_alg): every array the method must move,
    each element once, attributed to the kernel that moves it.  Reading G and
    the labels, and writing the interaction-matrix rows (community, count),
    their weights, the own weights / a_v and G', belong to the row kernel;
    reading those back, the type-II aggregates S_w(c) (write + read), the
    intersection lists (4 bytes per step of W1 = sum over G' edges of
    min(d'(u), d'(w))) and writing R belong to the score kernel; top-k reads R
    and writes K (id, score) pairs."""
    ell, ellx, nx, w1 = c["sum_ell"], c["sum_ell_x"], 2 * c["m_inter"], c["sum_work_I"]
    rows = ((n + 1) * s_off + 4 * nnz + 4 * n                # G and labels
            + 8 * ell + 8 * (n + 1)                          # rows (community, count) + row pointer
            + 8 * ell + 8 * n                                # weights, own weight / a_v
            + 4 * nx + s_off * (n + 1))                      # G'
    score = (8 * ell + 8 * (n + 1) + 8 * ell + 8 * n + 4 * nx + s_off * (n + 1)   # read back
             + 2 * 8 * ellx                                  # S_w(c) write + read
             + 4 * w1                                        # intersections
             + 8 * n)                                        # R
    topk = 8 * n + 12 * k_top
    return {"k_rows": rows, "k_score": score, "topk": topk, "pass": rows + score + topk}


KERNEL_SRC = os.path.join(ROOT, "paper_2508_01485_amd", "csrc", "rs_kernels.hip")


def kernel_source_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by what the same counter
    reads for a plain device copy of known size), or None when there is none
    or the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("<!-- traffic "):
                rec = json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
    if not rec or rec.get("source_sha") != kernel_source_sha():
        return None
    k = rec["kernels"].get(kernel)
    if not k:
        return None
    fetch = k["fetch_kib"] * 1024.0 * rec["copy_bytes"] / (rec["copy_fetch_kib"] * 1024.0)
    write = k["write_kib"] * 1024.0 * rec["copy_bytes"] / (rec["copy_write_kib"] * 1024.0)
    return fetch + write


def copy_calibration():
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_copy_gbs(nbytes=1 << 30, reps=10):
    """Achievable device bandwidth: a plain device-to-device copy of nbytes
    (read + write counted), best of reps, timed with HIP events."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (best * 1e-3) / 1e9


def cpu_baseline(g, k_top, budget_s=12.0, targets=None, cores=None):
    import oracle
    if cores is None:
        try:
            cores = len(os.sched_getaffinity(0))
        except AttributeError:
            cores = os.cpu_count() or 1
        cores = min(cores, 16)
    if g.nnz > 100_000_000:
        return cpu_baseline_sampled(g, k_top, cores)
    alive, what = None, "full workload graph"
    if targets:
        g, alive = oracle.restrict_to_targets(g, targets)
        what = f"workload graph restricted to its {targets} largest communities"
    m = int(g.off[-1]) // 2
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        o = oracle.score(g, nthreads=cores)
        oracle.topk(o["R"], k_top, alive=alive)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end or len(times) >= 50:
            break
    t = float(np.median(times))
    return {"value": m / t, "unit": "edges/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}, {len(times)} repeats of score + top-{k_top}, median {t:.3f} s "
                      f"({cores} threads of {cpu_model()})"}


def cpu_baseline_sampled(g, k_top, cores, s1=20_000, s2=60_000):
    """The oracle on a graph too large to score whole within the bench: it
    builds every row (all weights, w_max) and scores two random vertex samples
    of sizes s1 and s2; the whole job is extrapolated as
    t(s1) + (t(s2) - t(s1)) / (s2 - s1) * (n - s1), plus the top-k time."""
    import oracle
    rng = np.random.default_rng(7)
    perm = rng.permutation(g.n)
    t = {}
    for s in (s1, s2):
        sub = np.sort(perm[:s])
        t0 = time.perf_counter()
        o = oracle.score(g, subset=sub, nthreads=cores)
        t[s] = time.perf_counter() - t0
        log(f"oracle on {s} sampled vertices: {t[s]:.1f}s")
    t0 = time.perf_counter()
    oracle.topk(o["R"], k_top)
    t_top = time.perf_counter() - t0
    per_vertex = max(t[s2] - t[s1], 0.0) / (s2 - s1)
    t_full = t[s1] + per_vertex * (g.n - s1) + t_top
    return {"value": g.m / t_full, "unit": "edges/s", "cores": cores, "kind": "oracle",
            "sample": (f"all rows and weights plus Eq. RSI for random samples of {s1} and {s2} vertices "
                       f"({t[s1]:.1f}s, {t[s2]:.1f}s), extrapolated linearly to all {g.n} vertices "
                       f"({t_full:.1f}s) plus top-{k_top}")}


def rescore_latency(rs, h, g, n_req, seed=11):
    """Re-score latency on the resident graph: a stream of removal requests,
    each either 1-1,000 random existing edges or 1-50 vertices drawn from the
    current top-1,000 (half each), applied with rs_apply_removals (validation,
    upload, incremental re-score) and followed by a top-100 query; the wall
    time of both is one request's latency.  Beside it, the plain baseline: a
    full recompute (rs_score + rs_topk(100)) of the same mutated graph right
    after each request, whose top-100 must be bit-identical to the
    incremental one.  Runs after the timed steps (it mutates the graph)."""
    rng = np.random.default_rng(seed)
    u, v = g.edges()
    alive = np.ones(u.size, bool)
    lat, full, aff = [], [], []
    same = True
    for _ in range(n_req):
        if rng.random() < 0.5:
            live = np.flatnonzero(alive)
            k = min(int(rng.integers(1, 1001)), live.size)
            pick = rng.choice(live, k, replace=False)
            alive[pick] = False
            kw = {"edges": np.stack([u[pick], v[pick]], 1)}
        else:
            ids, _ = rs.rs_topk(h, 1000)
            k = min(int(rng.integers(1, 51)), ids.size)
            kw = {"vertices": rng.choice(ids, k, replace=False)}
        t0 = time.perf_counter()
        res = rs.rs_apply_removals(h, **kw)
        i1, s1 = rs.rs_topk(h, 100)
        lat.append(time.perf_counter() - t0)
        aff.append(res["affected"])
        t0 = time.perf_counter()
        rs.rs_score(h)
        i2, s2 = rs.rs_topk(h, 100)
        full.append(time.perf_counter() - t0)
        same &= np.array_equal(i1, i2) and s1.tobytes() == s2.tobytes()
    pct = lambda x, q: 1000 * float(np.percentile(x, q))  # noqa: E731
    return {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": 1000 * float(np.mean(lat)), "requests": n_req,
            "mean_affected": float(np.mean(aff)),
            "full_recompute_ms": {"p50": pct(full, 50), "p99": pct(full, 99)},
            "speedup_p50": float(np.percentile(full, 50) / np.percentile(lat, 50)),
            "top100_identical": bool(same),
            "request": "half: 1-1,000 random existing edges; half: 1-50 vertices of the current top-1,000; "
                       "then a top-100 query; baseline: rs_score + rs_topk(100) of the same mutated graph"}


def _served_graph(args):
    gi, n = args
    from rsgen import cached, lfr
    return cached(f"served_{gi}_n{n}", lambda: lfr(int(n), 20.0, 5000, 0.1, 5000 + gi))


def bench_served(args):
    """The served form: several graphs behind rs_server, removal requests
    (half 1-1,000 random existing edges, half 1-50 vertices of the graph's
    latest top-100), each followed by a top-100 query.  Two phases, each on a
    fresh server: every graph resident (budget above the whole footprint),
    then an HBM budget of half the footprint (admission, eviction, reloads).
    Per phase: capacity = requests/s with all requests queued at once; then
    Poisson arrivals at 0.5, 0.8 and 1.0 times that rate, latency =
    completion - arrival (and service = completion - start) per request,
    also split into requests that reloaded an evicted graph and the rest.
    Beside them, the plain baseline: the same graphs resident on their own
    handles and each request of the resident phase's capacity mix answered
    by a full pass (rs_score) plus rs_topk(100) of its graph, one request
    after another; `value` is the resident phase's capacity."""
    import threading
    from concurrent.futures import ProcessPoolExecutor

    rng = np.random.default_rng(5000)
    ns = np.exp(rng.uniform(np.log(1e5), np.log(args.served_nmax), args.served_graphs)).astype(np.int64)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        graphs = list(ex.map(_served_graph, list(enumerate(ns.tolist()))))
    log(f"generated {len(graphs)} graphs (n={sum(g.n for g in graphs)}) in {time.perf_counter() - t0:.1f}s")
    import paper_2508_01485_amd as rs  # after the generator pool: no forked process has loaded the HIP library
    est = sum(48 * g.nnz + 360 * g.n + (8 << 20) for g in graphs)
    edges = [g.edges() for g in graphs]
    alive = [np.ones(e[0].size, bool) for e in edges]
    tops = [None] * len(graphs)
    lock = threading.Lock()
    picked = []

    def make_request(gi=None):
        gi = int(rng.integers(len(graphs))) if gi is None else gi
        picked.append(gi)
        u, v = edges[gi]
        with lock:
            top = tops[gi]
        if rng.random() < 0.5 or top is None or top.size == 0:
            # up to k random live edges: random indices, the live ones kept
            # (no scan of the whole liveness array per request)
            k = int(rng.integers(1, 1001))
            cand = np.unique(rng.integers(0, u.size, 2 * k + 16))
            cand = cand[alive[gi][cand]]
            pick = rng.permutation(cand)[:k]
            alive[gi][pick] = False
            return gi, {"edges": np.stack([u[pick], v[pick]], 1)}
        return gi, {"vertices": rng.choice(top, min(int(rng.integers(1, 51)), top.size), replace=False)}

    def pct(x):
        return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))} if len(x) else None

    def run(srv, gids, n_req, rate, order=None):
        """Submit n_req requests (all at once if rate is None, else Poisson;
        on the graphs of `order` in turn when given, else on random graphs),
        waiting for them in a second thread; returns per-request info.  The
        requests are drawn before the clock starts (vertex removals from
        each graph's latest top-100 known then)."""
        rids = []
        done = []
        cv = threading.Condition()

        def waiter():
            i = 0
            while True:
                with cv:
                    while i >= len(rids) and len(rids) < n_req:
                        cv.wait()
                    if i >= len(rids):
                        return
                    rid, gi = rids[i]
                i += 1
                ids, sc, info = srv.wait(rid)
                with lock:
                    tops[gi] = ids
                done.append(info)

        todo = [make_request(None if order is None else order[q]) for q in range(n_req)]
        gaps = [float(rng.exponential(1.0 / rate)) for _ in range(n_req)] if rate else None
        th = threading.Thread(target=waiter)
        th.start()
        t_begin = time.perf_counter()
        for q in range(n_req):
            if rate:
                time.sleep(gaps[q])
            gi, kw = todo[q]
            rid = srv.submit(gids[gi], 100, **kw)
            with cv:
                rids.append((rid, gi))
                cv.notify()
        th.join()
        wall = time.perf_counter() - t_begin
        lat = np.array([(d["t_done"] - d["t_submit"]) / 1e6 for d in done])
        svc = np.array([(d["t_done"] - d["t_start"]) / 1e6 for d in done])
        reload = np.array([bool(d["loaded"]) for d in done])
        return {"requests": n_req, "wall_s": wall, "requests_per_s": n_req / wall,
                "latency_ms": pct(lat), "service_ms": pct(svc),
                "latency_ms_without_reloads": pct(lat[~reload]), "latency_ms_reloads": pct(lat[reload]),
                "mean_affected": float(np.mean([d["affected"] for d in done])),
                "reloads": int(reload.sum())}

    def phase(budget):
        """A fresh server under `budget`: warm-up (every graph loaded), then
        capacity and the three Poisson rates."""
        srv = rs.RSServer(slots=args.served_slots, hbm_budget=budget)
        gids = [srv.add_graph(g.off, g.col, g.labels) for g in graphs]
        log(f"budget {budget / 2**30:.1f} GiB: warm-up (every graph loaded, one request each)")
        run(srv, gids, len(graphs), None, order=list(range(len(graphs))))
        n0 = len(picked)
        cap = run(srv, gids, args.served_requests, None)
        mix = picked[n0:]
        mu = cap["requests_per_s"]
        rates = {}
        for f in (0.5, 0.8, 1.0):
            log(f"Poisson arrivals at {f} x capacity ({f * mu:.0f}/s)")
            rates[str(f)] = run(srv, gids, args.served_requests, f * mu)
        st = srv.stats()
        srv.free()
        return {"hbm_budget_bytes": int(budget), "capacity": cap, "poisson": rates, "server": st}, mix

    # every graph resident (a budget above the whole footprint): the served
    # form against the plain baseline on the same request mix
    resident, mix = phase(int(est * 1.25))
    # half the footprint: admission, eviction and reloads
    budgeted, _ = phase(est // 2)
    log("plain baseline: a full pass per request")
    plain_ms = []
    for g in graphs:
        h = rs.rs_load_graph(g.off, g.col, g.labels)
        rs.rs_score(h)
        rs.rs_topk(h, 100)
        ts = []
        for _ in range(5):
            t1 = time.perf_counter()
            rs.rs_score(h)
            rs.rs_topk(h, 100)
            ts.append(time.perf_counter() - t1)
        h.free()
        plain_ms.append(1000.0 * float(np.median(ts)))
    per_req = np.asarray(plain_ms)[np.asarray(mix, np.int64)]
    plain_rps = 1000.0 / float(per_req.mean())
    mu = resident["capacity"]["requests_per_s"]
    m_total = sum(g.m for g in graphs)
    out = {
        "metric": METRIC, "value": mu, "unit": "requests/s", "n_gpus": 1, "steps": args.served_requests,
        "warmup": len(graphs), "ms_per_step": 1000.0 / mu, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"served: {len(graphs)} {WORKLOADS['served'][0]}".replace("nmax", f"{args.served_nmax:.0e}"),
                   "graphs": len(graphs), "n_total": int(sum(g.n for g in graphs)), "m_total": int(m_total),
                   "n_max": int(max(g.n for g in graphs)), "slots": args.served_slots,
                   "footprint_estimate_bytes": int(est), "top_k": 100},
        "resident": resident,
        "budget_half": budgeted,
        "plain_baseline": {"what": "every graph resident on its own handle; each request of the resident run's "
                                   "capacity mix answered by rs_score + rs_topk(100) of its graph, one after "
                                   "another (the removal itself not counted)",
                           "requests_per_s": plain_rps, "service_ms": pct(per_req),
                           "served_speedup": mu / plain_rps},
    }
    print(json.dumps(out), flush=True)


def batch_arrays(n_graphs):
    """The batched workload packed as one disjoint union (vertex offsets, row
    offsets, columns, labels) and its statistics; cached in $RS_GRAPH_CACHE
    when that is set, so a later run (e.g. under a profiler) starts no
    generator workers."""
    from rsgen import Graph, cached, cfg_batch, pack_batch

    def make():
        graphs = cfg_batch(n_graphs, workers=min(16, os.cpu_count() or 1))
        vo, off, col, lab = pack_batch(graphs)
        deg = [g.nnz / max(g.n, 1) for g in graphs]
        meta = {"vertex_offsets": [int(x) for x in vo], "n_max": int(max(g.n for g in graphs)),
                "mean_degree_range": [round(min(deg), 2), round(max(deg), 2)],
                "sbm_graphs": int(sum(g.meta["kind"] == "sbm" for g in graphs))}
        return Graph(int(vo[-1]), off, col, lab, meta=meta)

    g = cached(f"batch_{n_graphs}", make, log=log)
    return np.asarray(g.meta["vertex_offsets"], np.int64), g.off, g.col, g.labels, g.meta


def graph_of_batch(vo, off, col, lab, i):
    """Graph i of a packed batch, with ids relative to the graph."""
    a, b = int(vo[i]), int(vo[i + 1])
    e0, e1 = int(off[a]), int(off[b])
    return off[a:b + 1] - e0, col[e0:e1] - np.int32(a), lab[a:b]


def bench_batch(args):
    """The batched form: G graphs packed into one disjoint union and scored by
    one pass (rs_score + rs_topk_batch(20)), first with the default schedule,
    then with the cut-offs the autotuner picks for the batch's degree
    signature (searched on a cache miss, then served from the cache); beside
    it the same graphs loaded as G separate resident graphs, each scored by
    rs_score + rs_topk(20) in turn.  Every per-graph top-20 is compared:
    tuned against untuned, and batch against one by one."""
    import tempfile

    import torch

    import paper_2508_01485_amd as rs
    from paper_2508_01485_amd import autotune
    K = WORKLOADS["batch"][1]
    t0 = time.perf_counter()
    vo, off, col, lab, meta = batch_arrays(args.batch_graphs)
    G = vo.size - 1
    n_tot, m_tot = int(vo[-1]), int(off[-1]) // 2
    log(f"{G} graphs (n={n_tot}, m={m_tot}) ready in {time.perf_counter() - t0:.1f}s")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    h = rs.rs_load_batch(vo, off, col, lab, stream=stream)
    load_s = time.perf_counter() - t0
    log(f"batch loaded in {load_s:.2f}s")

    def timed():
        for _ in range(args.warmup):
            rs.rs_score(h)
            rs.rs_topk_batch(h, K)
        lat = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            rs.rs_score(h)
            top = rs.rs_topk_batch(h, K)  # waits for the stream
            lat.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t_start) / args.steps
        rs.rs_set_timing(h, True)
        rs.rs_read_timings(h)
        for _ in range(args.steps):
            rs.rs_score(h)
            rs.rs_topk_batch(h, K)
        torch.cuda.synchronize()
        tm = rs.rs_read_timings(h)
        rs.rs_set_timing(h, False)
        return t, lat, top, tm

    t_untuned, _, top_u, _ = timed()
    log(f"untuned {1000 * t_untuned:.2f} ms per step; tuning")
    cache_path = args.tune_cache or os.path.join(tempfile.mkdtemp(), "tiling.json")
    tune = autotune.tune(h, off, n_graphs=G, cache_path=cache_path)
    log(f"tuned: {tune}")
    t_batch, lat, (bids, bsc, bcnt), timings = timed()
    tuned_same = bool(np.array_equal(bids, top_u[0]) and np.array_equal(bcnt, top_u[2]))
    tuned_rel = float(np.max(np.abs(bsc - top_u[1]) / np.maximum(np.maximum(np.abs(bsc), np.abs(top_u[1])), 1e-300)))
    again = autotune.tune(h, off, n_graphs=G, cache_path=cache_path)  # the same signature: from the cache
    rs.rs_score(h)
    counts = rs.rs_read_counts(h)
    rs.rs_free_graph(h)
    log("kernel ms/launch:", {k: round(v[0] / v[1], 4) for k, v in timings.items() if v[1]})

    def avg(name):
        ms, nl = timings.get(name, (0.0, 0))
        return 1000.0 * ms / nl if nl else 0.0
    kb = kernel_bytes(counts, n_tot, 2 * m_tot, 8, K * G)
    avg_us = {"k_rows": avg("k_rows"),
              "k_score": avg("k_hub_filters") + avg("k_score") + avg("k_score_hub") + avg("k_hub_sum")}
    dom = max(avg_us, key=avg_us.get)
    achieved = kb[dom] / (avg_us[dom] * 1e-6) / 1e9
    out = {
        "metric": METRIC, "value": m_tot / t_batch, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * t_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch: {G} {WORKLOADS['batch'][0]}", "graphs": G,
                   "n_total": n_tot, "m_total": m_tot, "n_max": meta["n_max"],
                   "mean_degree_range": meta["mean_degree_range"], "sbm_graphs": meta["sbm_graphs"], "top_k": K},
        "latency_ms": {"p50": 1000 * float(np.percentile(lat, 50)), "p90": 1000 * float(np.percentile(lat, 90))},
        "load_s": load_s,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": kb[dom],
                     "avg_us": avg_us[dom]},
        "kernels_us": {k: round(1000.0 * v[0] / v[1], 3) for k, v in timings.items() if v[1]},
        "autotune": {"untuned_ms_per_step": 1000.0 * t_untuned, "tuned_ms_per_step": 1000.0 * t_batch,
                     "speedup": t_untuned / t_batch, "tiling": tune["tiling"], "default": autotune.DEFAULT,
                     "signature": tune["signature"], "search_s": round(tune["seconds"], 2),
                     "candidates_timed": tune.get("candidates_timed"), "cache_hit_after": again["cached"],
                     "cache_hit_s": round(again["seconds"], 3), "top20_ids_identical_to_untuned": tuned_same,
                     "top20_max_rel_diff_to_untuned": tuned_rel},
    }
    if args.batch_sweeps > 0:  # the same graphs one by one
        log("loading the graphs one by one")
        t0 = time.perf_counter()
        hs = []
        for i in range(G):
            o, c, lb = graph_of_batch(vo, off, col, lab, i)
            hs.append(rs.rs_load_graph(o, c, lb, stream=stream))
        log(f"{len(hs)} graphs loaded in {time.perf_counter() - t0:.1f}s")
        for x in hs:  # warm-up sweep
            rs.rs_score(x)
            rs.rs_topk(x, K)
        seq = []
        same, rel = True, 0.0
        for rep_i in range(args.batch_sweeps):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            tops = []
            for x in hs:
                rs.rs_score(x)
                tops.append(rs.rs_topk(x, K))
            torch.cuda.synchronize()
            seq.append(time.perf_counter() - s0)
            if rep_i == 0:
                for i, (ids, sc) in enumerate(tops):
                    c = int(bcnt[i])
                    same &= c == ids.size and np.array_equal(bids[i, :c], ids)
                    if c and c == ids.size:
                        rel = max(rel, float(np.max(np.abs(bsc[i, :c] - sc) / np.maximum(np.abs(sc), 1e-300))))
        for x in hs:
            x.free()
        t_seq = float(np.median(seq))
        out["one_by_one"] = {"ms_per_sweep": 1000.0 * t_seq, "edges_per_s": m_tot / t_seq,
                             "batch_speedup": t_seq / t_batch, "batch_speedup_untuned": t_seq / t_untuned,
                             "top20_ids_identical": bool(same), "top20_max_rel_diff": rel}
    print(json.dumps(out), flush=True)


def bench_robustness(args):
    """The robustness workload (absolute AWCC, Section VII-B): the top-25 RS
    vertices of the intact graph against 25 random border vertices; 5% of
    the original edges (or vertices) removed per step, up to 75%; after each
    step the absolute AWCC of both sets, mean over v of |zeta(v)| / d0(v)
    with d0 the intact degree, for two readings of zeta(v): the communities
    reachable by paths in the disrupted graph (rs_reachable_communities) and
    those of v's remaining neighbours (the row length ell).  Each step's
    removal (with the incremental re-score) and reach query are timed."""
    import torch

    import paper_2508_01485_amd as rs
    from rsgen import lfr
    n = args.robust_n
    g = lfr(n, 20.0, 1000, 0.1, 0, cmin=50, cmax=5000)
    log(f"graph n={g.n} m={g.m}")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    u, v = g.edges()
    d0 = np.diff(g.off).astype(np.float64)
    curves, t_rem, t_reach = {}, [], []
    for mode in ("edges", "vertices"):
        rng = np.random.default_rng(11 if mode == "edges" else 12)
        h = rs.rs_load_graph(g.off, g.col, g.labels, stream=stream)
        rs.rs_score(h)
        s_rs, _ = rs.rs_topk(h, 25)
        border = np.flatnonzero(rs.rs_read_vertex_counts(h)["border"])
        s_rand = rng.choice(border, 25, replace=False)
        src = np.concatenate([s_rs, s_rand]).astype(np.int32)
        order = rng.permutation(u.size if mode == "edges" else g.n)
        per = (u.size if mode == "edges" else g.n) // 20
        cur = {"removed_pct": [], "rs_paths": [], "random_paths": [], "rs_neighbours": [], "random_neighbours": []}
        for step in range(16):
            if step:
                pick = order[(step - 1) * per: step * per]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "edges":
                    rs.rs_apply_removals(h, edges=np.stack([u[pick], v[pick]], 1))
                else:
                    rs.rs_apply_removals(h, vertices=pick)
                t_rem.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            reach = rs.rs_reachable_communities(h, src)
            t_reach.append(time.perf_counter() - t0)
            ell = rs.rs_read_vertex_counts(h)["ell"][src]
            a_reach = reach / d0[src]
            a_hop = ell / d0[src]
            cur["removed_pct"].append(5 * step)
            cur["rs_paths"].append(round(float(a_reach[:25].mean()), 5))
            cur["random_paths"].append(round(float(a_reach[25:].mean()), 5))
            cur["rs_neighbours"].append(round(float(a_hop[:25].mean()), 5))
            cur["random_neighbours"].append(round(float(a_hop[25:].mean()), 5))
        h.free()
        curves[mode] = cur
        log(mode, cur)
    ms_step = 1000.0 * (float(np.mean(t_rem)) + float(np.mean(t_reach)))
    out = {
        "metric": METRIC, "value": 1000.0 / ms_step, "unit": "disruption steps/s", "n_gpus": 1,
        "steps": len(t_rem), "warmup": 0, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"robustness: {WORKLOADS['robustness'][0]}", "n": g.n, "m": g.m, "sets": 25},
        "removal_ms": {"p50": 1000 * float(np.percentile(t_rem, 50)), "p99": 1000 * float(np.percentile(t_rem, 99))},
        "reach_ms": {"p50": 1000 * float(np.percentile(t_reach, 50)), "p99": 1000 * float(np.percentile(t_reach, 99))},
        "absolute_awcc": curves,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lfr_20m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--targets", type=int, default=0,
                    help="target-community mode: score only the K largest communities (0: all)")
    ap.add_argument("--robust-n", type=int, default=100_000)
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-sweeps", type=int, default=3)
    ap.add_argument("--tune-cache", default="",
                    help="autotuner cache file for the batch workload (default: a fresh temporary file)")
    ap.add_argument("--served-graphs", type=int, default=64)
    ap.add_argument("--served-nmax", type=float, default=5e6)
    ap.add_argument("--served-slots", type=int, default=4)
    ap.add_argument("--served-requests", type=int, default=300)
    ap.add_argument("--rescore-requests", type=int, default=None,
                    help="removal requests timed after the steps (0: skip; default 200, 20 above 1e8 entries)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library scores one resident graph per device and "
              "has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    if args.workload == "served":
        bench_served(args)
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "robustness":
        bench_robustness(args)
        return

    import torch

    import paper_2508_01485_amd as rs

    desc, k_top = WORKLOADS[args.workload]
    log("generating", args.workload)
    t0 = time.perf_counter()
    g = make_graph(args.workload)
    log(f"generated n={g.n} m={g.m} in {time.perf_counter() - t0:.1f}s")

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    h = rs.rs_load_graph(g.off, g.col, g.labels, stream=stream)
    load_s = time.perf_counter() - t0
    log(f"loaded in {load_s:.2f}s")
    m_scored = g.m
    if args.targets:
        res = rs.rs_restrict_to_targets(h, args.targets)
        m_scored = g.m - res["edges_removed"]
        log(f"restricted to the {args.targets} largest communities: {m_scored} edges, "
            f"{g.n - res['vertices_removed']} vertices")

    for _ in range(args.warmup):
        rs.rs_score(h)
        rs.rs_topk(h, k_top)
    torch.cuda.synchronize()

    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        rs.rs_score(h)
        ids, sc = rs.rs_topk(h, k_top)  # waits for the stream
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    # per-kernel durations: the same steps again with HIP events recorded by
    # the library around every launch on the graph's stream (eager launches;
    # the timed steps above replay captured HIP graphs)
    rs.rs_set_timing(h, True)
    rs.rs_read_timings(h)  # reset
    for _ in range(args.steps):
        rs.rs_score(h)
        rs.rs_topk(h, k_top)
    torch.cuda.synchronize()
    timings = rs.rs_read_timings(h)
    rs.rs_set_timing(h, False)
    counts = rs.rs_read_counts(h)
    log("kernel ms/launch:", {k: round(v[0] / v[1], 4) for k, v in timings.items() if v[1]})

    ms_per_step = 1000.0 * t_total / args.steps
    value = m_scored / (t_total / args.steps)
    s_off = 8 if g.nnz > 2**31 - 1 else 4
    kb = kernel_bytes(counts, g.n, g.nnz, s_off, k_top)
    def avg(name):
        ms, nl = timings.get(name, (0.0, 0))
        return 1000.0 * ms / nl if nl else 0.0

    avg_us = {"k_rows": avg("k_rows"),
              "k_score": avg("k_hub_filters") + avg("k_score") + avg("k_score_hub") + avg("k_hub_sum")}
    dom = max(avg_us, key=avg_us.get)
    achieved = kb[dom] / (avg_us[dom] * 1e-6) / 1e9
    gpu_ms = sum(v[0] for v in timings.values()) / args.steps
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {desc}",
            "n": g.n, "m": g.m, "nnz": g.nnz, "communities": int(counts["n_communities"]),
            "mean_degree": round(g.nnz / max(g.n, 1), 3), "max_degree": int(np.diff(g.off).max()),
            "mu_realized": round(2 * counts["m_inter"] / max(g.nnz, 1), 4), "top_k": k_top,
            "row_offsets": f"int{8 * s_off}",
        },
        "latency_ms": {"p50": 1000 * float(np.percentile(lat, 50)), "p10": 1000 * float(np.percentile(lat, 10)),
                       "p90": 1000 * float(np.percentile(lat, 90)), "p99": 1000 * float(np.percentile(lat, 99))},
        "load_s": load_s,
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            # the counters were taken on the whole graph; target mode scores another one
            "traffic": measured_traffic(args.workload, dom) if not args.targets else None,
            "bytes_per_launch": kb[dom], "avg_us": avg_us[dom],
        },
        "kernels_us": {k: round(1000.0 * v[0] / v[1], 3) for k, v in timings.items() if v[1]},
        "pass": {"alg_bytes": kb["pass"], "gpu_ms_per_step": gpu_ms,
                 "alg_GBs": kb["pass"] / (gpu_ms * 1e-3) / 1e9 if gpu_ms else None},
        "counts": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in counts.items()},
    }
    if args.targets:
        c = out["config"]
        c["workload"] += f"; target-community mode: the {args.targets} largest communities only"
        c["target_communities"] = args.targets
        c["m_scored"] = int(m_scored)
        c["mu_realized"] = round(counts["m_inter"] / max(m_scored, 1), 4)
    copy_gbs = measured_copy_gbs()
    out["roofline"]["copy_GBs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = achieved / copy_gbs
    n_req = args.rescore_requests if args.rescore_requests is not None else (200 if g.nnz < 100_000_000 else 20)
    if n_req > 0:
        log(f"timing {n_req} removal + incremental re-score requests")
        out["rescore_latency_ms"] = rescore_latency(rs, h, g, n_req)
    rs.rs_free_graph(h)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(g, k_top, targets=args.targets)
        if g.nnz <= 100_000_000:
            log("timing the CPU oracle on one core")
            out["cpu_baseline_1core"] = cpu_baseline(g, k_top, budget_s=8.0, targets=args.targets, cores=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
