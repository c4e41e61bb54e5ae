#!/usr/bin/env python3
"""Benchmark of the Stop-and-Stare hot path on one MI355X.

Default workload (--workload twitter-ic-dssa), the largest single-GPU
configuration: the Twitter-shaped Chung-Lu graph (41.7M nodes, 1.47B edges,
out- and in-degree exponent 2.0, reverse CSR of about 12 GB resident in
HBM), IC weighted cascade; each step is three full D-SSA queries
(Algorithm 4: RR-set sampling, incidence, greedy max-coverage, stare step,
FP64 checkpoint logic) with k = 1, 100 and 1000, eps = 0.1, delta = 1/n and
stream key = step index.

Other workloads (one JSON line each, same fields):
  rmat20-lt-dssa  R-MAT scale-20 graph (1,048,576 nodes, 16M draws with
                  a,b,c = 0.57, 0.19, 0.19, self-loops and repeats dropped),
                  LT model with uniform(0,1) in-weights normalised to sum 1
                  per node; each step is one D-SSA query, k = 100.
  pokec-ic-ssa64  Pokec-shaped Chung-Lu graph (4.8M nodes, 69M edges,
                  exponent 2.3), IC trivalency; each step is 64 concurrent
                  SSA queries (k log-uniform in [1, 500], eps in
                  {0.05, 0.1, 0.2}, delta = 1/n, key = query index) through
                  the multi-query engine, all sampling fused per pass.
  serving         Poisson stream of queries over the resident NetHEPT-,
                  R-MAT-20- and Pokec-shaped graphs through the request loop
                  (continuous batching, admission by RR-pool bytes).

Inputs are resident in HBM before the timed region. Prints one JSON line:
RR sets/s over the timed steps (whole job), edges traversed/s, query latency
p50/p99, the sampler kernel's roofline (event-timed live on the library's
stream) and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
METRIC = "RR sets/s + edges traversed/s vs HBM roofline; IM-query p50/p99 latency"


def lt_bytes(steps: int, sets: int) -> int:
    """Algorithmic bytes of LT sampling: per walk step 16 B of offsets, 8 B
    for the two bracketing thresholds, 4 B src, 4 B visited check, 4 B pool
    write; 8 B per set offset."""
    return 36 * steps + 8 * sets


def ic_bytes(steps: int, nodes: int, sets: int, edge_bytes: int = 8) -> int:
    """Algorithmic bytes of IC sampling: per visited node 16 B of offsets and
    4 B pool write, 8 B per in-edge examined ({src, threshold}), about 4 B of
    visited check per newly reached node; 8 B per set offset. With
    edge_bytes=4: the same count for the compact form of a graph whose
    in-edges of each node share one threshold (16 B node record, 4 B src)."""
    return 16 * nodes + edge_bytes * steps + 4 * max(nodes - sets, 0) + 4 * nodes + 8 * sets


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def measured_traffic(kernel: str, steps: int | None = None, warmup: int | None = None):
    """HBM bytes per timed launch of `kernel` (for the IC sampler: its wave
    pass and both workgroup tiers) from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (scaled by a plain copy of known size), or None when the
    kernel's sources, or the query loop that sizes its launches, changed
    since the counters were taken, or when the record names the bench's
    --steps / --warmup (which fix the launches averaged) and this run's
    differ."""
    import hashlib

    path = ROOT / "profiles" / "traffic.json"
    if not path.exists():
        return None
    rec = json.loads(path.read_text()).get(kernel)
    if rec is None:
        return None
    if ("steps" in rec and rec["steps"] != steps) or ("warmup" in rec and rec["warmup"] != warmup):
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update((ROOT / src).read_bytes())
    return rec["hbm_bytes_per_dispatch"] if h.hexdigest() == rec["source_sha256"] else None


GATHER_SHAPES = {}


def gather_bandwidth(segs=(32, 64, 128, 256, 512), buffer_bytes: int = 16 << 30, trials: int = 3,
                     record: str = "") -> dict:
    """Measured random-gather bandwidth (GB/s of segment bytes) per segment
    size, from the probe library: hashed random segment-aligned reads of a
    buffer (by default far larger than the 256 MB last-level cache), in two
    access shapes (a lane per segment; the lanes of a wave splitting
    segments 16 bytes each, eight in flight per lane). The faster shape is
    the roofline; both curves are kept in GATHER_SHAPES[record]."""
    import ctypes

    lib = ctypes.CDLL(str(ROOT / "paper_1605_07990_amd" / "libimprobe.so"))
    lib.im_probe_gather_shape.restype = ctypes.c_int
    lib.im_probe_gather_shape.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    out, shapes = {}, {"lane": {}, "coop": {}}
    for seg in segs:
        for shape, name in ((0, "lane"), (1, "coop")):
            g = ctypes.c_double(0.0)
            if lib.im_probe_gather_shape(0, buffer_bytes, seg, trials, shape, ctypes.byref(g)) != 0:
                raise RuntimeError(f"gather probe failed for {seg}-byte segments ({name})")
            shapes[name][seg] = round(g.value, 1)
        out[seg] = max(shapes["lane"][seg], shapes["coop"][seg])
    if record:
        GATHER_SHAPES[record] = shapes
    return out


def roofline(kt: dict, model: int, traffic_measured_here: bool = False, traffic_key: str = "",
             steps: int | None = None, warmup: int | None = None, compact: bool = False) -> dict:
    """Roofline of the main sampler kernel from its event timing: algorithmic
    bytes per launch over the mean launch duration, against HBM peak.
    `traffic` (HBM bytes per launch from the committed counter runs) is
    reported only for the configuration those runs measured, since bytes
    per launch follow the launch size."""
    launches = max(kt["sample_launches"], 1)
    if model == 1:
        total = lt_bytes(kt["sample_steps"], kt["sample_sets"])
        name = "lt_main_kernel (LT RR-set sampler)"
    else:
        total = ic_bytes(kt["sample_steps"], kt["sample_nodes"], kt["sample_sets"])
        name = "ic_main_kernel + ic_group_kernel (IC RR-set sampler: wave pass and workgroup tier)"
    bytes_per_launch = total / launches
    ms_per_launch = kt["sample_ms"] / launches
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9 if ms_per_launch > 0 else 0.0
    sec = kt["sample_ms"] * 1e-3
    key = traffic_key or ("lt_main_kernel" if model == 1 else "ic_sampler")
    traffic = measured_traffic(key, steps, warmup) if traffic_measured_here else None
    out = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "launches": kt["sample_launches"],
            "avg_launch_ms": round(ms_per_launch, 5), "algorithmic_bytes_per_launch": round(bytes_per_launch),
           "sampler_sets_per_s": round(kt["sample_sets"] / sec) if sec else None,
           "sampler_steps_per_s": round(kt["sample_steps"] / sec) if sec else None}
    if model == 0 and compact:
        # the sampler read the compact form (4 B per in-edge, the threshold
        # once per node): the same rate counted in the bytes it needs
        cb = ic_bytes(kt["sample_steps"], kt["sample_nodes"], kt["sample_sets"], edge_bytes=4) / launches
        ca = cb / (ms_per_launch * 1e-3) / 1e9 if ms_per_launch > 0 else 0.0
        out["compact_form"] = {"algorithmic_bytes_per_launch": round(cb), "achieved": round(ca, 2),
                               "frac": round(ca / HBM_PEAK_GBS, 5)}
    if model == 0 and kt.get("group_launches"):
        out["workgroup_tier"] = {"ms_per_launch": round(kt["group_ms"] / kt["group_launches"], 5),
                                 "samples": kt["group_samples"], "edges": kt["group_edges"],
                                 "mean_levels": round(kt["group_levels"] / max(kt["group_samples"], 1), 2)}
    if GATHER:
        # segment size of one gather: an LT step reads an 8-record threshold
        # window (64 B); an IC node its in-list (mean length x 8 B)
        if model == 1:
            seg = 64
        else:
            mean = 8.0 * kt["sample_steps"] / max(kt["sample_nodes"], 1)
            seg = min(GATHER, key=lambda x: abs(math.log2(x) - math.log2(max(mean, 1.0))))
        out["gather_gbs"] = GATHER
        out["gather_gbs_by_shape"] = GATHER_SHAPES.get("hbm")
        out["gather_segment_bytes"] = seg
        out["gather_frac"] = round(achieved / GATHER[seg], 5)
        if seg in GATHER_MALL:
            # the same probe on a buffer the last-level cache holds, the
            # roofline of graphs that fit there (R-MAT-20: 143 MB)
            out["gather_cache_resident_gbs"] = GATHER_MALL[seg]
            out["gather_cache_resident_frac"] = round(achieved / GATHER_MALL[seg], 5)
    return out


GATHER = {}
GATHER_MALL = {}


def log_uniform_k(rng, hi: int, n: int) -> int:
    return int(min(n, max(1, round(math.exp(rng.uniform(0.0, math.log(hi)))))))


def pokec_queries(n: int, count: int = 64, seed: int = 64):
    """The 64-query mix: k = round(exp(U(0, ln 500))), eps uniform over
    {0.05, 0.1, 0.2}, key = query index."""
    import numpy as np

    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        k = log_uniform_k(rng, 500, n)
        eps = float((0.05, 0.1, 0.2)[int(rng.integers(3))])
        out.append((k, eps, q))
    return out


# ----------------------------------------------------------- workloads ----

def run_engine_batch(im, ctx, dg, model, algo, queries, budget, max_active):
    """Run `queries` [(k, eps, delta, key)] concurrently through one engine;
    returns per-query (seeds, stats) and latency from submission in ms."""
    eng = im.Engine(ctx, pool_budget_bytes=budget, max_active=max_active)
    t_sub = time.perf_counter()
    tickets = [eng.submit(dg, model, algo, k, eps, delta, key) for k, eps, delta, key in queries]
    done = {}
    while len(done) < len(tickets):
        eng.step()
        now = time.perf_counter()
        for t in tickets:
            if t not in done and eng.poll(t) != 0:
                done[t] = (now - t_sub) * 1e3
    res = [eng.result(t) for t in tickets]
    eng.close()
    return res, [done[t] for t in tickets]


def run_rmat20(args, im, ctx, sync):
    import synth

    g = synth.make("rmat20")
    n, k, eps = g.n, args.k, args.eps
    delta = 1.0 / n
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_lt=g.w_lt)
    B = args.queries_per_step
    budget = int(args.pool_budget_gb * (1 << 30))

    def step(i):
        if B == 1:
            q0 = time.perf_counter()
            _, st = dg.dssa(im.IM_LT, k, eps, delta, i)
            return [st], [(time.perf_counter() - q0) * 1e3]
        res, lat_ = run_engine_batch(im, ctx, dg, im.IM_LT, "dssa", [(k, eps, delta, i * B + j) for j in range(B)],
                                     budget, B)
        return [st for _, st in res], lat_

    for i in range(args.warmup):
        step(1_000_000 + i)
    ctx.set_timing(True)
    ctx.read_timing(reset=True)
    sync()
    lat, sets, edges, iters = [], 0, 0, []
    stage = {"ms_sample": 0.0, "ms_cover": 0.0, "ms_verify": 0.0}
    t0 = time.perf_counter()
    for i in range(args.steps):
        sts, l_ = step(i)
        lat += l_
        for st in sts:
            sets += st["n_sets"]
            edges += st["edges"]
            iters.append(st["iterations"])
            for key in stage:
                stage[key] += st[key] / B
    sync()
    dt = time.perf_counter() - t0
    kt = ctx.read_timing(reset=True)
    ctx.set_timing(False)
    dg.close()
    out = {"value": round(sets / dt, 1), "ms_per_step": round(dt * 1e3 / args.steps, 4),
           "config": {"workload": "R-MAT-20 LT D-SSA", "n": n, "m": g.m, "k": k, "eps": eps, "delta": "1/n",
                      "queries_per_step": B},
           "edges_per_s": round(edges / dt, 1), "p50_ms": round(percentile(lat, 50), 3),
           "p99_ms": round(percentile(lat, 99), 3), "rr_sets_per_query": sets // max(args.steps * B, 1),
           "iterations_per_query": sorted(set(iters)),
           "stage_ms_per_query": {k_: round(v_ / args.steps, 3) for k_, v_ in stage.items()},
           "roofline": roofline(kt, 1, traffic_measured_here=(B == 1 and not args.param and not args.no_speculate
                                                               and args.greedy_wg_max_entries is None))}

    def cpu(budget_s):
        import oracle

        og = oracle.Graph(oracle.LT, g.n, g.src, g.dst, g.w_lt)
        s_ = e_ = q = 0
        t = time.perf_counter()
        while True:
            _, ost = og.dssa(k, eps, delta, q)
            s_ += ost["n_sets"]
            e_ += ost["edges"]
            q += 1
            if time.perf_counter() - t >= budget_s:
                break
        d = time.perf_counter() - t
        return {"value": s_ / d, "unit": "RR sets/s", "cores": 1, "kind": "oracle", "edges_per_s": e_ / d,
                "sample": f"{q} sequential oracle D-SSA queries (k={k}, eps={eps}, delta=1/n, keys 0..{q - 1}) "
                          f"on the same graph, {d:.1f} s on one host core"}

    return out, cpu


def run_pokec64(args, im, ctx, sync):
    import synth

    g = synth.make("pokec")
    n = g.n
    delta = 1.0 / n
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    qs = pokec_queries(n)
    budget = int(args.pool_budget_gb * (1 << 30))

    def one_batch(key_base):
        return run_engine_batch(im, ctx, dg, im.IM_IC, "ssa", [(k, eps, delta, key_base + key) for k, eps, key in qs],
                                budget, 64)

    for i in range(args.warmup):
        one_batch(1_000_000 * (i + 1))
    ctx.set_timing(True)
    ctx.read_timing(reset=True)
    sync()
    lat, sets, edges = [], 0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, l_ = one_batch(0)
        lat += l_
        for _, st in res:
            sets += st["n_sets"] + st["n_verify"]
            edges += st["edges"]
    sync()
    dt = time.perf_counter() - t0
    kt = ctx.read_timing(reset=True)
    ctx.set_timing(False)
    out = {"value": round(sets / dt, 1), "ms_per_step": round(dt * 1e3 / args.steps, 4),
           "config": {"workload": "Pokec-shaped IC trivalency, 64 concurrent SSA queries", "n": n, "m": g.m,
                      "k": "log-uniform [1,500]", "eps": [0.05, 0.1, 0.2], "delta": "1/n", "queries_per_step": 64},
           "edges_per_s": round(edges / dt, 1), "p50_ms": round(percentile(lat, 50), 3),
           "p99_ms": round(percentile(lat, 99), 3), "rr_sets_per_step": sets // max(args.steps, 1),
           "roofline": roofline(kt, 0, compact=bool(dg.info()[2] & 4) and ctx.get_param("ic_compact") == 1)}
    if args.compare_plain:
        # the same 64 queries one after another through im_ssa
        sync()
        p0 = time.perf_counter()
        psets = 0
        for k, eps, key in qs:
            _, st = dg.ssa(im.IM_IC, k, eps, delta, key)
            psets += st["n_sets"] + st["n_verify"]
        sync()
        pdt = time.perf_counter() - p0
        out["one_query_at_a_time"] = {"ms": round(pdt * 1e3, 3), "rr_sets_per_s": round(psets / pdt, 1),
                                      "engine_speedup": round(pdt / (dt / args.steps), 3)}
    dg.close()

    def cpu(budget_s):
        import oracle

        og = oracle.Graph(oracle.IC, g.n, g.src, g.dst, g.w_ic)
        pool = oracle.Pool(og, 0)
        c = 0
        t = time.perf_counter()
        chunk = 20000
        while time.perf_counter() - t < budget_s:
            c += chunk
            pool.extend(c)
        d = time.perf_counter() - t
        return {"value": c / d, "unit": "RR sets/s", "cores": 1, "kind": "oracle",
                "sample": f"oracle RR-set sampling of samples 0..{c - 1} of query 0's stream on the same graph "
                          f"({d:.1f} s, one host core); sampling only, no greedy"}

    return out, cpu


def run_serving(args, im, ctx, sync):
    import synth
    from paper_1605_07990_amd import serve

    graphs, shapes = {}, {}
    for name in ("nethept", "rmat20", "pokec"):
        g = synth.make(name)
        graphs[name] = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic, w_lt=g.w_lt)
        shapes[name] = (g.n, g.w_ic is not None, g.w_lt is not None)
    budget = int(args.pool_budget_gb * (1 << 30))
    if args.warmup:
        eng = im.Engine(ctx, pool_budget_bytes=budget, max_active=args.max_active)
        serve.serve(eng, graphs, serve.poisson_requests(shapes, args.qps, max(8, args.warmup), seed=999,
                                                        algo=None, key_base=1 << 40))
        eng.close()
    reqs = serve.poisson_requests(shapes, args.qps, args.queries, seed=args.seed, algo=None)
    eng = im.Engine(ctx, pool_budget_bytes=budget, max_active=args.max_active)
    ctx.set_timing(True)
    ctx.read_timing(reset=True)
    sync()
    last = [0.0]

    def progress(done, total, active):
        now = time.perf_counter()
        if now - last[0] > 5.0 or done == total:
            last[0] = now
            print(f"[serve] {done}/{total} done, {active} active", file=sys.stderr, flush=True)

    r = serve.serve(eng, graphs, reqs, progress=progress)
    sync()
    kt = ctx.read_timing(reset=True)
    ctx.set_timing(False)
    eng.close()
    for dg in graphs.values():
        dg.close()
    out = {"value": round(r["rr_sets_per_s"], 1), "ms_per_step": round(r["wall_s"] * 1e3, 3),
           "config": {"workload": "serving: Poisson stream over NetHEPT-, R-MAT-20-, Pokec-shaped graphs",
                      "qps": args.qps, "queries": args.queries, "k": "log-uniform [1,1000]",
                      "eps": [0.05, 0.1, 0.2], "model": "IC or LT 50/50", "algo": "SSA or D-SSA 50/50",
                      "pool_budget_gb": args.pool_budget_gb, "max_active": args.max_active},
           "edges_per_s": round(r["edges_per_s"], 1), "p50_ms": round(r["p50_ms"], 3),
           "p99_ms": round(r["p99_ms"], 3), "achieved_qps": round(r["achieved_qps"], 3),
           "offered_qps": round(r["offered_qps"], 3), "engine_steps": r["engine_steps"],
           "max_active": r["max_active"], "slowest": r["slowest"], "roofline": None,
           "roofline_note": "none: the stream mixes IC and LT queries on three graphs, two of them cache-resident, "
                            "so no single kernel or byte model applies; see the per-workload bench lines"}
    return out, None


def run_twitter(args, im, ctx, sync):
    import synth

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t_gen = time.perf_counter()
    g = synth.make("twitter", cache=os.environ.get("IM_CACHE_BIG", "") == "1")
    t_gen = time.perf_counter() - t_gen
    progress(f"graph n={g.n} m={g.m} generated in {t_gen:.1f} s")
    n = g.n
    delta = 1.0 / n
    t_load = time.perf_counter()
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    sync()
    t_load = time.perf_counter() - t_load
    progress(f"graph loaded in {t_load:.1f} s")
    ks = args.ks or [1, 100, 1000]
    for i in range(args.warmup):
        dg.dssa(im.IM_IC, 100, 0.1, delta, 1_000_000 + i)
    ctx.set_timing(True)
    ctx.read_timing(reset=True)
    sync()
    lat, sets, edges, per_k = [], 0, 0, {}
    budget = int(args.pool_budget_gb * (1 << 30))
    t0 = time.perf_counter()
    for step in range(args.steps):
        if args.engine:
            res, l_ = run_engine_batch(im, ctx, dg, im.IM_IC, "dssa", [(k, 0.1, delta, step) for k in ks], budget,
                                       len(ks))
            lat += l_
            for k, (_, st), ms in zip(ks, res, l_):
                progress(f"step {step} k={k}: {ms:.1f} ms (engine), {st['n_sets']} sets")
                sets += st["n_sets"]
                edges += st["edges"]
                per_k.setdefault(k, []).append({"ms": round(ms, 3), "n_sets": st["n_sets"], "edges": st["edges"],
                                                "iterations": st["iterations"]})
            continue
        for k in ks:
            q0 = time.perf_counter()
            _, st = dg.dssa(im.IM_IC, k, 0.1, delta, step)
            ms = (time.perf_counter() - q0) * 1e3
            progress(f"step {step} k={k}: {ms:.1f} ms, {st['n_sets']} sets, {st['iterations']} iterations")
            lat.append(ms)
            sets += st["n_sets"]
            edges += st["edges"]
            per_k.setdefault(k, []).append({"ms": round(ms, 3), "n_sets": st["n_sets"], "edges": st["edges"],
                                            "iterations": st["iterations"],
                                            "ms_sample": round(st["ms_sample"], 3),
                                            "ms_cover": round(st["ms_cover"], 3)})
    sync()
    dt = time.perf_counter() - t0
    kt = ctx.read_timing(reset=True)
    ctx.set_timing(False)
    out = {"value": round(sets / dt, 1), "ms_per_step": round(dt * 1e3 / args.steps, 4),
           "config": {"workload": "Twitter-shaped IC weighted cascade D-SSA, k in {1, 100, 1000}", "n": n,
                      "m": g.m, "k": ks, "eps": 0.1, "delta": "1/n", "queries_per_step": len(ks)},
           "edges_per_s": round(edges / dt, 1), "p50_ms": round(percentile(lat, 50), 3),
           "p99_ms": round(percentile(lat, 99), 3), "per_k": per_k,
           "graph_generate_s": round(t_gen, 1), "graph_load_s": round(t_load, 2),
           "roofline": roofline(kt, 0, traffic_measured_here=(not args.engine and args.ks is None and not args.param
                                                              and not args.no_speculate
                                                              and args.greedy_wg_max_entries is None),
                                traffic_key="ic_sampler_twitter", steps=args.steps, warmup=args.warmup,
                                compact=bool(dg.info()[2] & 4) and ctx.get_param("ic_compact") == 1)}
    if args.engine:
        out["config"]["workload"] += ", concurrent through the engine"
    if not args.no_batching_compare:
        out["batching"] = batching_compare(im, ctx, dg, sync, progress)
        out["greedy_roofline"] = greedy_roofline(im, dg, sync, progress)
    if args.compare_plain:
        # the same step-0 queries one after another through im_dssa
        sync()
        p0 = time.perf_counter()
        psets = 0
        for k in ks:
            _, st = dg.dssa(im.IM_IC, k, 0.1, delta, 0)
            psets += st["n_sets"]
        sync()
        pdt = time.perf_counter() - p0
        out["one_query_at_a_time"] = {"ms": round(pdt * 1e3, 3), "rr_sets_per_s": round(psets / pdt, 1),
                                      "speedup_of_this_run": round(pdt / (dt / args.steps), 3)}
    dg.close()

    def cpu(budget_s):
        return oracle_sampling_baseline(g, budget_s)

    return out, cpu


def greedy_roofline(im, dg, sync, progress, sets: int = 72_672, ks=(100, 1000)) -> dict:
    """Max-Coverage (Algorithm 2: the node-to-set incidence, then k greedy
    rounds; im_max_coverage_range) over a pool of `sets` RR sets (key 0; the
    default is the greedy range N_t of the last iteration of a k = 100 D-SSA
    run on the Twitter-shaped graph),
    host wall time around synchronised calls, best of two per k, against
    the HBM stream peak with the streaming bytes of the method: the
    incidence's three passes of 4 B per pool entry plus 8 B per node, and
    4 B per pool entry of marginal-count decrements (the argmax's own bytes
    depend on the schedule and are not counted)."""
    pool = im.Pool(dg, im.IM_IC, 0)
    pool.sample(sets)
    sync()
    count, entries = pool.info()
    n = dg.n
    algo_bytes = 16 * entries + 8 * n
    out = {"kernel": "incidence + greedy rounds (im_max_coverage_range)", "pool_sets": count,
           "pool_entries": entries, "algorithmic_bytes": algo_bytes, "peak_gbs": HBM_PEAK_GBS, "by_k": {}}
    for k in ks:
        best = None
        for _ in range(2):
            sync()
            t = time.perf_counter()
            pool.max_coverage(k)
            sync()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        gbs = algo_bytes / best / 1e9
        out["by_k"][str(k)] = {"ms": round(best * 1e3, 3), "achieved_gbs": round(gbs, 2),
                               "frac": round(gbs / HBM_PEAK_GBS, 5)}
        progress(f"greedy k={k} over {count} sets: {best * 1e3:.2f} ms, {gbs:.1f} GB/s")
    pool.close()
    return out


def batching_compare(im, ctx, dg, sync, progress, queries: int = 8, per_query: int = 145_344) -> dict:
    """The batched persistent IC sampler against one launch per query, on
    the same RR sets: `queries` pools (keys 0..queries-1), each drawing
    `per_query` sets (a k = 100 D-SSA run's 2 N_t at its stop on this graph).
      fused   one im_sample_rr_multi call: every pool's samples in one device
              work queue (tickets), heavy samples moved to workgroup tiers;
      per_query  one im_sample_rr per pool, same kernels;
      plain   one im_sample_rr per pool with IM_PARAM_IC_PLAIN: static
              assignment of samples to waves, no tiers (samples that outgrow
              a wave's LDS go to the one-wave-per-sample long path).
    Host wall time of each (the calls synchronise), best of two; the three
    must leave identical pools (offsets and per-set node sums checked)."""
    import numpy as np

    def run(mode):
        best, sig = None, None
        for rep in range(2):
            pools = [im.Pool(dg, im.IM_IC, q) for q in range(queries)]
            ctx.set_param("ic_plain", 1 if mode == "plain" else 0)
            sync()
            t = time.perf_counter()
            if mode == "fused":
                im.Pool.sample_multi(pools, [per_query] * queries)
            else:
                for p_ in pools:
                    p_.sample(per_query)
            sync()
            dt = time.perf_counter() - t
            ctx.set_param("ic_plain", 0)
            best = dt if best is None else min(best, dt)
            if rep == 0:
                sig = []
                for p_ in pools:
                    off, nodes = p_.read()
                    sums = np.add.reduceat(nodes.astype(np.uint64), off[:-1].astype(np.int64)) if nodes.size else 0
                    sig.append((off.tobytes(), np.asarray(sums).tobytes()))
            del pools
        progress(f"batching comparison: {mode} {best * 1e3:.1f} ms")
        return best, sig

    t_fused, s_fused = run("fused")
    t_pq, s_pq = run("per_query")
    t_plain, s_plain = run("plain")
    sets = queries * per_query
    return {"workload": f"{queries} IC pools on the Twitter-shaped graph (keys 0..{queries - 1}), {per_query} RR sets "
                        f"each (a k=100 D-SSA run's 2 N_t at its stop)",
            "sets": sets, "fused_ms": round(t_fused * 1e3, 3), "per_query_ms": round(t_pq * 1e3, 3),
            "plain_ms": round(t_plain * 1e3, 3), "fused_sets_per_s": round(sets / t_fused),
            "plain_sets_per_s": round(sets / t_plain),
            "speedup_vs_plain": round(t_plain / t_fused, 3), "speedup_vs_per_query": round(t_pq / t_fused, 3),
            "identical_pools": s_fused == s_pq == s_plain}


def host_threads() -> int:
    """Host threads for the multi-core oracle: the cores this process may
    run on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_sampling_baseline(g, budget_s: float) -> dict:
    """The oracle's RR-set sampling on the host (IC, key 0, the same graph):
    the first 2^16 samples on one core (sequential, as the oracle draws
    them), then the samples after them on every host thread (contiguous
    sample blocks per thread, the same sets), sized to take about half the
    budget each. Sampling only: the oracle's greedy over 41.7M nodes is a
    linear argmax per round."""
    import oracle

    og = oracle.Graph(oracle.IC, g.n, g.src, g.dst, g.w_ic)
    pool = oracle.Pool(og, 0)
    c = 0
    t = time.perf_counter()
    while time.perf_counter() - t < budget_s / 2 and c < (1 << 16):
        c += 4096
        pool.extend(c)
    d1 = time.perf_counter() - t
    e1 = pool.edges
    one = {"value": c / d1, "edges_per_s": e1 / d1, "cores": 1, "samples": c, "seconds": round(d1, 2)}
    threads = host_threads()
    rate = c / d1
    more = int(min(1 << 22, max(4096, rate * threads * budget_s / 2)))
    t = time.perf_counter()
    pool.extend(c + more, threads=threads)
    dm = time.perf_counter() - t
    multi = {"value": more / dm, "edges_per_s": (pool.edges - e1) / dm, "cores": threads, "samples": more,
             "seconds": round(dm, 2)}
    return {"value": multi["value"], "unit": "RR sets/s", "cores": threads, "kind": "oracle",
            "edges_per_s": multi["edges_per_s"], "single_core": one,
            "sample": f"oracle RR-set sampling of key 0 on the same graph, sampling only: samples 0..{c - 1} on one "
                      f"core ({d1:.1f} s), then samples {c}..{c + more - 1} on {threads} host threads "
                      f"({dm:.1f} s); value and cores are the multi-thread figures"}


WORKLOADS = {"rmat20-lt-dssa": run_rmat20, "pokec-ic-ssa64": run_pokec64, "serving": run_serving,
             "twitter-ic-dssa": run_twitter}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="twitter-ic-dssa")
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--pool-budget-gb", type=float, default=64.0)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--qps", type=float, default=20.0)
    ap.add_argument("--queries", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--compare-plain", action="store_true", help="also time the queries one at a time")
    ap.add_argument("--engine", action="store_true",
                    help="Twitter-shaped workload: run each step's queries concurrently through the engine")
    ap.add_argument("--ks", type=int, nargs="*", default=None, help="Twitter-shaped workload: the k values")
    ap.add_argument("--queries-per-step", type=int, default=1,
                    help="R-MAT-20: concurrent D-SSA queries per step through the multi-query engine")
    ap.add_argument("--greedy-wg-max-entries", type=int, default=None,
                    help="launch parameter: largest Max-Coverage range whose rounds all run in one "
                         "workgroup over the full max index (with --param greedy_wg_cand_max_entries 0)")
    ap.add_argument("--param", nargs=2, action="append", default=[], metavar=("NAME", "VALUE"),
                    help="set a launch parameter (im_ctx_set_param) before the run")
    ap.add_argument("--no-speculate", action="store_true",
                    help="launch parameter: D-SSA draws each iteration's sets only after the previous check")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batching-compare", action="store_true",
                    help="Twitter-shaped workload: skip timing the batched sampler against one launch per query")
    ap.add_argument("--no-gather-probe", action="store_true",
                    help="skip measuring the random-gather bandwidth the sampler is compared with")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is a design "
              "note, not an implemented path.", file=sys.stderr)
        return 2

    from paper_1605_07990_amd import binding as im

    torch = None
    if os.environ.get("IM_NO_TORCH", "") != "1":
        import torch

    if not args.no_gather_probe:
        GATHER.update(gather_bandwidth(record="hbm"))
        GATHER_MALL.update(gather_bandwidth(segs=(64, 128, 256), buffer_bytes=128 << 20, record="mall"))
    ctx = im.Context(0)

    def sync():
        # the context's own streams and any dropped D-SSA covers still running
        # count in the timed region; then the device as torch sees it
        ctx.sync()
        if torch is not None:
            torch.cuda.synchronize()

    if args.greedy_wg_max_entries is not None:
        ctx.set_param("greedy_wg_max_entries", args.greedy_wg_max_entries)
    if args.no_speculate:
        ctx.set_param("dssa_speculate", 0)
    for name, value in args.param:
        ctx.set_param(name, int(value))
    body, cpu = WORKLOADS[args.workload](args, im, ctx, sync)
    steps = args.steps if args.workload != "serving" else 1
    out = {"metric": METRIC, "value": body.pop("value"), "unit": "RR sets/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": body.pop("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic"}
    out.update(body)
    if cpu is not None and not args.no_cpu_baseline:
        cb = cpu(args.cpu_budget)
        cb["host_cpus"] = os.cpu_count()
        out["cpu_baseline"] = cb
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
