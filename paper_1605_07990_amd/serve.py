"""Request loop for influence-maximization queries over resident graphs.

Queries (graph, model, algorithm, k, eps) arrive over time; the loop hands
each one to the multi-query engine of the HIP library as soon as it has
arrived, and keeps stepping the engine, so requests that arrive while
others are on the GPU join the next fused passes (continuous batching).
The engine admits queued queries as active slots and RR-pool bytes free up.
Graphs stay resident for the loop's life; every query carries its own
stream key, so its RR pool and its SSA verification streams are fresh.

All device work happens inside the library; this module only schedules
submissions by arrival time and records latencies.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import binding as im

EPS_CHOICES = (0.05, 0.1, 0.2)


@dataclass
class Request:
    arrival: float  # seconds after the start of the stream
    graph: str
    model: int
    algo: int
    k: int
    eps: float
    key: int


def poisson_requests(graphs: dict, qps: float, count: int, seed: int, k_max: int = 1000,
                     algo: str | None = "dssa", key_base: int = 0) -> list[Request]:
    """A seeded Poisson stream: exponential inter-arrival times at rate qps,
    graph uniform over `graphs` ({name: (n, has_ic, has_lt)}), model IC or LT
    with probability 1/2 each (among those the graph carries), k =
    round(exp(U(0, ln k_max))) clipped to n, eps uniform over 0.05/0.1/0.2,
    algorithm D-SSA, SSA, or either with probability 1/2 (algo=None), and
    stream key key_base + request index."""
    rng = np.random.default_rng(seed)
    names = sorted(graphs)
    arrivals = np.cumsum(rng.exponential(1.0 / qps, size=count))
    out = []
    for i in range(count):
        name = names[int(rng.integers(len(names)))]
        n, has_ic, has_lt = graphs[name]
        models = [m for m, ok in ((im.IM_IC, has_ic), (im.IM_LT, has_lt)) if ok]
        model = models[int(rng.integers(len(models)))]
        k = int(min(n, max(1, round(math.exp(rng.uniform(0.0, math.log(k_max)))))))
        eps = float(EPS_CHOICES[int(rng.integers(len(EPS_CHOICES)))])
        a = im.ALGOS[algo] if algo is not None else int(rng.integers(2))
        out.append(Request(float(arrivals[i]), name, model, a, k, eps, key_base + i))
    return out


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def serve(engine: "im.Engine", graphs: dict, requests: list[Request], keep_results: bool = False,
          progress=None) -> dict:
    """Replay `requests` against the wall clock through `engine`.

    graphs: {name: binding.Graph} resident on the engine's context.
    Returns latency percentiles (arrival to result), throughput and, with
    keep_results, every request's (seeds, stats) in request order.
    progress(done, total, active) is called after every engine step that
    finished a query.
    """
    reqs = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
    outstanding = {}  # ticket -> request index
    latency = [0.0] * len(requests)
    results = [None] * len(requests) if keep_results else None
    sets = edges = 0
    sizes = [0] * len(requests)  # RR sets each query drew (main plus verification)
    steps = 0
    max_active = 0
    nxt = 0
    t0 = time.perf_counter()
    while nxt < len(reqs) or outstanding:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and requests[reqs[nxt]].arrival <= now:
            r = requests[reqs[nxt]]
            g = graphs[r.graph]
            t = engine.submit(g, r.model, r.algo, r.k, r.eps, 1.0 / g.n, r.key)
            outstanding[t] = reqs[nxt]
            nxt += 1
        if not outstanding:
            # idle until the next arrival
            wait = requests[reqs[nxt]].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            continue
        active, _ = engine.step()
        steps += 1
        max_active = max(max_active, active)
        done_at = time.perf_counter() - t0
        finished = [t for t in outstanding if engine.poll(t) != 0]
        for t in finished:
            i = outstanding.pop(t)
            seeds, st = engine.result(t)
            latency[i] = (done_at - requests[i].arrival) * 1e3
            sets += st["n_sets"] + st["n_verify"]
            sizes[i] = int(st["n_sets"] + st["n_verify"])
            edges += st["edges"]
            if keep_results:
                results[i] = (seeds, st)
        if finished and progress is not None:
            progress(len(requests) - len(outstanding) - (len(reqs) - nxt), len(requests), active)
    wall = time.perf_counter() - t0
    span = requests[reqs[-1]].arrival if reqs else 0.0
    slowest = sorted(range(len(requests)), key=lambda i: -latency[i])[:10]
    out = {"queries": len(requests), "wall_s": wall, "arrival_span_s": span,
           "slowest": [{"graph": requests[i].graph, "model": "IC" if requests[i].model == im.IM_IC else "LT",
                        "algo": "D-SSA" if requests[i].algo == im.ALGOS["dssa"] else "SSA", "k": requests[i].k,
                        "eps": requests[i].eps, "ms": round(latency[i], 1), "rr_sets": sizes[i]} for i in slowest],
           "offered_qps": len(requests) / span if span > 0 else float("inf"),
           "achieved_qps": len(requests) / wall if wall > 0 else 0.0,
           "p50_ms": percentile(latency, 50), "p99_ms": percentile(latency, 99),
           "mean_ms": float(np.mean(latency)) if latency else 0.0,
           "rr_sets_per_s": sets / wall if wall > 0 else 0.0, "edges_per_s": edges / wall if wall > 0 else 0.0,
           "engine_steps": steps, "max_active": max_active}
    if keep_results:
        out["results"] = results
    return out
