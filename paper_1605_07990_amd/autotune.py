"""Autotuner for the library's launch parameters (im_param).

Runs a fixed set of queries on a resident graph once per candidate setting,
times each pass on the device's stream, checks that every setting returns
the same seeds (the parameters only change how work is launched), and
reports the fastest setting per parameter, tuned one parameter at a time in
the order given. The result is a JSON object that `apply` sets on a context.

    python -m paper_1605_07990_amd.autotune --graph rmat20 --model lt --algo dssa --k 100 --queries 4
"""
from __future__ import annotations

import argparse
import json
import time

from . import binding as im

CANDIDATES = {
    "greedy_wg_max_entries": [0, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 62],
    "ic_ticket_block": [0, 1, 2, 4, 8, 16, 32],
    "dssa_speculate": [0, 1],
    "greedy_mark_min_chunks": [0, 1 << 14, 1 << 16, 1 << 62],
    "greedy_cover_blocks": [0, 64, 128, 256, 512, 1024],
    "ic_edge_budget": [512, 1024, 2048, 4096, 8192, 16384, 65536],
    "greedy_candidates": [0, 8, 16, 32, 64],
    "greedy_candidates_batch": [0, 8, 16, 32, 64],
    "dssa_draw_ahead": [1, 2, 4, 8],
    "greedy_wg_cand_max_entries": [0, 1 << 20, 1 << 22, 1 << 24, 1 << 62],
    "greedy_wg_cand_grid_rounds": [0, 4, 8, 16, 32],
    "dssa_greedy_ahead": [0, 1, 2],
    "greedy_wg_cand_batch": [0, 1 << 20, 1 << 21, 1 << 23, 1 << 62],
    "greedy_flat_levels": [1, 0],
    "greedy_dense": [1, 0],
}


def _run(graph, model, algo, k, eps, keys, batch, ctx, sync):
    """Wall time of the query set and every query's seeds."""
    sync()
    t0 = time.perf_counter()
    seeds = []
    if batch <= 1:
        for key in keys:
            s, _ = getattr(graph, algo)(model, k, eps, 1.0 / graph.n, key)
            seeds.append(s.tolist())
    else:
        eng = im.Engine(ctx, max_active=batch)
        tickets = [eng.submit(graph, model, algo, k, eps, 1.0 / graph.n, key) for key in keys]
        eng.run()
        seeds = [eng.result(t)[0].tolist() for t in tickets]
        eng.close()
    sync()
    return time.perf_counter() - t0, seeds


def tune(ctx, graph, model, algo, k, eps, keys, batch=1, params=None, sync=lambda: None, log=print):
    """Coordinate search over `params` (default: every tunable). Returns
    {param: best value} and the timing table."""
    params = list(params or CANDIDATES)
    best = {p: ctx.get_param(p) for p in params}
    table = {}
    ref = None
    _run(graph, model, algo, k, eps, keys, batch, ctx, sync)  # warm caches and buffers
    for p in params:
        times = {}
        for value in CANDIDATES[p]:
            ctx.set_param(p, value)
            dt, seeds = _run(graph, model, algo, k, eps, keys, batch, ctx, sync)
            if ref is None:
                ref = seeds
            elif seeds != ref:
                raise RuntimeError(f"{p}={value} changed the seeds: launch parameters must not change results")
            times[value] = dt
            log(f"{p}={value}: {dt * 1e3:.2f} ms")
        best[p] = min(times, key=times.get)
        ctx.set_param(p, best[p])
        table[p] = {str(v): round(t * 1e3, 3) for v, t in times.items()}
    return best, table


def apply(ctx, tuned: dict):
    """Set every parameter of a `tune` result (or its JSON) on a context."""
    for name, value in tuned.items():
        ctx.set_param(name, int(value))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--graph", default="rmat20")
    ap.add_argument("--model", choices=["ic", "lt"], default="lt")
    ap.add_argument("--algo", choices=["ssa", "dssa"], default="dssa")
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--queries", type=int, default=4)
    ap.add_argument("--batch", type=int, default=1, help="queries run together through the engine")
    ap.add_argument("--params", nargs="*", default=None)
    ap.add_argument("--out", default=None, help="write the tuned parameters as JSON")
    args = ap.parse_args()

    import synth
    import torch

    g = synth.make(args.graph)
    ctx = im.Context(0)
    model = im.MODELS[args.model]
    w = g.w_ic if model == im.IM_IC else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == im.IM_IC else None,
                  w_lt=w if model == im.IM_LT else None)
    best, table = tune(ctx, dg, model, args.algo, args.k, args.eps, list(range(args.queries)), args.batch,
                       args.params, sync=torch.cuda.synchronize)
    out = {"workload": vars(args), "best": best, "ms": table}
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(best, f)
    dg.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
