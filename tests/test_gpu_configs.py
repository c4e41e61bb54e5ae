"""Parity on the Pokec-shaped workload at full size (4.8M nodes, 69M edges,
Chung-Lu exponent 2.3, IC trivalency): the 64 concurrent SSA queries
(k = round(exp(U(0, ln 500))), eps uniform over {0.05, 0.1, 0.2},
delta = 1/n, key = query index) run through the engine in one fused run,
and every query's result (seeds, every integer of the trajectory, the FP64
estimates to 1e-12) equals the oracle's plain sequential SSA (Algorithm 1).

The 64 oracle runs take about 1000 s of host CPU in all (the longest, k =
403 at eps = 0.05, about 90 s, dominated by its linear-argmax greedy over
4.8M nodes); they go on the host's cores (one run per thread, largest k
first) while the GPU runs the batch. The first 2^16 sets of four of the
queries' streams are also compared set by set."""
import math
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from gpu_util import assert_pool_equal, note

pytestmark = pytest.mark.gpu

INT_KEYS = ["iterations", "stopped_by_cap", "n_sets", "n_verify", "cov", "cov_c", "it_sets", "it_cov",
            "it_cov_c"]
FP_KEYS = ["i_hat", "i_c", "eps1", "eps2", "eps3", "eps_t"]


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def pokec_queries(n: int, count: int = 64, seed: int = 64):
    """The 64-query mix (the same draw as the benchmark's)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        k = int(min(n, max(1, round(math.exp(rng.uniform(0.0, math.log(500)))))))
        eps = float((0.05, 0.1, 0.2)[int(rng.integers(3))])
        out.append((k, eps, q))
    return out


def compare_to_oracle(res, ores, label):
    seeds, st = res
    oseeds, ost = ores
    assert seeds.tolist() == oseeds.tolist(), label
    for key in INT_KEYS:
        assert st[key] == ost[key], (label, key, st[key], ost[key])
    for key in FP_KEYS:
        assert st[key] == pytest.approx(ost[key], rel=1e-12, abs=1e-300), (label, key)
    for a, b in zip(st["it_eps_t"], ost["it_eps_t"]):
        assert a == pytest.approx(b, rel=1e-12), label


@pytest.mark.timeout(1200)
def test_pokec_64_fused_ssa_queries_match_oracle(oracle_lib):
    from paper_1605_07990_amd import binding as im

    t0 = time.perf_counter()
    note("generating the Pokec-shaped graph")
    g = synth.make("pokec")
    delta = 1.0 / g.n
    og = oracle_lib.Graph(oracle_lib.IC, g.n, g.src, g.dst, g.w_ic)
    qs = pokec_queries(g.n)
    threads = host_threads()
    note(f"n={g.n} m={g.m}; 64 oracle SSA runs on {threads} host threads")
    ex = ThreadPoolExecutor(threads)
    futs = {}
    for k, eps, key in sorted(qs, key=lambda q: -q[0]):
        futs[key] = ex.submit(og.ssa, k, eps, delta, key)

    ctx = im.Context(0)
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    note("engine: 64 SSA queries in one fused run")
    eng = im.Engine(ctx, pool_budget_bytes=64 << 30, max_active=64)
    tickets = [eng.submit(dg, im.IM_IC, "ssa", k, eps, delta, key) for k, eps, key in qs]
    eng.run()
    res = {key: eng.result(t) for (k, eps, key), t in zip(qs, tickets)}
    eng.close()
    note(f"engine done after {time.perf_counter() - t0:.0f} s")

    for key in (1, 6, 18, 50):
        note(f"first 2^16 sets of query {key}'s stream")
        p = im.Pool(dg, im.IM_IC, key)
        p.sample(1 << 16)
        op = oracle_lib.Pool(og, key)
        op.extend(1 << 16)
        assert_pool_equal(p, op, 0, 1 << 16)

    for k, eps, key in qs:
        ores = futs[key].result()
        compare_to_oracle(res[key], ores, (key, k, eps))
    ex.shutdown()
    note(f"64 queries equal the oracle after {time.perf_counter() - t0:.0f} s")
    dg.close()
    ctx.close()
