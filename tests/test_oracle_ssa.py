"""Pins for the oracle's SSA (Algorithm 1) and D-SSA (Algorithm 4).

* Theorems 2 and 5: I(S_k) >= (1 - 1/e - eps) OPT_k with probability >= 1 -
  delta, checked over many stream keys on tiny graphs whose I and OPT_k are
  exact (live-edge enumeration, exhaustive k-subsets).
* Schedule: checkpoints at ceil(Lambda) 2^(t-1) sets; D-SSA reports
  2 N_t sets at the stop; stop conditions C1/C2 and D1/D2 hold at a stop
  that is not the cap.
* Graph without edges: every RR set is a singleton, so I(S) = k for every
  seed set and the estimate tracks k.
"""
import itertools
import math

import numpy as np
import pytest

import bruteforce as bf

ONE_M = 1 - 1 / math.e


@pytest.mark.slow
@pytest.mark.parametrize("model", [0, 1])
def test_approximation_guarantee(oracle_lib, model):
    rng = np.random.default_rng(70 + model)
    n, k, eps, delta = 7, 2, 0.2, 0.2
    edges = bf.random_tiny_graph(rng, n, 11, model)
    src, dst, w = bf.arrays(edges)
    og = oracle_lib.Graph(model, n, src, dst, w)
    spread = bf.ic_exact_spread if model == 0 else bf.lt_exact_spread
    table = {S: spread(n, edges, S) for S in itertools.combinations(range(n), k)}
    opt = max(table.values())
    fails = 0
    runs = 40
    for key in range(runs):
        for algo in (og.ssa, og.dssa):
            seeds, st = algo(k, eps, delta, key)
            val = table[tuple(sorted(seeds.tolist()))]
            fails += val < (1 - 1 / math.e - eps) * opt
    assert fails <= delta * 2 * runs
    assert fails == 0


@pytest.mark.parametrize("model", [0, 1])
def test_schedule_and_stop_conditions(oracle_lib, synth_lib, model):
    g = synth_lib.make("cl_small")
    w = g.w_ic if model == 0 else g.w_lt
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    k, eps, delta = 10, 0.2, 1.0 / g.n
    c = oracle_lib.ssa_constants(g.n, k, eps, delta)
    seeds, st = og.ssa(k, eps, delta, key=3)
    n1 = math.ceil(c["lambda"])
    assert st["it_sets"] == [n1 << t for t in range(st["iterations"])]
    assert len(set(seeds.tolist())) == k
    if not st["stopped_by_cap"]:
        assert st["cov"] >= c["lambda1"]
        assert st["i_c"] > 0 and st["i_hat"] <= (1 + c["eps1"]) * st["i_c"]
        assert st["i_hat"] == pytest.approx(g.n * st["cov"] / st["n_sets"], rel=1e-15)

    d = oracle_lib.dssa_constants(g.n, k, eps, delta)
    seeds, st = og.dssa(k, eps, delta, key=3)
    n1 = math.ceil(d["lambda"])
    assert st["it_sets"] == [n1 << t for t in range(st["iterations"])]
    assert st["n_sets"] == 2 * st["it_sets"][-1]
    if not st["stopped_by_cap"]:
        assert st["cov_c"] >= d["lambda1"]
        assert st["eps_t"] <= eps
    # eps_t is never computed at an iteration that failed D1
    for cov_c, e in zip(st["it_cov_c"], st["it_eps_t"]):
        if cov_c < d["lambda1"]:
            assert e == -1.0


def test_edgeless_graph(oracle_lib):
    n, k = 50, 5
    og = oracle_lib.Graph(oracle_lib.IC, n, np.array([], np.uint32), np.array([], np.uint32),
                          np.array([], np.float32))
    for algo in (og.ssa, og.dssa):
        seeds, st = algo(k, 0.2, 0.05, 9)
        assert len(set(seeds.tolist())) == k
        assert abs(st["i_hat"] / k - 1) < 0.25
