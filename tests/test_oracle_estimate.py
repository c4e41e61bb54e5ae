"""Pins for the oracle's Estimate-Inf (Algorithm 3).

* S = V covers every RR set, so the stopping count is reached exactly at
  T = ceil(Lambda2) and I_c = n Lambda2 / ceil(Lambda2).
* T_max below ceil(Lambda2) can never reach the count: -1.
* Lemma 3: Pr[I_c > (1+eps') I(S)] <= delta', measured over independent
  streams on a graph whose I(S) is known exactly (live-edge enumeration).
"""
import math

import numpy as np
import pytest

import bruteforce as bf


def _lambda2(oracle_lib, eps, delta):
    return 1 + (1 + eps) * oracle_lib.upsilon(eps, delta)


def test_all_nodes_stop_at_ceil_lambda2(oracle_lib, synth_lib):
    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(oracle_lib.IC, g.n, g.src, g.dst, g.w_ic)
    lam2 = _lambda2(oracle_lib, 0.2, 0.01)
    ic, T = og.estimate_inf(np.arange(g.n), 0.2, 0.01, 1e9, key=4)
    assert T == math.ceil(lam2)
    assert ic == pytest.approx(g.n * lam2 / math.ceil(lam2), rel=1e-15)


def test_tmax_too_small_returns_minus_one(oracle_lib, synth_lib):
    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(oracle_lib.LT, g.n, g.src, g.dst, g.w_lt)
    lam2 = _lambda2(oracle_lib, 0.2, 0.01)
    ic, T = og.estimate_inf(np.arange(g.n), 0.2, 0.01, math.ceil(lam2) - 0.5, key=4)
    assert ic == -1.0 and T == math.ceil(lam2) - 1


@pytest.mark.parametrize("model", [0, 1])
def test_lemma3_one_sided_error(oracle_lib, model):
    rng = np.random.default_rng(40 + model)
    n = 6
    edges = bf.random_tiny_graph(rng, n, 10, model)
    src, dst, w = bf.arrays(edges)
    og = oracle_lib.Graph(model, n, src, dst, w)
    S = (1, 4)
    exact = (bf.ic_exact_spread if model == 0 else bf.lt_exact_spread)(n, edges, S)
    eps_p, delta_p = 0.25, 0.1
    runs = 1500
    over = 0
    vals = []
    for r in range(runs):
        ic, T = og.estimate_inf(S, eps_p, delta_p, 1e9, key=1000 + r)
        assert ic > 0
        vals.append(ic)
        over += ic > (1 + eps_p) * exact
    rate = over / runs
    assert rate <= delta_p + 3 * math.sqrt(delta_p * (1 - delta_p) / runs)
    # and the estimate is centred: the stopping-rule estimator is within eps'
    assert abs(np.mean(vals) / exact - 1) < eps_p
