"""Pins for weighted RR sets (WRIS, targeted viral marketing, Section 7.3).

With integer node weights w, a source is drawn with probability w_v / W
(W = sum of w) and the objective is the weighted spread I_w(S), the expected
total weight of the nodes S reaches. Lemma 1 then reads
I_w(S) = W Pr[S meets an RR set], so every estimate scales by W, not n.

* Lemma 1, weighted: W Cov / N against I_w(S) computed exactly by
  enumerating live-edge graphs (IC and LT), within 5 sigma.
* S = V meets every set: Estimate-Inf stops at T = ceil(Lambda2) exactly and
  returns W Lambda2 / T (a closed form in W).
* SSA and D-SSA on weighted sources: the reported estimates track I_w(S_k)
  (n-scaled ones would be off by W/n = 14/6 here), and S_k meets the
  (1-1/e-eps) guarantee against the exhaustive weighted optimum.
"""
import itertools
import math

import numpy as np
import pytest

import bruteforce as bf

NODE_W = np.array([0, 4, 1, 0, 7, 2], np.uint32)  # W = 14, n = 6


def tiny(oracle_lib, model, seed):
    rng = np.random.default_rng(seed)
    edges = bf.random_tiny_graph(rng, 6, 10, model)
    src, dst, w = bf.arrays(edges)
    og = oracle_lib.Graph(model, 6, src, dst, w, node_weights=NODE_W)
    spread = bf.ic_exact_spread if model == 0 else bf.lt_exact_spread
    return og, (lambda S: spread(6, edges, S, NODE_W))


@pytest.mark.parametrize("model", [0, 1])
def test_weighted_lemma1(oracle_lib, model):
    og, exact = tiny(oracle_lib, model, 90 + model)
    W = float(NODE_W.sum())
    N = 100_000
    pool = oracle_lib.Pool(og, 5)
    pool.extend(N)
    for S in [(0,), (1, 3), (2, 4), (0, 1, 5)]:
        mu = exact(S) / W
        est = W * pool.coverage(np.array(S, np.uint32)) / N
        sigma = W * math.sqrt(mu * (1 - mu) / N)
        assert abs(est - exact(S)) <= 5 * sigma + 1e-9, (S, est, exact(S))


def test_weighted_estimate_inf_all_nodes(oracle_lib):
    og, _ = tiny(oracle_lib, 0, 91)
    eps_p, delta_p = 0.2, 0.01
    lam2 = 1 + (1 + eps_p) * oracle_lib.upsilon(eps_p, delta_p)
    ic, T = og.estimate_inf(np.arange(6), eps_p, delta_p, 1e9, key=4)
    assert T == math.ceil(lam2)
    assert ic == pytest.approx(14.0 * lam2 / math.ceil(lam2), rel=1e-15)


@pytest.mark.parametrize("model", [0, 1])
def test_weighted_ssa_dssa_estimates(oracle_lib, model):
    og, exact = tiny(oracle_lib, model, 92 + model)
    k, eps, delta = 2, 0.2, 0.2
    opt = max(exact(S) for S in itertools.combinations(range(6), k))
    for key in range(6):
        for algo in ("ssa", "dssa"):
            seeds, st = getattr(og, algo)(k, eps, delta, key)
            val = exact(tuple(sorted(seeds.tolist())))
            assert val >= (1 - 1 / math.e - eps) * opt
            assert abs(st["i_hat"] / val - 1) < 0.15, (algo, key, st["i_hat"], val)
            if st["i_c"] > 0:
                assert abs(st["i_c"] / val - 1) < 0.25, (algo, key, st["i_c"], val)
