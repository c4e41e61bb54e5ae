"""Pins for the oracle's fixed-threshold RIS and SSA with a caller's
precision split (eps1, eps2, eps3).

* The fixed threshold is the paper's simplification of the RIS bound (the
  threshold equation of Section 3 with OPT_k >= k): the unsimplified value
  N = 2n((1-1/e)a + b)^2 / (eps^2 OPT_k), a = sqrt(ln 2/delta),
  b = sqrt((1-1/e)(ln 2/delta + ln C(n,k))), computed here with lgamma,
  must lie between theta/4 and theta (the simplification only loosens, by
  the two inequalities the paper applies, each at most a factor of 2).
* Fixed-theta RIS and SSA with admissible splits keep the (1-1/e-eps)
  guarantee against exhaustive OPT_k on tiny graphs with exact spreads.
* Eq. 14 admits Eq. 15's default split (with equality) and rejects splits
  that break it.
"""
import itertools
import math

import numpy as np
import pytest

import bruteforce as bf

ONE_M = 1 - 1 / math.e


def ln_choose(n, k):
    return math.lgamma(n + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1)


@pytest.mark.parametrize("n,k,eps,delta", [(15233, 50, 0.1, 1 / 15233), (1 << 20, 100, 0.1, 2 ** -20),
                                           (1000, 1, 0.3, 0.05), (41_700_000, 1000, 0.05, 1 / 41_700_000),
                                           (50, 50, 0.2, 0.1)])
def test_theta_brackets_unsimplified_bound(oracle_lib, n, k, eps, delta):
    theta = oracle_lib.ris_theta(n, k, eps, delta)
    a = math.sqrt(math.log(2 / delta))
    b = math.sqrt(ONE_M * (math.log(2 / delta) + ln_choose(n, k)))
    exact = 2 * n * (ONE_M * a + b) ** 2 / (eps ** 2 * k)
    assert exact <= theta * (1 + 1e-12)
    assert theta <= 4 * exact * (1 + 1e-12)


def test_theta_scaling(oracle_lib):
    # theta ~ 1/eps^2 and ~ n/k for fixed ln terms
    t1 = oracle_lib.ris_theta(10_000, 10, 0.1, 0.01)
    t2 = oracle_lib.ris_theta(10_000, 10, 0.2, 0.01)
    assert t1 / t2 == pytest.approx(4.0, rel=1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("model", [0, 1])
def test_fixed_theta_ris_guarantee(oracle_lib, model):
    rng = np.random.default_rng(90 + model)
    n, k, eps, delta = 7, 2, 0.3, 0.2
    edges = bf.random_tiny_graph(rng, n, 11, model)
    src, dst, w = bf.arrays(edges)
    og = oracle_lib.Graph(model, n, src, dst, w)
    spread = bf.ic_exact_spread if model == 0 else bf.lt_exact_spread
    table = {S: spread(n, edges, S) for S in itertools.combinations(range(n), k)}
    opt = max(table.values())
    theta = math.ceil(oracle_lib.ris_theta(n, k, eps, delta))
    for key in range(10):
        seeds, st = og.ris(k, eps, delta, key)
        assert st["n_sets"] == theta
        assert len(set(seeds.tolist())) == k
        assert table[tuple(sorted(seeds.tolist()))] >= (ONE_M - eps) * opt
        # the returned estimate is n Cov / theta
        assert st["i_hat"] == pytest.approx(n * st["cov"] / theta, rel=1e-15)


def test_eq14_admissibility(oracle_lib):
    for eps in (0.05, 0.1, 0.2, 0.3):
        c = oracle_lib.ssa_constants(1000, 5, eps, 0.01)
        assert oracle_lib.eps_admissible(eps, c["eps1"], c["eps2"], c["eps3"])
        # a split 1% larger in every part breaks Eq. 14
        assert not oracle_lib.eps_admissible(eps, 1.01 * c["eps1"], 1.01 * c["eps2"], 1.01 * c["eps3"])
    assert not oracle_lib.eps_admissible(0.1, 0.2, 0.2, 0.2)
    assert not oracle_lib.eps_admissible(0.5, 0.0, 0.1, 0.1)
    assert not oracle_lib.eps_admissible(0.5, 1.0, 0.01, 0.01)


def test_ssa_eps_with_default_split_is_ssa(oracle_lib, synth_lib):
    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    c = oracle_lib.ssa_constants(g.n, 10, 0.2, 1 / g.n)
    a = og.ssa(10, 0.2, 1 / g.n, 3)
    b = og.ssa_eps(10, 0.2, c["eps1"], c["eps2"], c["eps3"], 1 / g.n, 3)
    assert a[0].tolist() == b[0].tolist()
    assert a[1]["it_cov"] == b[1]["it_cov"] and a[1]["n_sets"] == b[1]["n_sets"]
    with pytest.raises(oracle_lib.OracleError):
        og.ssa_eps(10, 0.1, 0.2, 0.2, 0.2, 1 / g.n, 3)


@pytest.mark.slow
@pytest.mark.parametrize("split", [(0.02, 0.075, 0.075), (0.06, 0.06, 0.06), (0.005, 0.09, 0.09)])
def test_ssa_eps_guarantee(oracle_lib, split):
    eps = 0.2
    rng = np.random.default_rng(95)
    n, k, delta = 7, 2, 0.2
    edges = bf.random_tiny_graph(rng, n, 11, 0)
    src, dst, w = bf.arrays(edges)
    og = oracle_lib.Graph(0, n, src, dst, w)
    table = {S: bf.ic_exact_spread(n, edges, S) for S in itertools.combinations(range(n), k)}
    opt = max(table.values())
    assert oracle_lib.eps_admissible(eps, *split)
    for key in range(20):
        seeds, st = og.ssa_eps(k, eps, *split, delta, key)
        assert table[tuple(sorted(seeds.tolist()))] >= (ONE_M - eps) * opt
        assert (st["eps1"], st["eps2"], st["eps3"]) == split
