"""Pins for the oracle's Max-Coverage (Algorithm 2).

* Nemhauser et al.: greedy coverage >= (1 - 1/e) of the exhaustive optimum.
* First pick = most frequent node, lowest id on ties (Lemma 1 intuition of
  Section 3.1.1 and the tie-break reading).
* Lazy (CELF-style) evaluation of the same greedy rule gives the same seeds
  and coverage; marginal gains never increase (submodularity).
* Coverage (Eq. 1) against Python set intersection.
"""
import itertools
import math

import numpy as np
import pytest


def _cov(sets, S):
    S = set(S)
    return sum(1 for r in sets if S & set(r))


def _lazy_greedy(sets, n, k):
    # CELF: keep stale upper bounds in a list; re-evaluate the best stale
    # one until the best bound is fresh. Ties -> lowest id.
    chosen = []
    covered = [False] * len(sets)
    bound = {v: sum(1 for r in sets if v in r) for v in range(n)}
    fresh_round = {v: 0 for v in range(n)}
    for rnd in range(k):
        while True:
            cand = min((v for v in range(n) if v not in chosen), key=lambda v: (-bound[v], v))
            if fresh_round[cand] == rnd:
                break
            bound[cand] = sum(1 for j, r in enumerate(sets) if not covered[j] and cand in r)
            fresh_round[cand] = rnd
        # among nodes with equal fresh gain, a lower id with a stale bound
        # equal to the gain may still tie; settle ties exactly
        best_gain = bound[cand]
        for v in range(cand):
            if v in chosen:
                continue
            g = sum(1 for j, r in enumerate(sets) if not covered[j] and v in r)
            if g == best_gain:
                cand = v
                break
        chosen.append(cand)
        for j, r in enumerate(sets):
            if cand in r:
                covered[j] = True
        for v in range(n):
            fresh_round[v] = min(fresh_round[v], rnd)  # bounds stay valid upper bounds
    return chosen, sum(covered)


def _random_pool(rng, n_sets, n):
    sets = []
    for _ in range(n_sets):
        size = int(rng.integers(0, 5))
        sets.append(sorted(rng.choice(n, size=size, replace=False).tolist()))
    return sets


@pytest.mark.parametrize("seed", range(12))
def test_greedy_vs_exhaustive(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n = 10
    sets = _random_pool(rng, 12, n)
    pool = oracle_lib.Pool.from_sets(n, sets)
    for k in (1, 2, 3, 4):
        seeds, cov = pool.max_coverage(k)
        assert len(set(seeds.tolist())) == k
        assert cov == _cov(sets, seeds.tolist())
        opt = max(_cov(sets, S) for S in itertools.combinations(range(n), k))
        assert cov >= (1 - 1 / math.e) * opt - 1e-9
        lazy, lazy_cov = _lazy_greedy(sets, n, k)
        assert seeds.tolist() == lazy and cov == lazy_cov


def test_first_pick_most_frequent_lowest_id(oracle_lib):
    sets = [[2, 5], [5], [2, 7], [1], [7, 5, 2]]
    pool = oracle_lib.Pool.from_sets(8, sets)
    seeds, cov = pool.max_coverage(1)
    # node 2 and node 5 each appear 3 times -> lowest id 2
    assert seeds.tolist() == [2] and cov == 3


def test_gains_non_increasing_and_k_equals_n(oracle_lib, synth_lib):
    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(oracle_lib.IC, g.n, g.src, g.dst, g.w_ic)
    pool = oracle_lib.Pool(og, 2)
    pool.extend(3000)
    prev = None
    gains = []
    for k in range(1, 31):
        seeds, cov = pool.max_coverage(k)
        if prev is not None:
            assert seeds[:-1].tolist() == prev[0].tolist()  # greedy prefixes nest
            gains.append(cov - prev[1])
        prev = (seeds, cov)
    assert all(a >= b for a, b in zip(gains, gains[1:]))
    # k = n picks every node once; every nonempty set is covered
    sets_small = [[0, 1], [], [2], [1, 2]]
    p2 = oracle_lib.Pool.from_sets(3, sets_small)
    seeds, cov = p2.max_coverage(3)
    assert sorted(seeds.tolist()) == [0, 1, 2] and cov == 3


def test_zero_gain_rounds_take_lowest_unchosen(oracle_lib):
    sets = [[4], [4], [3]]
    pool = oracle_lib.Pool.from_sets(6, sets)
    seeds, cov = pool.max_coverage(4)
    assert seeds.tolist() == [4, 3, 0, 1] and cov == 3


def test_range_and_coverage(oracle_lib):
    rng = np.random.default_rng(99)
    n = 9
    sets = _random_pool(rng, 40, n)
    pool = oracle_lib.Pool.from_sets(n, sets)
    seeds, cov = pool.max_coverage(3, 10, 30)
    assert cov == _cov(sets[10:30], seeds.tolist())
    for S in ([0], [1, 2], [3, 5, 8]):
        assert pool.coverage(S, 5, 35) == _cov(sets[5:35], S)
    with pytest.raises(oracle_lib.OracleError):
        pool.max_coverage(10)  # k > n
