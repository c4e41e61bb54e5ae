"""Pins for the oracle's RR sets (Definition 2) against the diffusion models.

* Lemma 1: I(S) = n Pr[S covers R] -- compared with the exact spread from
  enumerating live-edge graphs (IC) or live in-edge choices (LT), within 5
  standard errors, for sets S of one and two nodes, and per node through the
  inclusion frequencies Pr[u in R] = I({u})/n.
* The LT live-edge reading (Kempe et al.) checked against a simulation of
  the threshold model as defined.
* Special cases with textbook answers: IC p = 1 gives the ancestors of the
  source (scipy breadth-first order); p = 0 / w = 0 give the source alone;
  an LT path with weight 1 gives the whole prefix.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order

import bruteforce as bf

N_SAMPLES = 200_000


def _pool_sets(og, oracle_lib, key, count):
    pool = oracle_lib.Pool(og, key)
    pool.extend(count)
    off = pool.offsets()
    nodes = pool.nodes()
    return off, nodes


def _covers(off, nodes, S, n):
    mark = np.zeros(n, bool)
    mark[list(S)] = True
    hit = mark[nodes].astype(np.int64)
    csum = np.concatenate([[0], np.cumsum(hit)])
    return (csum[off[1:]] - csum[off[:-1]]) > 0


@pytest.mark.parametrize("model,seed", [(0, 1), (0, 2), (0, 3), (1, 4), (1, 5), (1, 6)])
def test_lemma1_spread_matches_exact(oracle_lib, model, seed):
    rng = np.random.default_rng(seed)
    n = 6
    edges = bf.random_tiny_graph(rng, n, 11, model)
    src, dst, w = bf.arrays(edges)
    og = oracle_lib.Graph(model, n, src, dst, w)
    off, nodes = _pool_sets(og, oracle_lib, key=seed, count=N_SAMPLES)
    exact_fn = bf.ic_exact_spread if model == 0 else bf.lt_exact_spread
    for S in [(0,), (3,), (1, 4), (2, 5)]:
        exact = exact_fn(n, edges, S)
        mu = exact / n
        est = _covers(off, nodes, S, n).mean()
        sigma = np.sqrt(mu * (1 - mu) / N_SAMPLES)
        assert abs(est - mu) <= 5 * sigma + 1e-12, (S, est * n, exact)
    # per-node inclusion frequency = I({u}) / n
    freq = np.bincount(nodes, minlength=n) / N_SAMPLES
    for u in range(n):
        mu = exact_fn(n, edges, (u,)) / n
        sigma = np.sqrt(mu * (1 - mu) / N_SAMPLES)
        assert abs(freq[u] - mu) <= 5 * sigma + 1e-12, (u, freq[u], mu)


@pytest.mark.parametrize("seed", [7, 8])
def test_lt_live_edge_reading_matches_threshold_model(seed):
    rng = np.random.default_rng(seed)
    n = 6
    edges = bf.random_tiny_graph(rng, n, 10, 1)
    for S in [(0,), (2, 3)]:
        exact = bf.lt_exact_spread(n, edges, S)
        mc = bf.lt_threshold_mc(n, edges, S, trials=20000, seed=seed)
        # spread <= n, so the Monte Carlo standard error is below n/(2 sqrt(T))
        assert abs(mc - exact) <= 5 * n / (2 * np.sqrt(20000)), (S, mc, exact)


def test_ic_exact_matches_forward_cascade():
    rng = np.random.default_rng(9)
    n = 6
    edges = bf.random_tiny_graph(rng, n, 10, 0)
    exact = bf.ic_exact_spread(n, edges, (1,))
    mc = bf.ic_forward_mc(n, edges, (1,), trials=20000, seed=9)
    assert abs(mc - exact) <= 5 * n / (2 * np.sqrt(20000))


def test_ic_p1_gives_ancestors(oracle_lib, synth_lib):
    g = synth_lib.make("cl_small")
    w = np.ones(g.m, np.float32)
    og = oracle_lib.Graph(oracle_lib.IC, g.n, g.src, g.dst, w)
    rev = sp.csr_matrix((np.ones(g.m), (g.dst.astype(np.int64), g.src.astype(np.int64))), shape=(g.n, g.n))
    for s in range(40):
        r, _ = og.rr_set(3, s)
        v = og.source(3, s)
        anc = np.sort(breadth_first_order(rev, v, directed=True, return_predecessors=False))
        assert r.tolist() == anc.tolist()


def test_zero_weights_give_singletons(oracle_lib, synth_lib):
    g = synth_lib.make("cl_small")
    w0 = np.zeros(g.m, np.float32)
    for model in (0, 1):
        og = oracle_lib.Graph(model, g.n, g.src, g.dst, w0)
        for s in range(50):
            r, _ = og.rr_set(11, s)
            assert r.tolist() == [og.source(11, s)]


def test_lt_path_weight_one_gives_prefix(oracle_lib):
    # path 0 -> 1 -> ... -> 9 with w = 1: RR set of source v = {0..v}
    n = 10
    src = np.arange(0, n - 1, dtype=np.uint32)
    dst = np.arange(1, n, dtype=np.uint32)
    og = oracle_lib.Graph(oracle_lib.LT, n, src, dst, np.ones(n - 1, np.float32))
    for s in range(60):
        r, steps = og.rr_set(5, s)
        v = og.source(5, s)
        assert r.tolist() == list(range(v + 1))
        assert steps == v + 1


def test_star_spread(oracle_lib):
    # centre 0 with out-edges to 1..5, IC probabilities p_i: I({0}) = 1 + sum p_i
    p = np.array([0.1, 0.3, 0.5, 0.7, 0.9], np.float32)
    n = 6
    og = oracle_lib.Graph(oracle_lib.IC, n, np.zeros(5, np.uint32), np.arange(1, 6, dtype=np.uint32), p)
    off, nodes = _pool_sets(og, oracle_lib, key=17, count=N_SAMPLES)
    est = _covers(off, nodes, (0,), n).mean() * n
    exact = 1 + float(p.astype(np.float64).sum())
    mu = exact / n
    assert abs(est / n - mu) <= 5 * np.sqrt(mu * (1 - mu) / N_SAMPLES)


def test_sources_uniform(oracle_lib):
    n = 7
    og = oracle_lib.Graph(oracle_lib.IC, n, np.array([], np.uint32), np.array([], np.uint32),
                          np.array([], np.float32))
    counts = np.bincount([og.source(21, s) for s in range(70000)], minlength=n)
    # chi-square with 6 degrees of freedom: 99.99th percentile is about 27.9
    exp = 70000 / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 27.9


def test_weighted_sources_follow_node_weights(oracle_lib):
    n = 5
    wts = np.array([0, 1, 2, 3, 4], np.uint32)
    og = oracle_lib.Graph(oracle_lib.IC, n, np.array([], np.uint32), np.array([], np.uint32),
                          np.array([], np.float32), node_weights=wts)
    counts = np.bincount([og.source(22, s) for s in range(50000)], minlength=n)
    assert counts[0] == 0
    exp = 50000 * wts[1:] / wts.sum()
    chi2 = ((counts[1:] - exp) ** 2 / exp).sum()
    assert chi2 < 21.1  # 3 dof, 99.99th percentile


def test_sets_sorted_and_distinct(oracle_lib, synth_lib):
    g = synth_lib.make("rmat12")
    for model, w in ((0, g.w_ic), (1, g.w_lt)):
        og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
        for s in range(300):
            r, _ = og.rr_set(1, s)
            assert np.all(np.diff(r.astype(np.int64)) > 0)
            assert og.source(1, s) in set(r.tolist())


def test_threaded_extension_equals_sequential(oracle_lib, synth_lib):
    # The multi-core timing path draws contiguous sample blocks on host
    # threads; every set is a pure function of (key, s), so the pool (and its
    # edge count) must equal the sequential one, for any thread count.
    g = synth_lib.make("cl_small")
    for model, w in ((0, g.w_ic), (1, g.w_lt)):
        og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
        ref = oracle_lib.Pool(og, 12)
        ref.extend(3001)
        for threads in (2, 7, 16):
            p = oracle_lib.Pool(og, 12)
            p.extend(1000)
            p.extend(3001, threads=threads)
            assert np.array_equal(p.offsets(), ref.offsets())
            assert np.array_equal(p.nodes(), ref.nodes())
            assert p.edges == ref.edges


def test_concurrent_runs_on_threads(oracle_lib, synth_lib):
    # Runs on several host threads at once (ctypes releases the GIL) give the
    # results of the same runs one after another.
    from concurrent.futures import ThreadPoolExecutor

    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    keys = list(range(8))
    seq = [og.dssa(5, 0.2, 1.0 / g.n, key) for key in keys]
    with ThreadPoolExecutor(4) as ex:
        par = list(ex.map(lambda key: og.dssa(5, 0.2, 1.0 / g.n, key), keys))
    for (a, sa), (b, sb) in zip(seq, par):
        assert a.tolist() == b.tolist() and sa == sb
