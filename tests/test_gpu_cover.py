"""GPU parity of Max-Coverage (Algorithm 2), coverage counts (Eq. 1) and
Estimate-Inf (Algorithm 3) against the oracle: identical seeds (ties to the
lowest id), identical integer coverage, identical stopping index T."""
import math

import numpy as np
import pytest

import synth
from gpu_util import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def im():
    from paper_1605_07990_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(im):
    return im.Context(0)


@pytest.fixture(scope="module")
def pools(im, ctx, oracle_lib):
    out = {}
    for name, model, count, key in (("nethept", 0, 40000, 1), ("rmat16", 1, 30000, 2), ("cl_small", 1, 8000, 3)):
        g = synth.make(name)
        w = g.w_ic if model == 0 else g.w_lt
        dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
        og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
        p = im.Pool(dg, model, key)
        p.sample(count)
        op = oracle_lib.Pool(og, key)
        op.extend(count)
        out[name] = (g, dg, og, p, op)
    return out


@pytest.mark.parametrize("name", ["nethept", "rmat16", "cl_small"])
@pytest.mark.parametrize("k", [1, 7, 50, 200, 2000])
def test_max_coverage_matches_oracle(pools, name, k):
    g, dg, og, p, op = pools[name]
    note(f"max coverage {name} k={k}")
    seeds, cov = p.max_coverage(k)
    oseeds, ocov = op.max_coverage(k)
    assert cov == ocov
    assert seeds.tolist() == oseeds.tolist()


@pytest.mark.parametrize("name", ["nethept", "rmat16"])
def test_ranges_and_coverage(pools, name):
    g, dg, og, p, op = pools[name]
    c = p.count
    note(f"coverage ranges {name}")
    for begin, end, k in ((0, c // 2, 20), (c // 2, c, 20), (1234, 1234 + 4097, 5), (7, 8, 3), (100, 100, 2)):
        seeds, cov = p.max_coverage(k, begin, end)
        oseeds, ocov = op.max_coverage(k, begin, end)
        assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (begin, end, k)
        assert p.coverage(seeds, 0, c) == op.coverage(seeds, 0, c)
        assert p.coverage(seeds, end, c) == op.coverage(seeds, end, c)
    rng = np.random.default_rng(0)
    for _ in range(5):
        S = rng.choice(g.n, size=int(rng.integers(1, 40)), replace=False)
        assert p.coverage(S, 0, c) == op.coverage(S, 0, c)
    assert p.coverage(np.arange(g.n), 0, c) == c


def test_k_equals_n_and_errors(im, ctx, oracle_lib):
    note("k = n and bad k")
    n = 40
    e = np.array([], np.uint32)
    dg = im.Graph(ctx, n, e, e, w_ic=np.array([], np.float32))
    og = oracle_lib.Graph(0, n, e, e, np.array([], np.float32))
    p = im.Pool(dg, 0, 5)
    p.sample(300)
    op = oracle_lib.Pool(og, 5)
    op.extend(300)
    seeds, cov = p.max_coverage(n)
    oseeds, ocov = op.max_coverage(n)
    assert seeds.tolist() == oseeds.tolist() and cov == ocov == 300
    with pytest.raises(im.ImError):
        p.max_coverage(n + 1)
    with pytest.raises(im.ImError):
        p.max_coverage(0)


@pytest.mark.parametrize("name,model", [("nethept", 0), ("rmat16", 1), ("cl_small", 0), ("cl_small", 1)])
def test_estimate_inf_matches_oracle(im, ctx, oracle_lib, name, model):
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    rng = np.random.default_rng(1)
    note(f"estimate-inf {name} model={model}")
    cases = [(rng.choice(g.n, size=10, replace=False), 0.1, 1e-3, 1e9, 31),
             (rng.choice(g.n, size=3, replace=False), 0.2, 0.01, 1e9, 32),
             (np.arange(g.n), 0.15, 1e-4, 1e9, 33),
             (rng.choice(g.n, size=5, replace=False), 0.1, 1e-3, 5000.7, 34)]
    for S, e, d, tmax, key in cases:
        ic, T = dg.estimate_inf(model, S, e, d, tmax, key)
        oic, oT = og.estimate_inf(S, e, d, tmax, key)
        assert T == oT, (S[:5], e, d, tmax, T, oT)
        assert ic == oic
    # all nodes: the count is reached exactly at ceil(Lambda2)
    ic, T = dg.estimate_inf(model, np.arange(g.n), 0.2, 0.01, 1e9, 40)
    lam2 = 1 + 1.2 * oracle_lib.upsilon(0.2, 0.01)
    assert T == math.ceil(lam2)


@pytest.mark.parametrize("limit,mark,cand", [(0, 1 << 62, 0), (0, 0, 0), (1 << 62, 1 << 62, 0),
                                             (0, 1 << 62, 32), (0, 0, 32), (0, 1 << 62, 1), (0, 0, 1),
                                             (0, 1 << 62, 64), (0, 0, 5)])
@pytest.mark.parametrize("name", ["nethept", "rmat16", "cl_small"])
def test_greedy_paths_agree(im, ctx, pools, name, limit, mark, cand):
    """Every greedy schedule gives the oracle's seeds: grid-wide rounds over
    candidate chunks (cand > 0; 1 re-selects after nearly every round) or
    two launches per round (cand = 0), re-checking holders or re-deriving
    marked chunks (mark = 0), or all rounds in one workgroup."""
    g, dg, og, p, op = pools[name]
    note(f"greedy path limit={limit} mark={mark} cand={cand} {name}")
    names = ("greedy_wg_max_entries", "greedy_mark_min_chunks", "greedy_candidates", "greedy_wg_cand_max_entries")
    old = [ctx.get_param(x) for x in names]
    for x, v in zip(names, (limit, mark, cand, 0)):
        ctx.set_param(x, v)
    try:
        for k in (1, 50, 300):
            seeds, cov = p.max_coverage(k)
            oseeds, ocov = op.max_coverage(k)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), k
    finally:
        for x, v in zip(names, old):
            ctx.set_param(x, v)


@pytest.mark.parametrize("lead", [0, 3, 64])
@pytest.mark.parametrize("name", ["nethept", "rmat16", "cl_small"])
def test_wg_candidate_rounds_agree(im, ctx, pools, name, lead):
    """Rounds in one workgroup over candidate nodes, after `lead` grid-wide
    rounds, give the oracle's seeds, on whole pools and sub-ranges, from one
    seed to more seeds than one candidate set holds (several re-selections,
    the zero-gain tail)."""
    g, dg, og, p, op = pools[name]
    c = p.count
    note(f"one-workgroup candidate rounds {name} lead={lead}")
    old = ctx.get_param("greedy_wg_cand_max_entries"), ctx.get_param("greedy_wg_cand_grid_rounds")
    ctx.set_param("greedy_wg_cand_max_entries", 1 << 62)
    ctx.set_param("greedy_wg_cand_grid_rounds", lead)
    try:
        for begin, end, k in ((0, c, 1), (0, c, 50), (0, c, 700), (0, c, 2000), (c // 2, c, 20),
                              (1234, 1234 + 4097, 5), (7, 8, 3), (100, 100, 2)):
            seeds, cov = p.max_coverage(k, begin, end)
            oseeds, ocov = op.max_coverage(k, begin, end)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (begin, end, k)
    finally:
        ctx.set_param("greedy_wg_cand_max_entries", old[0])
        ctx.set_param("greedy_wg_cand_grid_rounds", old[1])


@pytest.mark.parametrize("flat", [1, 0])
@pytest.mark.parametrize("lead", [0, 2])
def test_wg_candidate_rounds_edge_cases(im, ctx, oracle_lib, lead, flat):
    """k = n on a graph without edges (every gain reaches zero), flat gains
    (the rounds by gain level, or the grid-wide rounds, take over), and more
    sets than the LDS covered-set bitmap holds."""
    note(f"one-workgroup candidate rounds: k = n, 400k sets, lead={lead} flat levels={flat}")
    old = (ctx.get_param("greedy_wg_cand_max_entries"), ctx.get_param("greedy_wg_cand_grid_rounds"),
           ctx.get_param("greedy_flat_levels"))
    ctx.set_param("greedy_wg_cand_max_entries", 1 << 62)
    ctx.set_param("greedy_wg_cand_grid_rounds", lead)
    ctx.set_param("greedy_flat_levels", flat)
    try:
        n = 40
        e = np.array([], np.uint32)
        dg = im.Graph(ctx, n, e, e, w_ic=np.array([], np.float32))
        og = oracle_lib.Graph(0, n, e, e, np.array([], np.float32))
        p = im.Pool(dg, 0, 5)
        p.sample(300)
        op = oracle_lib.Pool(og, 5)
        op.extend(300)
        for k in (1, 39, n):
            seeds, cov = p.max_coverage(k)
            oseeds, ocov = op.max_coverage(k)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), k
        # flat gains: every set is one node of 200k, so many nodes share each
        # gain and a bin cut soon keeps too few candidates (grid-wide rounds
        # finish the range)
        n = 200_000
        dg = im.Graph(ctx, n, e, e, w_ic=np.array([], np.float32))
        og = oracle_lib.Graph(0, n, e, e, np.array([], np.float32))
        p = im.Pool(dg, 0, 6)
        p.sample(200_000)
        op = oracle_lib.Pool(og, 6)
        op.extend(200_000)
        for k in (50, 300, 1500):
            seeds, cov = p.max_coverage(k)
            oseeds, ocov = op.max_coverage(k)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), k
        # more seeds than nodes that appear: the zero-gain tail after the levels
        for begin, end, k in ((0, 3000, 4000), (5000, 5700, 900)):
            seeds, cov = p.max_coverage(k, begin, end)
            oseeds, ocov = op.max_coverage(k, begin, end)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (begin, end, k)
        g = synth.make("cl_20k")
        dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
        og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
        p = im.Pool(dg, 0, 9)
        p.sample(400_000)
        op = oracle_lib.Pool(og, 9)
        op.extend(400_000)
        for k in (5, 600):
            seeds, cov = p.max_coverage(k)
            oseeds, ocov = op.max_coverage(k)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), k
    finally:
        ctx.set_param("greedy_wg_cand_max_entries", old[0])
        ctx.set_param("greedy_wg_cand_grid_rounds", old[1])
        ctx.set_param("greedy_flat_levels", old[2])


def test_one_workgroup_greedy_large_range(im, ctx, oracle_lib):
    """More sets than the LDS covered-set bitmap holds and more dirty chunks
    per round than the list holds, in one workgroup."""
    g = synth.make("cl_20k")
    note("one-workgroup greedy on 400k sets")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    p = im.Pool(dg, 0, 9)
    p.sample(400_000)
    op = oracle_lib.Pool(og, 9)
    op.extend(400_000)
    old = ctx.get_param("greedy_wg_max_entries"), ctx.get_param("greedy_wg_cand_max_entries")
    ctx.set_param("greedy_wg_max_entries", 1 << 62)
    ctx.set_param("greedy_wg_cand_max_entries", 0)
    try:
        for k in (5, 120):
            seeds, cov = p.max_coverage(k)
            oseeds, ocov = op.max_coverage(k)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), k
    finally:
        ctx.set_param("greedy_wg_max_entries", old[0])
        ctx.set_param("greedy_wg_cand_max_entries", old[1])


@pytest.mark.parametrize("graph", [1, 0])
def test_greedy_round_graph_replays(im, ctx, pools, graph):
    """The per-round launches of one range replayed from the cached graph
    (built the second time a round count and launch shape recur) give the
    oracle's seeds on every call, across ranges of one shape and of several
    and across pools."""
    note(f"greedy round graph {graph}")
    old = ctx.get_param("greedy_graph"), ctx.get_param("greedy_candidates"), ctx.get_param("greedy_wg_cand_max_entries")
    ctx.set_param("greedy_graph", graph)
    ctx.set_param("greedy_candidates", 0)
    ctx.set_param("greedy_wg_cand_max_entries", 0)
    try:
        for rep in range(3):
            for name in ("nethept", "rmat16"):
                g, dg, og, p, op = pools[name]
                c = p.count
                for b, e, k in ((0, c, 50), (0, c // 2, 50), (c // 2, c, 50), (0, c, 7), (3, c - 5, 50)):
                    seeds, cov = p.max_coverage(k, b, e)
                    oseeds, ocov = op.max_coverage(k, b, e)
                    assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (rep, name, b, e, k)
    finally:
        ctx.set_param("greedy_graph", old[0])
        ctx.set_param("greedy_candidates", old[1])
        ctx.set_param("greedy_wg_cand_max_entries", old[2])


@pytest.mark.parametrize("dense", [1, 0])
def test_greedy_over_held_nodes_matches_oracle(im, ctx, oracle_lib, dense):
    """Max-Coverage of ranges holding fewer entries than half the nodes runs
    over the nodes the range holds (ranked in id order) when the parameter
    is on: the picks equal Algorithm 2 over all nodes, including rounds
    after every set is covered (the lowest unpicked ids, nodes outside the
    range among them) and k above the number of nodes the range holds."""
    note(f"greedy over held nodes: dense={dense}")
    old = ctx.get_param("greedy_dense")
    ctx.set_param("greedy_dense", dense)
    try:
        g = synth.make("cl_mid")
        dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
        og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
        p = im.Pool(dg, 0, 21)
        p.sample(3000)
        op = oracle_lib.Pool(og, 21)
        op.extend(3000)
        for begin, end, k in ((0, 3000, 1), (0, 3000, 10), (0, 3000, 400), (700, 1900, 2500), (17, 41, 100),
                              (2999, 3000, 3), (0, 3000, 5000)):
            seeds, cov = p.max_coverage(k, begin, end)
            oseeds, ocov = op.max_coverage(k, begin, end)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (begin, end, k)
        # every set a single source node: the held nodes are the sources
        n = 200_000
        e = np.array([], np.uint32)
        dg = im.Graph(ctx, n, e, e, w_ic=np.array([], np.float32))
        og = oracle_lib.Graph(0, n, e, e, np.array([], np.float32))
        p = im.Pool(dg, 0, 22)
        p.sample(5000)
        op = oracle_lib.Pool(og, 22)
        op.extend(5000)
        for begin, end, k in ((0, 100, 150), (250, 4250, 60), (0, 5000, 5200)):
            seeds, cov = p.max_coverage(k, begin, end)
            oseeds, ocov = op.max_coverage(k, begin, end)
            assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (begin, end, k)
    finally:
        ctx.set_param("greedy_dense", old)


def test_one_seed_over_growing_prefixes(im, ctx, oracle_lib):
    """Max-Coverage with k = 1 over a prefix [0, end) keeps the node counts
    of the last prefix of the same pool and adds only the new sets' entries
    (SSA and D-SSA double their prefixes); a one-seed coverage count over
    [end, 2 end) right after it (D-SSA's stare step) is the seed's count over
    the range's entries and leaves the counts at [0, 2 end). Every answer
    must be the oracle's: growing, repeated and shrinking prefixes, a range
    not at 0, another pool in between, stares that do and do not start
    where the counts end, and a prefix reaching sets appended after the
    last call."""
    g = synth.make("nethept")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    p, q = im.Pool(dg, 0, 41), im.Pool(dg, 0, 42)
    op, oq = oracle_lib.Pool(og, 41), oracle_lib.Pool(og, 42)
    p.sample(20000)
    op.extend(30000)
    q.sample(5000)
    oq.extend(5000)
    note("k = 1 over growing prefixes")
    steps = [(p, op, 0, 1000), (p, op, 0, 4000), (p, op, 0, 4000), (q, oq, 0, 3000), (p, op, 0, 16000),
             (p, op, 1000, 5000), (p, op, 0, 20000), (p, op, 0, 2000), (p, op, 0, 8000), (q, oq, 0, 5000)]
    def same(pool, opool, begin, end):
        seeds, cov = pool.max_coverage(1, begin, end)
        oseeds, ocov = opool.max_coverage(1, begin, end)
        assert (seeds.tolist(), cov) == (oseeds.tolist(), ocov), (pool.key, begin, end)
        return seeds

    def stare(pool, opool, seeds, begin, end):
        assert pool.coverage(seeds, begin, end) == opool.coverage(seeds, begin, end), (pool.key, begin, end)

    for pool, opool, begin, end in steps:
        seeds = same(pool, opool, begin, end)
        if begin == 0 and 2 * end <= pool.count:
            stare(pool, opool, seeds, end, 2 * end)  # starts where the counts end
            stare(pool, opool, seeds, end, 2 * end)  # the counts now reach 2 end: the plain count
            other = np.array([(int(seeds[0]) + 1) % g.n], dtype=np.uint32)
            stare(pool, opool, other, 2 * end, min(pool.count, 3 * end))  # another node, at the counts' end
    seeds = same(p, op, 0, 4000)
    stare(p, op, seeds, 2000, 6000)  # a range that does not start where the counts end
    same(p, op, 0, 6000)
    p.sample(10000)  # appended: the next prefix holds sets drawn after the counts were taken
    seeds = same(p, op, 0, 15000)
    stare(p, op, seeds, 15000, 30000)
    same(p, op, 0, 30000)
    same(p, op, 0, 25000)
