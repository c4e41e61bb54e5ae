"""GPU tests of the multi-query engine: every query's result equals the
single-query run (im_ssa / im_dssa) with the same arguments and the oracle,
whatever else is admitted beside it, under any admission limits."""
import numpy as np
import pytest

import synth
from gpu_util import note

pytestmark = pytest.mark.gpu

INT_KEYS = ["iterations", "stopped_by_cap", "n_sets", "n_verify", "cov", "cov_c", "edges", "it_sets", "it_cov",
            "it_cov_c"]
FP_KEYS = ["i_hat", "i_c", "eps1", "eps2", "eps3", "eps_t"]


@pytest.fixture(scope="module")
def im():
    from paper_1605_07990_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(im):
    c = im.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def graphs(im, ctx):
    out = {}
    for name in ("cl_small", "nethept", "rmat16"):
        g = synth.make(name)
        out[name] = (g, im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic, w_lt=g.w_lt))
    return out


def _same(a, b):
    """Engine and single-query results agree exactly (the engine runs the
    same FP64 code on the same integers)."""
    sa, sta = a
    sb, stb = b
    assert sa.tolist() == sb.tolist()
    for key in INT_KEYS:
        assert sta[key] == stb[key], (key, sta[key], stb[key])
    for key in FP_KEYS:
        assert sta[key] == stb[key], (key, sta[key], stb[key])
    assert sta["it_eps_t"] == stb["it_eps_t"]


# (graph, model, algo, k, eps, key): a mix of IC and LT, SSA and D-SSA,
# budgets from 1 to 60 and several precisions, all on shared graphs.
MIX = [
    ("cl_small", 0, "ssa", 10, 0.2, 1),
    ("cl_small", 1, "dssa", 10, 0.2, 2),
    ("cl_small", 0, "dssa", 1, 0.1, 3),
    ("cl_small", 1, "ssa", 25, 0.15, 4),
    ("nethept", 0, "ssa", 50, 0.1, 0),
    ("nethept", 0, "dssa", 50, 0.1, 0),
    ("nethept", 1, "dssa", 20, 0.2, 7),
    ("nethept", 1, "ssa", 5, 0.1, 8),
    ("rmat16", 1, "dssa", 40, 0.1, 6),
    ("rmat16", 0, "ssa", 60, 0.2, 9),
    ("rmat16", 0, "dssa", 3, 0.3, 10),
]


def _single(graphs, case):
    name, model, algo, k, eps, key = case
    g, dg = graphs[name]
    return getattr(dg, algo)(model, k, eps, 1.0 / g.n, key)


def _engine(im, ctx, graphs, cases, budget=16 << 30, max_active=64):
    eng = im.Engine(ctx, pool_budget_bytes=budget, max_active=max_active)
    tickets = []
    for name, model, algo, k, eps, key in cases:
        g, dg = graphs[name]
        tickets.append(eng.submit(dg, model, algo, k, eps, 1.0 / g.n, key))
    steps = 0
    while True:
        active, pending = eng.step()
        steps += 1
        if active + pending == 0:
            break
        assert steps < 10_000
    res = [eng.result(t) for t in tickets]
    eng.close()
    return res, steps


@pytest.mark.parametrize("limit,mark,cand", [(None, None, None), (0, None, None), (0, 0, None),
                                             (1 << 62, None, None), (0, None, 0), (0, 0, 1), (0, 1 << 62, 64)])
def test_engine_mix_matches_single(im, ctx, graphs, limit, mark, cand):
    """limit: the one-workgroup greedy threshold (None = default, which
    runs one-workgroup rounds over candidate nodes; 0 forces the batched
    grid-wide rounds, 2^62 all rounds in one workgroup per job); mark: the
    chunk count above which the cover step marks touched chunks (0: always);
    cand: candidate chunks of the grid-wide rounds (0: two launches per
    round). The single-query runs use the defaults."""
    note(f"engine mix of {len(MIX)} queries vs single-query runs, greedy limit {limit} mark {mark} cand {cand}")
    names = ("greedy_wg_max_entries", "greedy_mark_min_chunks", "greedy_candidates_batch", "greedy_wg_cand_batch")
    old = [ctx.get_param(x) for x in names]
    # any schedule asked for is the batched one it names, not the
    # one-workgroup candidate rounds (which the default case runs)
    pinned = (limit, mark, cand) != (None, None, None)
    for x, v in zip(names, (limit, mark, cand, 0 if pinned else None)):
        if v is not None:
            ctx.set_param(x, v)
    try:
        res, _ = _engine(im, ctx, graphs, MIX)
    finally:
        for x, v in zip(names, old):
            ctx.set_param(x, v)
    for case, r in zip(MIX, res):
        note(f"compare {case}")
        _same(r, _single(graphs, case))


@pytest.mark.parametrize("lead", [16, 0, 3])
def test_engine_wg_candidate_batch_matches_single(im, ctx, graphs, lead):
    """The engine's batched Max-Coverage as one-workgroup rounds over
    candidate nodes, a workgroup per query, after `lead` grid-wide rounds
    shared by all queries, gives every query its single-query result."""
    note(f"engine mix with one-workgroup batched rounds, lead {lead}")
    names = ("greedy_wg_cand_batch", "greedy_wg_cand_grid_rounds")
    old = [ctx.get_param(x) for x in names]
    ctx.set_param("greedy_wg_cand_batch", 1 << 62)
    ctx.set_param("greedy_wg_cand_grid_rounds", lead)
    try:
        res, _ = _engine(im, ctx, graphs, MIX)
        single = [_single(graphs, case) for case in MIX]
    finally:
        for x, v in zip(names, old):
            ctx.set_param(x, v)
    for case, r, sr in zip(MIX, res, single):
        note(f"compare {case}")
        _same(r, sr)


def test_engine_wg_candidate_batch_flat_gains(im, ctx):
    """Flat gains (every RR set one node of an edgeless graph): some
    queries' cuts keep too few candidates and finish with grid-wide rounds
    of their own while the others go on in their workgroups."""
    note("engine one-workgroup batched rounds, flat gains")
    n = 200_000
    e = np.array([], np.uint32)
    dg = im.Graph(ctx, n, e, e, w_ic=np.array([], np.float32))
    cases = [(0, "dssa", 300, 0.2, 1), (0, "dssa", 40, 0.2, 2), (0, "ssa", 1200, 0.3, 3)]
    old = ctx.get_param("greedy_wg_cand_batch")
    ctx.set_param("greedy_wg_cand_batch", 1 << 62)
    try:
        eng = im.Engine(ctx, pool_budget_bytes=16 << 30, max_active=64)
        tickets = [eng.submit(dg, m, a, k, eps, 1.0 / n, key) for m, a, k, eps, key in cases]
        eng.run()
        res = [eng.result(t) for t in tickets]
        eng.close()
        single = [getattr(dg, a)(m, k, eps, 1.0 / n, key) for m, a, k, eps, key in cases]
    finally:
        ctx.set_param("greedy_wg_cand_batch", old)
    for r, sr in zip(res, single):
        _same(r, sr)


def test_engine_matches_oracle(im, ctx, graphs, oracle_lib):
    cases = [MIX[0], MIX[1], MIX[4], MIX[6]]
    note("engine vs oracle")
    res, _ = _engine(im, ctx, graphs, cases)
    for (name, model, algo, k, eps, key), (seeds, st) in zip(cases, res):
        g, _ = graphs[name]
        w = g.w_ic if model == 0 else g.w_lt
        og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
        oseeds, ost = getattr(og, algo)(k, eps, 1.0 / g.n, key)
        assert seeds.tolist() == oseeds.tolist()
        keys = ["iterations", "n_sets", "n_verify", "cov", "cov_c", "it_sets", "it_cov", "it_cov_c"]
        if algo == "dssa":
            keys.append("edges")
        for kk in keys:
            assert st[kk] == ost[kk], (kk, st[kk], ost[kk])


def test_alone_vs_mix_bit_identical(im, ctx, graphs):
    probe = MIX[5]
    note("alone vs mix")
    alone, _ = _engine(im, ctx, graphs, [probe])
    mixed, _ = _engine(im, ctx, graphs, MIX[::-1])
    _same(alone[0], mixed[MIX[::-1].index(probe)])


@pytest.mark.parametrize("budget,max_active", [(1, 64), (64 << 20, 3), (16 << 30, 1)])
def test_admission_limits(im, ctx, graphs, budget, max_active):
    cases = MIX[:6]
    note(f"admission budget={budget} max_active={max_active}")
    res, steps = _engine(im, ctx, graphs, cases, budget=budget, max_active=max_active)
    ref, ref_steps = _engine(im, ctx, graphs, cases)
    assert steps >= ref_steps
    for a, b in zip(res, ref):
        _same(a, b)


def test_engine_errors(im, ctx, graphs):
    g, dg = graphs["cl_small"]
    eng = im.Engine(ctx, max_active=4)
    note("engine argument errors")
    with pytest.raises(im.ImError):
        eng.submit(dg, 0, "ssa", 0, 0.1, 0.1, 0)
    with pytest.raises(im.ImError):
        eng.submit(dg, 0, "dssa", 5, 0.9, 0.1, 0)
    t = eng.submit(dg, 0, "dssa", 5, 0.1, 1.0 / g.n, 0)
    assert eng.poll(t) == 0
    with pytest.raises(im.ImError) as e:
        eng.result(t)
    assert e.value.status == -6
    eng.run()
    assert eng.poll(t) == 1
    seeds, st = eng.result(t)
    assert len(set(seeds.tolist())) == 5
    with pytest.raises(im.ImError):
        eng.poll(t)
    with pytest.raises(im.ImError):
        eng.result(12345)
    eng.close()


def test_engine_empty_step(im, ctx):
    eng = im.Engine(ctx)
    note("empty engine step")
    assert eng.step() == (0, 0)
    eng.run()
    eng.close()


def test_engine_estimate_queries(im, ctx, graphs, oracle_lib):
    """Influence-estimate queries ride the same fused verification passes
    as the SSA queries beside them and give im_estimate_inf's (and the
    oracle's) I_c and T exactly."""
    import numpy as np

    rng = np.random.default_rng(12)
    eng = im.Engine(ctx, max_active=32)
    cases = []
    for name, model in (("cl_small", 0), ("cl_small", 1), ("nethept", 0), ("rmat16", 1)):
        g, dg = graphs[name]
        for j, (size, tmax) in enumerate(((5, 1e9), (40, 1e9), (3, 3000.5), (g.n, 1e9))):
            S = np.arange(g.n) if size == g.n else rng.choice(g.n, size=size, replace=False)
            key = 500 + 10 * len(cases) + j
            cases.append((name, model, S, 0.15, 1e-3, tmax, key,
                          eng.submit_estimate(dg, model, S, 0.15, 1e-3, tmax, key)))
    ssa_t = [eng.submit(graphs[c[0]][1], c[1], c[2], c[3], c[4], 1.0 / graphs[c[0]][0].n, c[5])
             for c in MIX[:4]]
    note(f"engine with {len(cases)} estimate queries and {len(ssa_t)} SSA/D-SSA queries")
    eng.run()
    for name, model, S, e, d, tmax, key, t in cases:
        g, dg = graphs[name]
        seeds, st = eng.result(t)
        assert seeds.tolist() == np.asarray(S, dtype=np.uint32).tolist()
        ic, T = dg.estimate_inf(model, S, e, d, tmax, key)
        w = g.w_ic if model == 0 else g.w_lt
        oic, oT = oracle_lib.Graph(model, g.n, g.src, g.dst, w).estimate_inf(S, e, d, tmax, key)
        assert (st["cov_c"], st["i_c"]) == (T, ic) == (oT, oic), (name, model, len(S), tmax)
    for t, case in zip(ssa_t, MIX[:4]):
        _same(eng.result(t), _single(graphs, case))
    with pytest.raises(im.ImError):
        eng.submit_estimate(graphs["cl_small"][1], 0, [graphs["cl_small"][0].n], 0.1, 0.1, 10.0, 1)
    eng.close()
