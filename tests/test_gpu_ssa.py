"""GPU parity of the full SSA (Algorithm 1) and D-SSA (Algorithm 4) runs:
same seed sets, same integer trajectory (|R|, Cov, Cov_c / T per
iteration), FP64 estimates equal to 1e-12 relative. Includes the two
full-size workloads: the NetHEPT-shaped IC SSA query (k=50, eps=0.1,
delta=1/n, key 0) and the R-MAT-20 LT D-SSA query (k=100)."""
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


def _compare(st, ost, algo):
    keys = ["iterations", "stopped_by_cap", "n_sets", "n_verify", "cov", "cov_c", "it_sets", "it_cov", "it_cov_c"]
    if algo == "dssa":
        # SSA's verification sets stop at the first seed hit on the GPU, so
        # only D-SSA's edge count is comparable
        keys.append("edges")
    for key in keys:
        assert st[key] == ost[key], (key, st[key], ost[key])
    for key in ("i_hat", "i_c", "eps1", "eps2", "eps3", "eps_t"):
        assert st[key] == pytest.approx(ost[key], rel=1e-12, abs=1e-300), key
    for a, b in zip(st["it_eps_t"], ost["it_eps_t"]):
        assert a == pytest.approx(b, rel=1e-12)


@pytest.mark.parametrize("algo,name,model,k,eps,key", [
    ("ssa", "nethept", 0, 50, 0.1, 0),
    ("dssa", "nethept", 0, 50, 0.1, 0),
    ("ssa", "nethept", 0, 1, 0.1, 2),
    ("ssa", "cl_small", 1, 10, 0.2, 3),
    ("dssa", "cl_small", 1, 10, 0.2, 3),
    ("ssa", "rmat12", 0, 25, 0.1, 5),
    ("dssa", "rmat16", 1, 40, 0.1, 6),
    ("dssa", "rmat20", 1, 100, 0.1, 0),
])
def test_run_matches_oracle(im, ctx, oracle_lib, algo, name, model, k, eps, key):
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    note(f"{algo} {name} model={model} k={k} eps={eps} key={key}")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    delta = 1.0 / g.n
    seeds, st = getattr(dg, algo)(model, k, eps, delta, key)
    oseeds, ost = getattr(og, algo)(k, eps, delta, key)
    assert seeds.tolist() == oseeds.tolist()
    _compare(st, ost, algo)


@pytest.mark.parametrize("algo,model,k,key", [("ssa", 0, 20, 1), ("dssa", 0, 20, 2), ("ssa", 1, 15, 3),
                                               ("dssa", 1, 15, 4)])
def test_weighted_runs_match_oracle(im, ctx, oracle_lib, algo, model, k, key):
    """Targeted sources (WRIS, Section 7.3): seeds, trajectories and the
    estimates, which scale by the total node weight, equal the oracle's;
    the same query through the engine gives the same result."""
    g = synth.make("cl_20k")
    w = g.w_ic if model == 0 else g.w_lt
    wts = synth.node_weights(g.n, 0.2, 2.1, 5)
    note(f"weighted {algo} cl_20k model={model} k={k} key={key}")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    dg.set_source_weights(wts)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w, node_weights=wts)
    delta = 1.0 / g.n
    seeds, st = getattr(dg, algo)(model, k, 0.1, delta, key)
    oseeds, ost = getattr(og, algo)(k, 0.1, delta, key)
    assert seeds.tolist() == oseeds.tolist()
    _compare(st, ost, algo)
    assert st["i_hat"] == pytest.approx(float(wts.sum()) * st["cov"] / (st["it_sets"][-1]), rel=1e-12)
    eng = im.Engine(ctx, pool_budget_bytes=1 << 30, max_active=4)
    t = eng.submit(dg, model, algo, k, 0.1, delta, key)
    eng.run()
    eseeds, est = eng.result(t)
    eng.close()
    assert eseeds.tolist() == seeds.tolist()
    _compare(est, ost, algo)
    dg.close()


def test_query_errors(im, ctx):
    g = synth.make("cl_small")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    note("query argument errors")
    for args in ((0, 0, 0.1, 0.1), (0, g.n + 1, 0.1, 0.1), (0, 5, 0.0, 0.1), (0, 5, 0.7, 0.1), (0, 5, 0.1, 1.0),
                 (1, 5, 0.1, 0.1)):
        with pytest.raises(im.ImError):
            dg.ssa(*args, 0)
        with pytest.raises(im.ImError):
            dg.dssa(*args, 0)


@pytest.mark.parametrize("name,model,k", [("rmat16", 1, 40), ("nethept", 0, 50), ("rmat20", 1, 100)])
def test_dssa_speculation_changes_nothing(im, ctx, name, model, k):
    """Drawing the next iteration's sets on the second stream while the
    current one is covered gives the same run as drawing them afterwards
    (IC runs with their minimum draw off, which side sampling needs)."""
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    note(f"dssa speculation on/off {name}")
    old = ctx.get_param("dssa_speculate"), ctx.get_param("dssa_ic_min_draw")
    try:
        ctx.set_param("dssa_ic_min_draw", 0)
        out = {}
        for flag in (1, 0):
            ctx.set_param("dssa_speculate", flag)
            out[flag] = [dg.dssa(model, k, 0.1, 1.0 / g.n, key) for key in (0, 1, 2)]
    finally:
        ctx.set_param("dssa_speculate", old[0])
        ctx.set_param("dssa_ic_min_draw", old[1])
    for (s1, st1), (s0, st0) in zip(out[1], out[0]):
        assert s1.tolist() == s0.tolist()
        for key in ("iterations", "n_sets", "cov", "cov_c", "edges", "it_cov", "it_cov_c", "eps_t", "i_hat"):
            assert st1[key] == st0[key], key


@pytest.mark.parametrize("name,k", [("rmat16", 40), ("cl_small", 5), ("rmat20", 100)])
@pytest.mark.parametrize("ahead", [1, 2, 64])
def test_dssa_draw_ahead_changes_nothing(im, ctx, oracle_lib, name, k, ahead):
    """LT D-SSA drawing later iterations' sets early gives the oracle's run,
    edges included (they count only the sets the query used)."""
    g = synth.make(name)
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_lt=g.w_lt)
    og = oracle_lib.Graph(1, g.n, g.src, g.dst, g.w_lt)
    note(f"dssa draw-ahead {ahead} {name} k={k}")
    old = ctx.get_param("dssa_draw_ahead"), ctx.get_param("dssa_speculate")
    try:
        ctx.set_param("dssa_draw_ahead", ahead)
        for spec in (1, 0):
            ctx.set_param("dssa_speculate", spec)
            for key in (0, 3):
                seeds, st = dg.dssa(1, k, 0.1, 1.0 / g.n, key)
                oseeds, ost = og.dssa(k, 0.1, 1.0 / g.n, key)
                assert seeds.tolist() == oseeds.tolist()
                for kk in ("iterations", "n_sets", "cov", "cov_c", "edges", "it_sets", "it_cov", "it_cov_c"):
                    assert st[kk] == ost[kk], (kk, st[kk], ost[kk])
    finally:
        ctx.set_param("dssa_draw_ahead", old[0])
        ctx.set_param("dssa_speculate", old[1])


@pytest.mark.parametrize("name", ["nethept", "cl_mid", "rmat16"])
@pytest.mark.parametrize("min_draw", [262144, 0, 4096])
def test_dssa_ic_draw_ahead_matches_oracle(im, ctx, oracle_lib, name, min_draw):
    """IC D-SSA drawing later iterations' sets with the first ones (up to
    the largest 2 N_t within the minimum draw) gives the oracle's run, edges
    included: a run that stops inside a block drawn ahead counts only the
    in-edges of the sets it used. k = 1 (no greedy rounds, no helpers) and
    k = 20 (helpers covering drawn-ahead iterations)."""
    g = synth.make(name)
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    note(f"dssa IC min draw {min_draw} {name}")
    old = ctx.get_param("dssa_ic_min_draw")
    try:
        ctx.set_param("dssa_ic_min_draw", min_draw)
        for k, key, eps in ((1, 0, 0.1), (1, 7, 0.2), (1, 11, 0.05), (20, 3, 0.1), (20, 5, 0.2)):
            seeds, st = dg.dssa(0, k, eps, 1.0 / g.n, key)
            oseeds, ost = og.dssa(k, eps, 1.0 / g.n, key)
            assert seeds.tolist() == oseeds.tolist(), (k, key)
            _compare(st, ost, "dssa")
    finally:
        ctx.set_param("dssa_ic_min_draw", old)


@pytest.mark.parametrize("algo,name,model,k", [("dssa", "rmat16", 1, 40), ("ssa", "nethept", 0, 50),
                                               ("dssa", "rmat20", 1, 100)])
def test_wg_candidate_rounds_runs_match_oracle(im, ctx, oracle_lib, algo, name, model, k):
    """Whole SSA / D-SSA runs with every Max-Coverage in one workgroup over
    candidate nodes give the oracle's runs."""
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    note(f"{algo} with one-workgroup candidate rounds {name} k={k}")
    old = ctx.get_param("greedy_wg_cand_max_entries")
    ctx.set_param("greedy_wg_cand_max_entries", 1 << 62)
    try:
        for key in (0, 3):
            seeds, st = getattr(dg, algo)(model, k, 0.1, 1.0 / g.n, key)
            oseeds, ost = getattr(og, algo)(k, 0.1, 1.0 / g.n, key)
            assert seeds.tolist() == oseeds.tolist()
            _compare(st, ost, algo)
    finally:
        ctx.set_param("greedy_wg_cand_max_entries", old)


@pytest.mark.parametrize("name,model,k", [("rmat16", 1, 40), ("cl_small", 1, 5), ("nethept", 0, 50),
                                          ("rmat20", 1, 100)])
@pytest.mark.parametrize("ahead", [0, 1, 2, 3])
def test_dssa_greedy_ahead_matches_oracle(im, ctx, oracle_lib, name, model, k, ahead):
    """D-SSA covering later iterations on helper contexts while the current
    one is covered gives the oracle's run, with and without drawing ahead and
    speculation (the helpers' results are used or dropped, never changed)."""
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    note(f"dssa greedy ahead {ahead} {name} k={k}")
    names = ("dssa_greedy_ahead", "dssa_draw_ahead", "dssa_speculate")
    old = [ctx.get_param(x) for x in names]
    try:
        ctx.set_param("dssa_greedy_ahead", ahead)
        for draw, spec in ((4, 1), (1, 0), (64, 1)):
            ctx.set_param("dssa_draw_ahead", draw)
            ctx.set_param("dssa_speculate", spec)
            for key in (0, 3):
                seeds, st = dg.dssa(model, k, 0.1, 1.0 / g.n, key)
                oseeds, ost = og.dssa(k, 0.1, 1.0 / g.n, key)
                assert seeds.tolist() == oseeds.tolist(), (draw, spec, key)
                _compare(st, ost, "dssa")
    finally:
        for x, v in zip(names, old):
            ctx.set_param(x, v)


def test_dssa_dropped_covers_outlive_the_run(im, oracle_lib):
    """A run that stops before a later iteration's cover is done returns
    without waiting for it. Later runs that need the helper, a graph freed
    right after such runs, im_ctx_sync and the context's own free all wait
    for those covers, and every run gives the oracle's result."""
    g = synth.make("rmat20")
    og = oracle_lib.Graph(1, g.n, g.src, g.dst, g.w_lt)
    keys = (0, 1, 2, 3)
    want = {key: og.dssa(100, 0.1, 1.0 / g.n, key) for key in keys}
    ctx2 = im.Context(0)
    try:
        for rep in range(2):
            note(f"dropped covers, graph lifetime {rep}")
            dg = im.Graph(ctx2, g.n, g.src, g.dst, w_lt=g.w_lt)
            for key in keys:
                seeds, st = dg.dssa(1, 100, 0.1, 1.0 / g.n, key)
                oseeds, ost = want[key]
                assert seeds.tolist() == oseeds.tolist(), (rep, key)
                _compare(st, ost, "dssa")
            dg.close()  # right after runs whose dropped covers may still run
        dg = im.Graph(ctx2, g.n, g.src, g.dst, w_lt=g.w_lt)
        seeds, _ = dg.dssa(1, 100, 0.1, 1.0 / g.n, 0)
        ctx2.sync()
        assert seeds.tolist() == want[0][0].tolist()
        seeds, _ = dg.dssa(1, 100, 0.1, 1.0 / g.n, 1)
        assert seeds.tolist() == want[1][0].tolist()
        dg.close()
    finally:
        ctx2.close()
