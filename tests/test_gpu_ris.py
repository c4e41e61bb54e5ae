"""GPU parity of fixed-threshold RIS and of SSA with a caller's precision
split (the Section 4.2 presets) against the oracle: same seeds, same
integer trajectory."""
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
    c = im.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,model,k,eps,key", [("cl_small", 0, 10, 0.3, 4), ("cl_small", 1, 25, 0.3, 5),
                                                  ("nethept", 0, 200, 0.3, 6)])
def test_fixed_theta_ris_matches_oracle(im, ctx, oracle_lib, name, model, k, eps, key):
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    note(f"fixed-theta RIS {name} model={model} k={k} theta={im.ris_theta(g.n, k, eps, 1 / g.n):.0f}")
    seeds, st = dg.ris(model, k, eps, 1.0 / g.n, key)
    oseeds, ost = og.ris(k, eps, 1.0 / g.n, key)
    assert seeds.tolist() == oseeds.tolist()
    for f in ("n_sets", "cov", "edges"):
        assert st[f] == ost[f], f
    assert st["i_hat"] == ost["i_hat"]


@pytest.mark.parametrize("regime", ["small", "moderate", "large"])
@pytest.mark.parametrize("name,model,algo_k", [("cl_small", 0, 10), ("nethept", 1, 30)])
def test_ssa_preset_split_matches_oracle(im, ctx, oracle_lib, regime, name, model, algo_k):
    g = synth.make(name)
    w = g.w_ic if model == 0 else g.w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, w)
    eps = 0.1
    split = im.ssa_eps_preset(regime, eps)
    note(f"ssa split {regime} {split} {name}")
    seeds, st = dg.ssa_eps(model, algo_k, eps, *split, 1.0 / g.n, 11)
    oseeds, ost = og.ssa_eps(algo_k, eps, *split, 1.0 / g.n, 11)
    assert seeds.tolist() == oseeds.tolist()
    for f in ("iterations", "n_sets", "n_verify", "cov", "cov_c", "it_cov", "it_cov_c"):
        assert st[f] == ost[f], f
    with pytest.raises(im.ImError):
        dg.ssa_eps(model, algo_k, eps, 0.2, 0.2, 0.2, 1.0 / g.n, 11)
