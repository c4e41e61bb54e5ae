"""GPU test of the request loop: a Poisson stream over three resident graphs
with continuous batching; every query's seeds and integer statistics equal
those of the same query run alone (im_ssa / im_dssa)."""
import pytest

import synth
from gpu_util import note

pytestmark = pytest.mark.gpu


def test_serving_results_equal_alone():
    from paper_1605_07990_amd import binding as im
    from paper_1605_07990_amd import serve

    ctx = im.Context(0)
    graphs, shapes = {}, {}
    for name in ("cl_small", "nethept", "rmat16"):
        g = synth.make(name)
        graphs[name] = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic, w_lt=g.w_lt)
        shapes[name] = (g.n, g.w_ic is not None, g.w_lt is not None)
    reqs = serve.poisson_requests(shapes, qps=400.0, count=60, seed=5, k_max=200, algo=None, key_base=100)
    eng = im.Engine(ctx, pool_budget_bytes=256 << 20, max_active=16)
    note("serving 60 queries at 400 qps")
    out = serve.serve(eng, graphs, reqs, keep_results=True)
    note(f"p50 {out['p50_ms']:.2f} ms p99 {out['p99_ms']:.2f} ms max_active {out['max_active']}")
    assert out["max_active"] > 1  # requests overlapped on the device
    for r, (seeds, st) in zip(reqs, out["results"]):
        g = graphs[r.graph]
        fn = g.ssa if r.algo == im.IM_ALGO_SSA else g.dssa
        aseeds, ast = fn(r.model, r.k, r.eps, 1.0 / g.n, r.key)
        assert seeds.tolist() == aseeds.tolist(), r
        for key in ("iterations", "n_sets", "n_verify", "cov", "cov_c", "edges", "it_cov", "it_cov_c"):
            assert st[key] == ast[key], (r, key)
        assert st["i_hat"] == ast["i_hat"] and st["eps_t"] == ast["eps_t"]
    eng.close()
