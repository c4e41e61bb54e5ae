"""Host logic of the request loop: the seeded Poisson request stream."""
import math

import numpy as np


def _serve():
    # host code only: importing the binding module loads no library
    from paper_1605_07990_amd import serve
    return serve


def test_stream_is_seeded_and_shaped():
    serve = _serve()
    graphs = {"a": (2000, True, True), "b": (15233, True, False)}
    r1 = serve.poisson_requests(graphs, qps=50.0, count=4000, seed=7, algo=None)
    r2 = serve.poisson_requests(graphs, qps=50.0, count=4000, seed=7, algo=None)
    assert r1 == r2
    arr = np.array([r.arrival for r in r1])
    assert np.all(np.diff(arr) > 0)
    # exponential inter-arrivals at rate 50: mean 1/50 within a few standard errors
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 0.02) < 4 * 0.02 / math.sqrt(len(gaps))
    # k log-uniform on [1, 1000]: ln k roughly uniform, within bounds
    ks = np.array([r.k for r in r1])
    assert ks.min() >= 1 and ks.max() <= 1000
    assert abs(np.log(ks).mean() - math.log(1000) / 2) < 0.15
    assert {r.eps for r in r1} == {0.05, 0.1, 0.2}
    assert {r.algo for r in r1} == {0, 1}
    # graph b has no LT weights: only IC is drawn for it
    assert {r.model for r in r1 if r.graph == "b"} == {0}
    assert {r.model for r in r1 if r.graph == "a"} == {0, 1}
    assert [r.key for r in r1] == list(range(4000))


def test_k_clipped_to_n():
    serve = _serve()
    rs = serve.poisson_requests({"tiny": (5, True, True)}, qps=10.0, count=500, seed=1)
    assert max(r.k for r in rs) == 5
