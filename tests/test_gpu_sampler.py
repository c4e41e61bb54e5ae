"""GPU parity of RR-set sampling (Definition 2): pools from the HIP sampler
must equal the oracle's bit for bit (offsets exactly, every set as a sorted
list), across graph shapes, both models, the LDS bitmap / LDS hash / long
paths, ragged batches and appends."""
import numpy as np
import pytest

import synth
from gpu_util import assert_pool_equal, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def im():
    from paper_1605_07990_amd import binding
    return binding


@pytest.fixture(scope="module")
def ctx(im):
    return im.Context(0)


def _graphs(im, ctx, oracle_lib, name, w_ic=None, w_lt=None):
    g = synth.make(name)
    w_ic = g.w_ic if w_ic is None else w_ic
    w_lt = g.w_lt if w_lt is None else w_lt
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w_ic, w_lt=w_lt)
    ogs = {}
    if w_ic is not None:
        ogs[0] = oracle_lib.Graph(0, g.n, g.src, g.dst, w_ic)
    if w_lt is not None:
        ogs[1] = oracle_lib.Graph(1, g.n, g.src, g.dst, w_lt)
    return g, dg, ogs


@pytest.mark.parametrize("name,model,count,key", [
    ("cl_small", 0, 20000, 1),
    ("cl_small", 1, 20000, 2),
    ("nethept", 0, 30000, 0),
    ("nethept", 1, 30000, 5),
    ("rmat12", 0, 20000, 3),
    ("rmat12", 1, 20000, 4),
    ("rmat16", 1, 20000, 6),
    ("rmat16", 0, 3000, 7),
])
def test_pool_matches_oracle(im, ctx, oracle_lib, name, model, count, key):
    note(f"pool parity {name} model={model} count={count} key={key}")
    g, dg, ogs = _graphs(im, ctx, oracle_lib, name)
    pool = im.Pool(dg, model, key)
    pool.sample(count)
    op = oracle_lib.Pool(ogs[model], key)
    op.extend(count)
    assert pool.count == count
    assert_pool_equal(pool, op, 0, count)


@pytest.mark.parametrize("model", [0, 1])
def test_appends_and_ragged_batches(im, ctx, oracle_lib, model):
    note(f"ragged appends model={model}")
    g, dg, ogs = _graphs(im, ctx, oracle_lib, "cl_small")
    pool = im.Pool(dg, model, 11)
    op = oracle_lib.Pool(ogs[model], 11)
    total = 0
    for c in (1, 0, 63, 64, 65, 255, 1023, 1025, 4097, 3):
        pool.sample(c)
        total += c
    op.extend(total)
    assert pool.count == total
    assert_pool_equal(pool, op, 0, total)
    assert_pool_equal(pool, op, 100, 2000)


def test_long_path_ic_ancestors(im, ctx, oracle_lib):
    # p = 1 everywhere: RR sets are whole ancestor sets, far above the LDS
    # queue, so every non-trivial sample takes the global long path.
    g = synth.make("cl_20k")
    w = np.ones(g.m, np.float32)
    note("long path IC p=1 cl_20k")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, w)
    pool = im.Pool(dg, 0, 21)
    pool.sample(300)
    op = oracle_lib.Pool(og, 21)
    op.extend(300)
    assert_pool_equal(pool, op, 0, 300)
    assert int(np.diff(op.offsets()).max()) > 4 * 1024  # sets far above the LDS queue


def test_long_path_lt_walks(im, ctx, oracle_lib):
    # a path 0 -> 1 -> ... -> n-1 with w = 1: the walk from v has v+1 nodes,
    # so most walks outgrow the per-sample staging region.
    n = 3000
    src = np.arange(0, n - 1, dtype=np.uint32)
    dst = np.arange(1, n, dtype=np.uint32)
    w = np.ones(n - 1, np.float32)
    note("long path LT path graph")
    dg = im.Graph(ctx, n, src, dst, w_lt=w)
    og = oracle_lib.Graph(1, n, src, dst, w)
    pool = im.Pool(dg, 1, 22)
    pool.sample(700)
    op = oracle_lib.Pool(og, 22)
    op.extend(700)
    assert_pool_equal(pool, op, 0, 700)


def test_hash_visited_large_n(im, ctx, oracle_lib):
    # n > 65536 uses the LDS hash; IC on an R-MAT-20 graph
    g, dg, ogs = _graphs(im, ctx, oracle_lib, "rmat20")
    note("rmat20 IC hash path")
    pool = im.Pool(dg, 0, 9)
    pool.sample(2000)
    op = oracle_lib.Pool(ogs[0], 9)
    op.extend(2000)
    assert_pool_equal(pool, op, 0, 2000)


def test_edge_cases(im, ctx, oracle_lib):
    note("edge cases: edgeless graph, single node, zero-weight edges")
    # no edges: every set is its source
    n = 50
    e = np.array([], np.uint32)
    dg = im.Graph(ctx, n, e, e, w_ic=np.array([], np.float32), w_lt=np.array([], np.float32))
    for model in (0, 1):
        og = oracle_lib.Graph(model, n, e, e, np.array([], np.float32))
        pool = im.Pool(dg, model, 3)
        pool.sample(500)
        op = oracle_lib.Pool(og, 3)
        op.extend(500)
        assert_pool_equal(pool, op, 0, 500)
    # one node
    d1 = im.Graph(ctx, 1, e, e, w_ic=np.array([], np.float32))
    p1 = im.Pool(d1, 0, 0)
    p1.sample(10)
    off, nodes = p1.read()
    assert off.tolist() == list(range(11)) and nodes.tolist() == [0] * 10
    # zero weights: singletons
    g = synth.make("cl_small")
    z = np.zeros(g.m, np.float32)
    dz = im.Graph(ctx, g.n, g.src, g.dst, w_ic=z, w_lt=z)
    for model in (0, 1):
        pool = im.Pool(dz, model, 4)
        pool.sample(1000)
        off, _ = pool.read()
        assert np.all(np.diff(off) == 1)



def _mixed_degree_graph(n, seed):
    """In-degrees alternating between 0-3 and 20 or more, so that 8-record
    windows around small in-lists take records of the neighbouring nodes;
    edges in (dst, src) order; LT weights per node sum to 0.6-1.0 (the
    live-edge reading of the LT model)."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for v in range(n):
        d = 20 + v % 13 if v % 5 == 0 else v % 4
        us = np.sort(rng.choice(np.delete(np.arange(n), v), size=min(d, n - 1), replace=False))
        src += us.tolist()
        dst += [v] * len(us)
    src = np.array(src, np.uint32)
    dst = np.array(dst, np.uint32)
    w_ic = rng.uniform(0.05, 1.0, len(src)).astype(np.float32)
    w_lt = np.zeros(len(src), np.float32)
    for v in range(n):
        idx = np.nonzero(dst == v)[0]
        if len(idx):
            r = rng.uniform(0.1, 1.0, len(idx))
            w_lt[idx] = (r / r.sum() * rng.uniform(0.6, 1.0)).astype(np.float32)
    return src, dst, w_ic, w_lt


def test_few_edges_and_neighbouring_windows(im, ctx, oracle_lib):
    """Edge arrays of fewer than eight records (the LT pick cannot take a full
    window there) and in-lists shorter than a window next to long ones (the
    window and the IC 4-edge groups reach into neighbouring nodes' records,
    which must be skipped)."""
    cases = [
        ("one edge", 3, np.array([1], np.uint32), np.array([0], np.uint32)),
        ("cycle of five", 5, np.array([1, 2, 3, 4, 0], np.uint32), np.array([0, 1, 2, 3, 4], np.uint32)),
        ("seven edges", 6, np.array([1, 2, 0, 3, 4, 5, 1], np.uint32), np.array([0, 0, 1, 2, 2, 3, 4], np.uint32)),
    ]
    for label, n, src, dst in cases:
        note(f"few edges: {label}")
        m = len(src)
        w_ic = np.full(m, 0.8, np.float32)
        w_lt = np.zeros(m, np.float32)
        for v in range(n):
            idx = np.nonzero(dst == v)[0]
            if len(idx):
                w_lt[idx] = np.float32(0.9 / len(idx))
        dg = im.Graph(ctx, n, src, dst, w_ic=w_ic, w_lt=w_lt)
        for model, w in ((0, w_ic), (1, w_lt)):
            og = oracle_lib.Graph(model, n, src, dst, w)
            pool = im.Pool(dg, model, 11 + model)
            pool.sample(2000)
            op = oracle_lib.Pool(og, 11 + model)
            op.extend(2000)
            assert_pool_equal(pool, op, 0, 2000)
    note("neighbouring windows: mixed in-degrees")
    n = 400
    src, dst, w_ic, w_lt = _mixed_degree_graph(n, 5)
    dg = im.Graph(ctx, n, src, dst, w_ic=w_ic, w_lt=w_lt)
    for model, w in ((0, w_ic), (1, w_lt)):
        og = oracle_lib.Graph(model, n, src, dst, w)
        pool = im.Pool(dg, model, 21 + model)
        pool.sample(5000)
        op = oracle_lib.Pool(og, 21 + model)
        op.extend(5000)
        assert_pool_equal(pool, op, 0, 5000)

def test_weighted_sources(im, ctx, oracle_lib):
    g = synth.make("cl_small")
    wts = synth.node_weights(g.n, 0.2, 2.1, 5)
    note("weighted sources (WRIS)")
    for model, w in ((0, g.w_ic), (1, g.w_lt)):
        dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w if model == 0 else None, w_lt=w if model == 1 else None)
        dg.set_source_weights(wts)
        og = oracle_lib.Graph(model, g.n, g.src, g.dst, w, node_weights=wts)
        pool = im.Pool(dg, model, 8)
        pool.sample(5000)
        op = oracle_lib.Pool(og, 8)
        op.extend(5000)
        assert_pool_equal(pool, op, 0, 5000)


def test_stream_mismatch_and_bad_graphs(im, ctx):
    note("error paths")
    g = synth.make("cl_small")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    pool = im.Pool(dg, 0, 1)
    with pytest.raises(im.ImError) as e:
        pool.sample(10, key=2)
    assert e.value.status == -5
    with pytest.raises(im.ImError):
        im.Pool(dg, 1, 1)  # no LT weights
    with pytest.raises(im.ImError) as e:
        im.Graph(ctx, 3, np.array([1, 2], np.uint32), np.array([0, 0], np.uint32),
                 w_lt=np.array([0.7, 0.7], np.float32))
    assert e.value.status == -3
    with pytest.raises(im.ImError) as e:
        im.Graph(ctx, 3, np.array([2, 1], np.uint32), np.array([0, 0], np.uint32),
                 w_ic=np.array([0.5, 0.5], np.float32))
    assert e.value.status == -1


@pytest.mark.parametrize("n,deg,p", [(3000, 24, 0.5), (6000, 40, 1.0), (12000, 20, 1.0)])
def test_heavy_ic_samples_workgroup_tier(im, ctx, oracle_lib, n, deg, p):
    """IC samples that examine more edges than one wave takes on go to the
    workgroup tier (1024 threads, LDS queue of 8192, LDS hash of 16384);
    those with more nodes than that go on to the long path. Every tier must
    give the oracle's sets."""
    rng = np.random.default_rng(n + deg)
    dst = np.repeat(np.arange(n, dtype=np.uint32), deg)
    src = rng.integers(0, n, size=n * deg).astype(np.uint32)
    keep = src != dst
    pairs = np.unique(np.stack([dst[keep], src[keep]], axis=1), axis=0)
    g = synth.from_edges(f"heavy{n}", n, pairs[:, 1], pairs[:, 0],
                         w_ic=np.full(pairs.shape[0], p, dtype=np.float32))
    note(f"heavy IC samples n={n} m={g.m} p={p}")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    count = 300
    pool = im.Pool(dg, 0, 17)
    pool.sample(count)
    op = oracle_lib.Pool(og, 17)
    op.extend(count)
    assert_pool_equal(pool, op, 0, count)
    # hits mode through the same tiers: Estimate-Inf's stopping index
    seeds = np.array([0, 1], dtype=np.uint32)
    assert dg.estimate_inf(0, seeds, 0.2, 0.1, 5000.0, 99) == og.estimate_inf(seeds, 0.2, 0.1, 5000.0, 99)


@pytest.mark.parametrize("name", ["cl_mid", "heavy6000"])
def test_plain_launches_and_fused_pools_match_oracle(im, ctx, oracle_lib, name):
    """The plain IC launch (static assignment, no workgroup tiers: samples
    that outgrow a wave's LDS go to the long path) and the fused multi-pool
    draw (im_sample_rr_multi: several pools' samples in one work queue) give
    the oracle's sets, including heavy samples and ragged counts."""
    if name == "cl_mid":
        g = synth.make("cl_mid")
    else:
        n, deg = 6000, 40
        rng = np.random.default_rng(n + deg)
        dst = np.repeat(np.arange(n, dtype=np.uint32), deg)
        src = rng.integers(0, n, size=n * deg).astype(np.uint32)
        keep = src != dst
        pairs = np.unique(np.stack([dst[keep], src[keep]], axis=1), axis=0)
        g = synth.from_edges(f"heavy{n}", n, pairs[:, 1], pairs[:, 0],
                             w_ic=np.full(pairs.shape[0], 0.3, dtype=np.float32))
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, g.w_ic)
    counts = [3000, 0, 5000, 1] if name == "cl_mid" else [300, 0, 257, 1]
    keys = [21, 22, 23, 24]
    note(f"fused pools {name} counts={counts}")
    pools = [im.Pool(dg, 0, key) for key in keys]
    im.Pool.sample_multi(pools, counts)
    im.Pool.sample_multi(pools, [7, 65, 0, 300])  # appends after the first batch
    for p, key, c in zip(pools, keys, [c + d for c, d in zip(counts, [7, 65, 0, 300])]):
        op = oracle_lib.Pool(og, key)
        op.extend(c)
        assert p.count == c
        if c:
            assert_pool_equal(p, op, 0, c)
    note(f"plain launches {name}")
    ctx.set_param("ic_plain", 1)
    try:
        for key, c in zip(keys, counts):
            p = im.Pool(dg, 0, key)
            p.sample(c)
            op = oracle_lib.Pool(og, key)
            op.extend(c)
            if c:
                assert_pool_equal(p, op, 0, c)
        seeds = np.array([0, 1], dtype=np.uint32)
        assert dg.estimate_inf(0, seeds, 0.2, 0.1, 5000.0, 99) == og.estimate_inf(seeds, 0.2, 0.1, 5000.0, 99)
    finally:
        ctx.set_param("ic_plain", 0)


def test_fused_pools_argument_errors(im, ctx):
    g = synth.make("cl_small")
    dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=g.w_ic, w_lt=g.w_lt)
    a, b = im.Pool(dg, 0, 1), im.Pool(dg, 1, 2)
    with pytest.raises(im.ImError) as e:
        im.Pool.sample_multi([a, b], [5, 5])  # mixed models
    assert e.value.status == -5
    with pytest.raises(im.ImError) as e:
        im.Pool.sample_multi([a, a], [5, 5])  # a pool twice
    assert e.value.status == -1
    assert a.count == 0 and b.count == 0


@pytest.mark.parametrize("name", ["nethept", "heavy6000", "rmat12", "nethept_mixed", "nethept_off"])
def test_compact_ic_form_matches_records_and_oracle(im, ctx, oracle_lib, name):
    """Graphs whose IC in-edges of each node share one threshold (weighted
    cascade, a constant p) hold the compact IC form (graph info bit 2) and
    IC draws read it; the sets must be the oracle's and the same as from the
    {src, thr} records (IM_PARAM_IC_COMPACT = 0), in pool and hits mode.
    Graphs with mixed thresholds (trivalency; weighted cascade with one
    weight changed) hold no compact form, nor does one loaded while the
    parameter is 0."""
    if name == "heavy6000":
        n, deg = 6000, 40
        rng = np.random.default_rng(n + deg)
        dst = np.repeat(np.arange(n, dtype=np.uint32), deg)
        src = rng.integers(0, n, size=n * deg).astype(np.uint32)
        keep = src != dst
        pairs = np.unique(np.stack([dst[keep], src[keep]], axis=1), axis=0)
        g = synth.from_edges(name, n, pairs[:, 1], pairs[:, 0], w_ic=np.full(pairs.shape[0], 0.3, dtype=np.float32))
        w, uniform, count = g.w_ic, True, 300
    else:
        g = synth.make(name.split("_")[0])
        w, uniform, count = g.w_ic, name in ("nethept", "heavy6000"), 20000
        if name == "nethept_mixed":
            # one in-edge of a node with several gets another weight
            indeg = np.bincount(g.dst, minlength=g.n)
            e = int(np.flatnonzero(indeg[g.dst] > 3)[0])
            w = g.w_ic.copy()
            w[e] = np.float32(min(1.0, float(w[e]) * 2.0))
            uniform = False
    ctx.set_param("ic_compact", 0 if name == "nethept_off" else 1)
    try:
        dg = im.Graph(ctx, g.n, g.src, g.dst, w_ic=w)
    finally:
        ctx.set_param("ic_compact", 1)
    og = oracle_lib.Graph(0, g.n, g.src, g.dst, w)
    assert bool(dg.info()[2] & 4) == uniform
    note(f"compact IC form {name} uniform={uniform} count={count}")
    op = oracle_lib.Pool(og, 31)
    op.extend(count)
    seeds = np.array([0, 1], dtype=np.uint32)
    est = og.estimate_inf(seeds, 0.2, 0.1, 5000.0, 99)
    assert ctx.get_param("ic_compact") == 1
    try:
        for compact in (1, 0):
            ctx.set_param("ic_compact", compact)
            pool = im.Pool(dg, 0, 31)
            pool.sample(count // 3)
            pool.sample(count - count // 3)  # an append
            assert_pool_equal(pool, op, 0, count)
            assert dg.estimate_inf(0, seeds, 0.2, 0.1, 5000.0, 99) == est
    finally:
        ctx.set_param("ic_compact", 1)
