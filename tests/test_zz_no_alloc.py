"""im_coverage_range_noalloc (the stare step's coverage count with a fixed
per-GPU scratch array) against im_coverage_range through the C-ABI: two
calls in a row, the second with a smaller pool range, fewer seeds and a
smaller graph (so stale bitmap words and counts of the first call must not
leak into it), plus the argument limits."""
import numpy as np
import pytest

import synth
from gpu_util import note

pytestmark = pytest.mark.gpu


def test_noalloc_coverage_equals_coverage_range(oracle_lib):
    from paper_1605_07990_amd import binding as im

    ctx = im.Context(0)
    big = synth.make("rmat16")
    small = synth.make("cl_small")
    dg_big = im.Graph(ctx, big.n, big.src, big.dst, w_ic=big.w_ic)
    dg_small = im.Graph(ctx, small.n, small.src, small.dst, w_ic=small.w_ic)
    pb = im.Pool(dg_big, im.IM_IC, 3)
    pb.sample(20000)
    ps = im.Pool(dg_small, im.IM_IC, 4)
    ps.sample(3000)
    rng = np.random.default_rng(9)
    seeds_big = rng.choice(big.n, size=3000, replace=False).astype(np.uint32)
    seeds_small = rng.choice(small.n, size=7, replace=False).astype(np.uint32)

    note("no-alloc coverage: first call, 20000 sets, 3000 seeds, n = 2^16")
    a1 = pb.coverage_noalloc(seeds_big, 0, 20000)
    b1 = pb.coverage(seeds_big, 0, 20000)
    assert a1 == b1 and a1 > 0
    note("no-alloc coverage: second call, 1500 sets, 7 seeds, n = 2000")
    a2 = ps.coverage_noalloc(seeds_small, 500, 2000)
    b2 = ps.coverage(seeds_small, 500, 2000)
    assert a2 == b2
    # the oracle's count of the same range
    og = oracle_lib.Graph(0, small.n, small.src, small.dst, small.w_ic)
    op = oracle_lib.Pool(og, 4)
    op.extend(3000)
    assert a2 == op.coverage(seeds_small, 500, 2000)
    # an empty range and no seeds
    assert ps.coverage_noalloc(seeds_small, 700, 700) == 0
    assert ps.coverage_noalloc(np.zeros(0, np.uint32), 0, 3000) == 0
    # limits and bad seeds are errors, not faults
    with pytest.raises(im.ImError):
        ps.coverage_noalloc(np.array([small.n], np.uint32), 0, 10)
    with pytest.raises(im.ImError):
        ps.coverage_noalloc(np.zeros(70000, np.uint32), 0, 10)
    with pytest.raises(im.ImError):
        ps.coverage_noalloc(seeds_small, 0, 3001)
    ctx.close()
