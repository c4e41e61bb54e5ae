"""Oracle graph construction: thresholds and input validation (Section 2)."""
import numpy as np
import pytest


def test_ic_thresholds_closed_form(oracle_lib):
    src = np.array([1, 2, 3, 0], np.uint32)
    dst = np.array([0, 0, 0, 1], np.uint32)
    w = np.array([1.0, 0.5, 0.0, 0.25], np.float32)
    g = oracle_lib.Graph(oracle_lib.IC, 4, src, dst, w)
    assert g.thresholds().tolist() == [0xFFFFFFFF, 1 << 31, 0, 1 << 30]
    assert g.offsets().tolist() == [0, 3, 4, 4, 4]
    assert g.sources().tolist() == [1, 2, 3, 0]


def test_lt_thresholds_cumulative(oracle_lib):
    # node 0 has in-weights 0.25, 0.25, 0.5 -> cumulative 0.25, 0.5, 1.0
    src = np.array([1, 2, 3, 2], np.uint32)
    dst = np.array([0, 0, 0, 1], np.uint32)
    w = np.array([0.25, 0.25, 0.5, 0.125], np.float32)
    g = oracle_lib.Graph(oracle_lib.LT, 4, src, dst, w)
    assert g.thresholds().tolist() == [1 << 30, 1 << 31, 0xFFFFFFFF, 1 << 29]


def test_rejects_bad_input(oracle_lib):
    ok_src = np.array([1, 0], np.uint32)
    ok_dst = np.array([0, 1], np.uint32)
    w = np.array([0.5, 0.5], np.float32)
    oracle_lib.Graph(oracle_lib.IC, 2, ok_src, ok_dst, w)
    with pytest.raises(oracle_lib.OracleError):  # not sorted by dst
        oracle_lib.Graph(oracle_lib.IC, 2, ok_src[::-1], ok_dst[::-1], w)
    with pytest.raises(oracle_lib.OracleError):  # id out of range
        oracle_lib.Graph(oracle_lib.IC, 2, np.array([2, 0], np.uint32), ok_dst, w)
    with pytest.raises(oracle_lib.OracleError):  # repeated pair
        oracle_lib.Graph(oracle_lib.IC, 3, np.array([1, 1], np.uint32), np.array([0, 0], np.uint32), w)
    with pytest.raises(oracle_lib.OracleError):  # weight outside [0, 1]
        oracle_lib.Graph(oracle_lib.IC, 2, ok_src, ok_dst, np.array([1.5, 0.5], np.float32))
    with pytest.raises(oracle_lib.OracleError):  # LT weights into node 0 sum to 1.2
        oracle_lib.Graph(oracle_lib.LT, 3, np.array([1, 2], np.uint32), np.array([0, 0], np.uint32),
                         np.array([0.6, 0.6], np.float32))


def test_synthetic_lt_weights_are_valid(oracle_lib, synth_lib):
    for name in ("cl_small", "rmat12"):
        g = synth_lib.make(name)
        oracle_lib.Graph(oracle_lib.LT, g.n, g.src, g.dst, g.w_lt)
        oracle_lib.Graph(oracle_lib.IC, g.n, g.src, g.dst, g.w_ic)


def test_synthetic_ic_thresholds_shared_per_node(oracle_lib, synth_lib):
    """The weighted cascade (w(u,v) = 1/d_in(v)) gives every in-edge of a
    node the same threshold, which is what lets the device hold the compact
    IC form for the NetHEPT- and Twitter-shaped inputs; trivalency weights
    differ within a node and keep the {src, thr} records."""
    def shared(g):
        thr = oracle_lib.Graph(oracle_lib.IC, g.n, g.src, g.dst, g.w_ic).thresholds()
        same = g.dst[1:] == g.dst[:-1]
        return bool(np.all(thr[1:][same] == thr[:-1][same]))

    for name in ("cl_small", "nethept"):
        g = synth_lib.make(name)
        assert shared(g), name
        indeg = np.bincount(g.dst, minlength=g.n)
        w = 1.0 / indeg[g.dst]  # rounded down to fp32 by the generator
        assert np.all(g.w_ic <= w) and np.allclose(g.w_ic, w, rtol=1e-6, atol=0), name
    assert not shared(synth_lib.make("rmat12"))
