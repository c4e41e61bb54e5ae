"""Host arithmetic of bench.py's roofline object: algorithmic bytes per
launch over the mean launch time, against the 8 TB/s HBM peak, with the IC
count in both the record form (8 B per examined in-edge) and the compact
form (4 B), and no counter traffic for launches the committed counter runs
did not measure."""
import pytest

import bench


def _kt(**kw):
    kt = {"sample_launches": 4, "sample_steps": 10_000_000, "sample_nodes": 400_000, "sample_sets": 20_000,
          "sample_ms": 8.0, "group_launches": 0}
    kt.update(kw)
    return kt


def test_ic_bytes_counts_each_term():
    # 16 B node record or offsets, 4 B pool write, 4 B visited check per newly
    # reached node, 8 B per set offset, 8 (or 4) B per examined in-edge
    assert bench.ic_bytes(100, 10, 2) == 16 * 10 + 8 * 100 + 4 * 8 + 4 * 10 + 8 * 2
    assert bench.ic_bytes(100, 10, 2, edge_bytes=4) == 16 * 10 + 4 * 100 + 4 * 8 + 4 * 10 + 8 * 2
    assert bench.ic_bytes(0, 3, 3) == 16 * 3 + 4 * 3 + 8 * 3  # every node a source: no visited checks
    assert bench.lt_bytes(7, 2) == 36 * 7 + 16


@pytest.mark.parametrize("compact", [False, True])
def test_ic_roofline_rate_and_fraction(compact):
    kt = _kt()
    r = bench.roofline(kt, 0, compact=compact)
    per_launch = bench.ic_bytes(kt["sample_steps"], kt["sample_nodes"], kt["sample_sets"]) / 4
    gbs = per_launch / 2e-3 / 1e9  # 8 ms over 4 launches
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(gbs, abs=0.01)
    assert r["frac"] == pytest.approx(gbs / 8000.0, abs=1e-5)
    assert r["algorithmic_bytes_per_launch"] == round(per_launch)
    assert r["traffic"] is None
    if compact:
        cb = bench.ic_bytes(kt["sample_steps"], kt["sample_nodes"], kt["sample_sets"], edge_bytes=4) / 4
        assert r["compact_form"]["algorithmic_bytes_per_launch"] == round(cb)
        assert r["compact_form"]["achieved"] == pytest.approx(cb / 2e-3 / 1e9, abs=0.01)
        assert r["compact_form"]["achieved"] < r["achieved"]
    else:
        assert "compact_form" not in r


def test_lt_roofline_and_traffic_gate():
    kt = _kt()
    r = bench.roofline(kt, 1)
    assert r["algorithmic_bytes_per_launch"] == round(bench.lt_bytes(kt["sample_steps"], kt["sample_sets"]) / 4)
    assert "compact_form" not in r
    # counter traffic is reported only for the step counts the counter runs used
    assert bench.measured_traffic("ic_sampler_twitter", 3, 1) is None
    assert bench.measured_traffic("no_such_kernel", 20, 5) is None
