"""Shared helpers for the GPU parity tests (HIP library vs oracle)."""
from __future__ import annotations

import sys

import numpy as np


def note(msg: str) -> None:
    """Name the case about to run on the GPU (flushed, so a fault names it)."""
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def canonical(off: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """Sort nodes within each set (the canonical form the oracle stores)."""
    sizes = np.diff(off.astype(np.int64))
    sid = np.repeat(np.arange(sizes.shape[0]), sizes)
    order = np.lexsort((nodes, sid))
    return nodes[order]


def assert_pool_equal(dev_pool, ora_pool, begin: int, end: int) -> None:
    off, nodes = dev_pool.read(begin, end)
    ooff_all = ora_pool.offsets()
    ooff = ooff_all[begin:end + 1] - ooff_all[begin]
    onodes = ora_pool.nodes()[int(ooff_all[begin]):int(ooff_all[end])]
    assert off.shape == ooff.shape
    bad = np.nonzero(off != ooff)[0]
    assert bad.size == 0, f"offsets differ first at set {begin + int(bad[0]) - 1 if bad[0] else begin}"
    cn = canonical(off, nodes)
    diff = np.nonzero(cn != onodes)[0]
    assert diff.size == 0, f"set contents differ at entry {int(diff[0])}"
