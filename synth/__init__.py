"""Seeded synthetic inputs shaped like the paper's networks (Section 7, Table 2).

Holds no influence-maximization arithmetic: it returns edge lists sorted by
(dst, src) and fp32 edge weights, which the oracle and the HIP library both
consume.  The recipes below are the named workloads; every one is a pure
function of its parameters and seed.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import subprocess
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_LIB_PATH = _HERE / "libsynth.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    if force or not _LIB_PATH.exists():
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               str(_HERE / "gen.c"), "-o", str(_LIB_PATH) + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(str(_LIB_PATH) + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            build(force=False)
        lib = ctypes.CDLL(str(_LIB_PATH))
        u32p = ctypes.POINTER(ctypes.c_uint32)
        f32p = ctypes.POINTER(ctypes.c_float)
        lib.synth_chung_lu.restype = ctypes.c_int64
        lib.synth_chung_lu.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                       ctypes.c_uint64, u32p, u32p]
        lib.synth_rmat.restype = ctypes.c_int64
        lib.synth_rmat.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_uint64, u32p, u32p]
        lib.synth_weights_wc.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, f32p]
        lib.synth_weights_trivalency.argtypes = [ctypes.c_uint64, ctypes.c_uint64, f32p]
        lib.synth_weights_lt_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p,
                                                 ctypes.c_uint64, f32p]
        lib.synth_node_weights.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_uint64, u32p]
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def chung_lu(n: int, m: int, gamma: float, seed: int):
    lib = _load()
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    got = lib.synth_chung_lu(n, m, gamma, seed, _p(src, ctypes.c_uint32), _p(dst, ctypes.c_uint32))
    if got < 0:
        raise MemoryError("synth_chung_lu failed")
    return src[:got].copy() if got < m else src, dst[:got].copy() if got < m else dst


def rmat(scale: int, draws: int, a: float, b: float, c: float, seed: int):
    lib = _load()
    src = np.empty(draws, dtype=np.uint32)
    dst = np.empty(draws, dtype=np.uint32)
    got = lib.synth_rmat(scale, draws, a, b, c, seed, _p(src, ctypes.c_uint32), _p(dst, ctypes.c_uint32))
    if got < 0:
        raise MemoryError("synth_rmat failed")
    return src[:got].copy(), dst[:got].copy()


def weights_wc(n: int, dst: np.ndarray) -> np.ndarray:
    w = np.empty(dst.shape[0], dtype=np.float32)
    _load().synth_weights_wc(n, dst.shape[0], _p(dst, ctypes.c_uint32), _p(w, ctypes.c_float))
    return w


def weights_trivalency(m: int, seed: int) -> np.ndarray:
    w = np.empty(m, dtype=np.float32)
    _load().synth_weights_trivalency(m, seed, _p(w, ctypes.c_float))
    return w


def weights_lt_uniform(n: int, dst: np.ndarray, seed: int) -> np.ndarray:
    w = np.empty(dst.shape[0], dtype=np.float32)
    _load().synth_weights_lt_uniform(n, dst.shape[0], _p(dst, ctypes.c_uint32), seed,
                                     _p(w, ctypes.c_float))
    return w


def node_weights(n: int, frac: float, gamma: float, seed: int) -> np.ndarray:
    """Integer topic-relevance weights (0 outside the target group)."""
    w = np.empty(n, dtype=np.uint32)
    _load().synth_node_weights(n, frac, gamma, seed, _p(w, ctypes.c_uint32))
    return w


@dataclass
class Graph:
    """A directed graph with edges sorted by (dst, src) and fp32 weights."""
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    w_ic: np.ndarray | None = None
    w_lt: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


# Named recipes. Shapes follow the workloads: a NetHEPT-like citation graph,
# an R-MAT-20 Kronecker graph, a Pokec/LiveJournal-like and a Twitter-like
# social graph (Table 2 gives the real graphs' n, m; the data are not here).
RECIPES = {
    "nethept": dict(kind="chung_lu", n=15233, m=62774, gamma=2.1, seed=1,
                    ic="wc", lt="wc"),
    "rmat20": dict(kind="rmat", scale=20, draws=16 << 20, abc=(0.57, 0.19, 0.19), seed=2,
                   ic="wc", lt="uniform"),
    "pokec": dict(kind="chung_lu", n=4_800_000, m=69_000_000, gamma=2.3, seed=3,
                  ic="trivalency", lt="wc"),
    "twitter": dict(kind="chung_lu", n=41_700_000, m=1_470_000_000, gamma=2.0, seed=4,
                    ic="wc", lt=None),
    # small graphs of the same families for fast parity cases
    "cl_small": dict(kind="chung_lu", n=2000, m=9000, gamma=2.1, seed=11, ic="wc", lt="uniform"),
    "rmat12": dict(kind="rmat", scale=12, draws=16 << 12, abc=(0.57, 0.19, 0.19), seed=12,
                   ic="trivalency", lt="uniform"),
    "rmat16": dict(kind="rmat", scale=16, draws=16 << 16, abc=(0.57, 0.19, 0.19), seed=13,
                   ic="wc", lt="uniform"),
    "cl_mid": dict(kind="chung_lu", n=200_000, m=2_000_000, gamma=2.0, seed=14, ic="wc", lt="uniform"),
    "cl_20k": dict(kind="chung_lu", n=20_000, m=120_000, gamma=2.1, seed=15, ic="wc", lt="uniform"),
}


def _cache_dir() -> Path:
    return Path(os.environ.get("IM_GRAPH_CACHE", "/tmp/im_graph_cache"))


def _recipe_key(name: str, r: dict) -> str:
    blob = json.dumps({"name": name, **r}, sort_keys=True).encode()
    src = (_HERE / "gen.c").read_bytes()
    return hashlib.sha256(blob + src).hexdigest()[:16]


def make(name: str, cache: bool = True) -> Graph:
    """Build (or load from the cache) the named synthetic graph."""
    r = RECIPES[name]
    key = _recipe_key(name, r)
    path = _cache_dir() / f"{name}-{key}.npz"
    if cache and path.exists():
        z = np.load(path, allow_pickle=False)
        g = Graph(name, int(z["n"]), z["src"], z["dst"],
                  z["w_ic"] if z["w_ic"].size else None,
                  z["w_lt"] if z["w_lt"].size else None,
                  json.loads(str(z["meta"])))
        return g
    if r["kind"] == "chung_lu":
        n = r["n"]
        src, dst = chung_lu(n, r["m"], r["gamma"], r["seed"])
    else:
        n = 1 << r["scale"]
        a, b, c = r["abc"]
        src, dst = rmat(r["scale"], r["draws"], a, b, c, r["seed"])
    w_ic = w_lt = None
    for which, rule in (("ic", r.get("ic")), ("lt", r.get("lt"))):
        if rule is None:
            continue
        if rule == "wc":
            w = weights_wc(n, dst)
        elif rule == "trivalency":
            w = weights_trivalency(dst.shape[0], r["seed"])
        elif rule == "uniform":
            w = weights_lt_uniform(n, dst, r["seed"])
        else:
            raise ValueError(rule)
        if which == "ic":
            w_ic = w
        else:
            w_lt = w
    indeg = np.bincount(dst, minlength=n)
    outdeg = np.bincount(src, minlength=n)
    meta = dict(recipe=r, n=n, m=int(dst.shape[0]), max_in=int(indeg.max()),
                max_out=int(outdeg.max()), zero_in=int((indeg == 0).sum()), key=key)
    g = Graph(name, n, src, dst, w_ic, w_lt, meta)
    if cache:
        try:
            path.parent.mkdir(parents=True, exist_ok=True)
            tmp = path.with_suffix(".tmp.npz")
            np.savez(tmp, n=np.int64(n), src=src, dst=dst,
                     w_ic=w_ic if w_ic is not None else np.empty(0, np.float32),
                     w_lt=w_lt if w_lt is not None else np.empty(0, np.float32),
                     meta=json.dumps(meta))
            os.replace(tmp, path)
        except OSError:
            pass
    return g


def from_edges(name: str, n: int, src, dst, w_ic=None, w_lt=None) -> Graph:
    """Wrap a hand-made edge list, sorting it by (dst, src)."""
    src = np.asarray(src, dtype=np.uint32)
    dst = np.asarray(dst, dtype=np.uint32)
    order = np.lexsort((src, dst))
    g = Graph(name, n, src[order].copy(), dst[order].copy())
    if w_ic is not None:
        g.w_ic = np.asarray(w_ic, dtype=np.float32)[order].copy()
    if w_lt is not None:
        g.w_lt = np.asarray(w_lt, dtype=np.float32)[order].copy()
    return g
