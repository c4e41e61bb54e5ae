"""ORACLE — test infrastructure only.

Python access (ctypes) to the plain sequential C oracle in ``oracle.c``.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the library under
``paper_1605_07990_amd`` never does, and the oracle never imports the
library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
# IM_ORACLE_LIB selects another build of oracle.c (e.g. a copy with a
# deliberately planted mistake, to check that the pins catch it).
_LIB_PATH = Path(os.environ.get("IM_ORACLE_LIB", str(_HERE / "liboracle.so")))
_lib = None

IC, LT = 0, 1
MAX_ITERS = 64


def build(force: bool = True) -> Path:
    if force or not _LIB_PATH.exists():
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-pthread", str(_HERE / "oracle.c"),
               "-o", str(_LIB_PATH) + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(str(_LIB_PATH) + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("model", ctypes.c_int),
                ("off", ctypes.POINTER(ctypes.c_uint64)), ("src", ctypes.POINTER(ctypes.c_uint32)),
                ("thr", ctypes.POINTER(ctypes.c_uint32)), ("src_cum", ctypes.POINTER(ctypes.c_uint64))]


class _Pool(ctypes.Structure):
    _fields_ = [("key", ctypes.c_uint64), ("count", ctypes.c_uint64), ("cap_sets", ctypes.c_uint64),
                ("cap_nodes", ctypes.c_uint64), ("off", ctypes.POINTER(ctypes.c_uint64)),
                ("nodes", ctypes.POINTER(ctypes.c_uint32)), ("edges", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint32), ("stopped_by_cap", ctypes.c_uint32),
                ("n_sets", ctypes.c_uint64), ("n_verify", ctypes.c_uint64),
                ("cov", ctypes.c_uint64), ("cov_c", ctypes.c_uint64),
                ("i_hat", ctypes.c_double), ("i_c", ctypes.c_double),
                ("eps1", ctypes.c_double), ("eps2", ctypes.c_double), ("eps3", ctypes.c_double),
                ("eps_t", ctypes.c_double), ("edges", ctypes.c_uint64),
                ("it_sets", ctypes.c_uint64 * MAX_ITERS), ("it_cov", ctypes.c_uint64 * MAX_ITERS),
                ("it_cov_c", ctypes.c_uint64 * MAX_ITERS), ("it_eps_t", ctypes.c_double * MAX_ITERS)]

    def as_dict(self) -> dict:
        t = min(self.iterations, MAX_ITERS)
        return dict(iterations=self.iterations, stopped_by_cap=bool(self.stopped_by_cap),
                    n_sets=self.n_sets, n_verify=self.n_verify, cov=self.cov, cov_c=self.cov_c,
                    i_hat=self.i_hat, i_c=self.i_c, eps1=self.eps1, eps2=self.eps2, eps3=self.eps3,
                    eps_t=self.eps_t, edges=self.edges,
                    it_sets=list(self.it_sets[:t]), it_cov=list(self.it_cov[:t]),
                    it_cov_c=list(self.it_cov_c[:t]), it_eps_t=list(self.it_eps_t[:t]))


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        build(force=False)
    lib = ctypes.CDLL(str(_LIB_PATH))
    u32p, u64p = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
    f32p, f64p = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    gp, pp, sp = ctypes.POINTER(_Graph), ctypes.POINTER(_Pool), ctypes.POINTER(_Stats)
    sig = {
        "ora_graph_init": (ctypes.c_int, [gp, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, f32p]),
        "ora_graph_set_source_weights": (ctypes.c_int, [gp, u32p]),
        "ora_graph_free": (None, [gp]),
        "ora_philox4x32_10": (None, [u32p, u32p, u32p]),
        "ora_source": (ctypes.c_uint32, [gp, ctypes.c_uint64, ctypes.c_uint64]),
        "ora_derived_key": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
        "ora_rr_set": (ctypes.c_uint32, [gp, ctypes.c_uint64, ctypes.c_uint64, u32p, u64p]),
        "ora_pool_init": (ctypes.c_int, [pp, ctypes.c_uint64]),
        "ora_pool_extend": (ctypes.c_int, [pp, gp, ctypes.c_uint64]),
        "ora_pool_extend_threads": (ctypes.c_int, [pp, gp, ctypes.c_uint64, ctypes.c_int]),
        "ora_pool_free": (None, [pp]),
        "ora_pool_load": (ctypes.c_int, [pp, ctypes.c_uint64, u64p, u32p]),
        "ora_max_coverage": (ctypes.c_int, [pp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                            ctypes.c_uint32, u32p, u64p]),
        "ora_coverage": (ctypes.c_uint64, [pp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, u32p,
                                           ctypes.c_uint32]),
        "ora_upsilon": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
        "ora_ln_choose": (ctypes.c_double, [ctypes.c_uint32, ctypes.c_uint32]),
        "ora_ssa_constants": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                             ctypes.c_double, f64p]),
        "ora_dssa_constants": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                              ctypes.c_double, f64p]),
        "ora_estimate_inf": (ctypes.c_double, [gp, u32p, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_uint64, u64p, u64p]),
        "ora_ssa": (ctypes.c_int, [gp, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                   u32p, sp]),
        "ora_dssa": (ctypes.c_int, [gp, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                    u32p, sp]),
        "ora_ssa_eps": (ctypes.c_int, [gp, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_uint64, u32p, sp]),
        "ora_ris": (ctypes.c_int, [gp, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                   u32p, sp]),
        "ora_ris_theta": (ctypes.c_double, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double]),
        "ora_eps_admissible": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double]),
        "ora_ssa_constants_eps": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, f64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


class OracleError(RuntimeError):
    pass


def philox(ctr, key):
    lib = _load()
    c, cp = _u32(ctr)
    k, kp = _u32(key)
    out = np.zeros(4, dtype=np.uint32)
    lib.ora_philox4x32_10(cp, kp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def derived_key(key: int, i: int) -> int:
    return int(_load().ora_derived_key(key, i))


def upsilon(eps: float, delta: float) -> float:
    return float(_load().ora_upsilon(eps, delta))


def ln_choose(n: int, k: int) -> float:
    return float(_load().ora_ln_choose(n, k))


def ssa_constants(n: int, k: int, eps: float, delta: float) -> dict:
    out = (ctypes.c_double * 8)()
    rc = _load().ora_ssa_constants(n, k, eps, delta, out)
    if rc:
        raise OracleError(f"ora_ssa_constants rc={rc}")
    keys = ["eps1", "eps2", "eps3", "n_max", "i_max", "lambda", "lambda1", "delta2p"]
    return dict(zip(keys, list(out)))


def ris_theta(n: int, k: int, eps: float, delta: float) -> float:
    """Fixed RIS threshold of the simplified bound (OPT_k >= k)."""
    return float(_load().ora_ris_theta(n, k, eps, delta))


def eps_admissible(eps: float, eps1: float, eps2: float, eps3: float) -> bool:
    """Eq. 14 for a precision split."""
    return bool(_load().ora_eps_admissible(eps, eps1, eps2, eps3))


def dssa_constants(n: int, k: int, eps: float, delta: float) -> dict:
    out = (ctypes.c_double * 4)()
    rc = _load().ora_dssa_constants(n, k, eps, delta, out)
    if rc:
        raise OracleError(f"ora_dssa_constants rc={rc}")
    return dict(zip(["n_max", "t_max", "lambda", "lambda1"], list(out)))


class Graph:
    """Oracle-side reverse adjacency built from an edge list sorted by (dst, src)."""

    def __init__(self, model: int, n: int, src, dst, w, node_weights=None):
        lib = _load()
        self._src, sp_ = _u32(src)
        self._dst, dp_ = _u32(dst)
        self._w = np.ascontiguousarray(w, dtype=np.float32)
        self.g = _Graph()
        rc = lib.ora_graph_init(ctypes.byref(self.g), model, n, self._src.shape[0], sp_, dp_,
                                self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        if rc:
            raise OracleError(f"ora_graph_init rc={rc}")
        self.n, self.m, self.model = n, int(self._src.shape[0]), model
        if node_weights is not None:
            nw, nwp = _u32(node_weights)
            rc = lib.ora_graph_set_source_weights(ctypes.byref(self.g), nwp)
            if rc:
                raise OracleError(f"ora_graph_set_source_weights rc={rc}")

    def __del__(self):
        try:
            _load().ora_graph_free(ctypes.byref(self.g))
        except Exception:
            pass

    @property
    def ref(self):
        return ctypes.byref(self.g)

    def offsets(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.g.off, shape=(self.n + 1,)).copy()

    def thresholds(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.g.thr, shape=(max(self.m, 1),))[: self.m].copy()

    def sources(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.g.src, shape=(max(self.m, 1),))[: self.m].copy()

    def source(self, key: int, s: int) -> int:
        return int(_load().ora_source(self.ref, key, s))

    def rr_set(self, key: int, s: int):
        buf = np.empty(self.n, dtype=np.uint32)
        ex = ctypes.c_uint64(0)
        size = _load().ora_rr_set(self.ref, key, s, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                  ctypes.byref(ex))
        return buf[:size].copy(), int(ex.value)

    def estimate_inf(self, seeds, eps_p, delta_p, t_max, key):
        s, sp_ = _u32(seeds)
        T = ctypes.c_uint64(0)
        ex = ctypes.c_uint64(0)
        ic = _load().ora_estimate_inf(self.ref, sp_, s.shape[0], eps_p, delta_p, t_max, key,
                                      ctypes.byref(T), ctypes.byref(ex))
        return float(ic), int(T.value)

    def ssa(self, k, eps, delta, key):
        seeds = np.zeros(k, dtype=np.uint32)
        st = _Stats()
        rc = _load().ora_ssa(self.ref, k, eps, delta, key,
                             seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st))
        if rc:
            raise OracleError(f"ora_ssa rc={rc}")
        return seeds, st.as_dict()

    def dssa(self, k, eps, delta, key):
        seeds = np.zeros(k, dtype=np.uint32)
        st = _Stats()
        rc = _load().ora_dssa(self.ref, k, eps, delta, key,
                              seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st))
        if rc:
            raise OracleError(f"ora_dssa rc={rc}")
        return seeds, st.as_dict()

    def ssa_eps(self, k, eps, eps1, eps2, eps3, delta, key):
        seeds = np.zeros(k, dtype=np.uint32)
        st = _Stats()
        rc = _load().ora_ssa_eps(self.ref, k, eps, eps1, eps2, eps3, delta, key,
                                 seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st))
        if rc:
            raise OracleError(f"ora_ssa_eps rc={rc}")
        return seeds, st.as_dict()

    def ris(self, k, eps, delta, key):
        seeds = np.zeros(k, dtype=np.uint32)
        st = _Stats()
        rc = _load().ora_ris(self.ref, k, eps, delta, key,
                             seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st))
        if rc:
            raise OracleError(f"ora_ris rc={rc}")
        return seeds, st.as_dict()


class Pool:
    """Oracle RR-set pool of one stream key."""

    def __init__(self, graph: Graph, key: int):
        self.graph = graph
        self.p = _Pool()
        if _load().ora_pool_init(ctypes.byref(self.p), key):
            raise MemoryError

    def __del__(self):
        try:
            _load().ora_pool_free(ctypes.byref(self.p))
        except Exception:
            pass

    @classmethod
    def from_sets(cls, graph_n: int, sets, key: int = 0) -> "Pool":
        """A pool holding the given sets (no graph; for Max-Coverage checks)."""
        obj = cls.__new__(cls)
        obj.graph = type("G", (), {"n": graph_n})()
        obj.p = _Pool()
        if _load().ora_pool_init(ctypes.byref(obj.p), key):
            raise MemoryError
        off = np.zeros(len(sets) + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(s) for s in sets])
        nodes = np.concatenate([np.asarray(s, dtype=np.uint32) for s in sets]) if sets else np.zeros(0, np.uint32)
        nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
        rc = _load().ora_pool_load(ctypes.byref(obj.p), len(sets),
                                   off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if rc:
            raise MemoryError
        return obj

    @property
    def count(self) -> int:
        return int(self.p.count)

    @property
    def edges(self) -> int:
        return int(self.p.edges)

    def extend(self, new_count: int, threads: int = 1):
        """Append sets up to new_count; threads > 1 splits the new samples
        into contiguous blocks drawn on that many host threads (same sets)."""
        if threads > 1:
            rc = _load().ora_pool_extend_threads(ctypes.byref(self.p), self.graph.ref, new_count, threads)
        else:
            rc = _load().ora_pool_extend(ctypes.byref(self.p), self.graph.ref, new_count)
        if rc:
            raise MemoryError

    def offsets(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.p.off, shape=(self.count + 1,)).copy()

    def nodes(self) -> np.ndarray:
        tot = int(self.offsets()[-1])
        if tot == 0:
            return np.empty(0, dtype=np.uint32)
        return np.ctypeslib.as_array(self.p.nodes, shape=(tot,)).copy()

    def max_coverage(self, k: int, begin: int = 0, end: int | None = None):
        end = self.count if end is None else end
        seeds = np.zeros(k, dtype=np.uint32)
        cov = ctypes.c_uint64(0)
        rc = _load().ora_max_coverage(ctypes.byref(self.p), begin, end, self.graph.n, k,
                                      seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                      ctypes.byref(cov))
        if rc:
            raise OracleError(f"ora_max_coverage rc={rc}")
        return seeds, int(cov.value)

    def coverage(self, seeds, begin: int = 0, end: int | None = None) -> int:
        end = self.count if end is None else end
        s, sp_ = _u32(seeds)
        return int(_load().ora_coverage(ctypes.byref(self.p), begin, end, self.graph.n, sp_, s.shape[0]))
