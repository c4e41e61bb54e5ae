"""Thin ctypes binding of libim (include/im.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts
numpy arrays to pointers, passes torch's current HIP stream and caching
allocator to the context, and turns error codes into exceptions. Importing
it on a machine without the built library raises at once.
"""
from __future__ import annotations

import ctypes
import sys
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libim.so"

IM_IC, IM_LT = 0, 1
MODELS = {"ic": IM_IC, "lt": IM_LT, IM_IC: IM_IC, IM_LT: IM_LT}
MAX_ITERS = 64

STATUS = {0: "IM_OK", -1: "IM_E_ARG", -2: "IM_E_OOM", -3: "IM_E_LT_WEIGHTS", -4: "IM_E_DEVICE",
          -5: "IM_E_STREAM_MISMATCH", -6: "IM_E_STATE"}

# Every symbol include/im.h declares.
EXPORTS = ["im_ctx_create", "im_ctx_free", "im_graph_load", "im_graph_set_source_weights", "im_graph_free",
           "im_graph_info", "im_pool_create", "im_pool_free", "im_sample_rr", "im_pool_info", "im_pool_read",
           "im_pool_device", "im_max_coverage", "im_max_coverage_range", "im_coverage_range", "im_estimate_inf",
           "im_ssa", "im_dssa", "im_derived_key", "im_last_error", "im_ctx_set_timing", "im_ctx_read_timing",
           "im_engine_create", "im_engine_free", "im_engine_submit", "im_engine_step", "im_engine_run",
           "im_engine_poll", "im_engine_result", "im_ctx_set_param", "im_ctx_get_param", "im_ssa_eps",
           "im_ssa_eps_preset", "im_ris_theta", "im_ris", "im_engine_submit_estimate", "im_ctx_sync",
           "im_coverage_range_noalloc", "im_sample_rr_multi"]

IM_NET_SMALL, IM_NET_MODERATE, IM_NET_LARGE = 0, 1, 2
REGIMES = {"small": IM_NET_SMALL, "moderate": IM_NET_MODERATE, "large": IM_NET_LARGE}

IM_PARAM_GREEDY_WG_MAX_ENTRIES, IM_PARAM_IC_TICKET_BLOCK, IM_PARAM_DSSA_SPECULATE = 0, 1, 2
IM_PARAM_GREEDY_MARK_MIN_CHUNKS, IM_PARAM_GREEDY_COVER_BLOCKS, IM_PARAM_IC_EDGE_BUDGET = 3, 4, 5
IM_PARAM_GREEDY_CANDIDATES, IM_PARAM_GREEDY_CANDIDATES_BATCH, IM_PARAM_DSSA_DRAW_AHEAD = 6, 7, 8
IM_PARAM_GREEDY_GRAPH, IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES, IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS = 9, 10, 11
IM_PARAM_DSSA_GREEDY_AHEAD, IM_PARAM_GREEDY_WG_CAND_BATCH, IM_PARAM_IC_PLAIN = 12, 13, 14
IM_PARAM_GREEDY_FLAT_LEVELS = 15
IM_PARAM_GREEDY_DENSE = 16
IM_PARAM_DSSA_IC_MIN_DRAW = 17
IM_PARAM_IC_COMPACT = 18
PARAMS = {"greedy_cover_blocks": IM_PARAM_GREEDY_COVER_BLOCKS, "ic_edge_budget": IM_PARAM_IC_EDGE_BUDGET, "greedy_wg_max_entries": IM_PARAM_GREEDY_WG_MAX_ENTRIES, "ic_ticket_block": IM_PARAM_IC_TICKET_BLOCK,
          "dssa_speculate": IM_PARAM_DSSA_SPECULATE, "greedy_mark_min_chunks": IM_PARAM_GREEDY_MARK_MIN_CHUNKS,
          "greedy_candidates": IM_PARAM_GREEDY_CANDIDATES, "greedy_candidates_batch": IM_PARAM_GREEDY_CANDIDATES_BATCH,
          "dssa_draw_ahead": IM_PARAM_DSSA_DRAW_AHEAD, "greedy_graph": IM_PARAM_GREEDY_GRAPH,
          "greedy_wg_cand_max_entries": IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES,
          "greedy_wg_cand_grid_rounds": IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS,
          "dssa_greedy_ahead": IM_PARAM_DSSA_GREEDY_AHEAD,
          "greedy_wg_cand_batch": IM_PARAM_GREEDY_WG_CAND_BATCH,
          "ic_plain": IM_PARAM_IC_PLAIN, "greedy_flat_levels": IM_PARAM_GREEDY_FLAT_LEVELS,
          "greedy_dense": IM_PARAM_GREEDY_DENSE, "dssa_ic_min_draw": IM_PARAM_DSSA_IC_MIN_DRAW,
          "ic_compact": IM_PARAM_IC_COMPACT}

IM_ALGO_SSA, IM_ALGO_DSSA, IM_ALGO_ESTIMATE = 0, 1, 2
ALGOS = {"ssa": IM_ALGO_SSA, "dssa": IM_ALGO_DSSA, IM_ALGO_SSA: IM_ALGO_SSA, IM_ALGO_DSSA: IM_ALGO_DSSA}


class ImError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint32), ("stopped_by_cap", ctypes.c_uint32),
                ("n_sets", ctypes.c_uint64), ("n_verify", ctypes.c_uint64),
                ("cov", ctypes.c_uint64), ("cov_c", ctypes.c_uint64),
                ("i_hat", ctypes.c_double), ("i_c", ctypes.c_double),
                ("eps1", ctypes.c_double), ("eps2", ctypes.c_double), ("eps3", ctypes.c_double),
                ("eps_t", ctypes.c_double), ("edges", ctypes.c_uint64),
                ("it_sets", ctypes.c_uint64 * MAX_ITERS), ("it_cov", ctypes.c_uint64 * MAX_ITERS),
                ("it_cov_c", ctypes.c_uint64 * MAX_ITERS), ("it_eps_t", ctypes.c_double * MAX_ITERS),
                ("ms_sample", ctypes.c_double), ("ms_cover", ctypes.c_double),
                ("ms_verify", ctypes.c_double), ("ms_total", ctypes.c_double)]

    def as_dict(self) -> dict:
        t = min(self.iterations, MAX_ITERS)
        return dict(iterations=self.iterations, stopped_by_cap=bool(self.stopped_by_cap), n_sets=self.n_sets,
                    n_verify=self.n_verify, cov=self.cov, cov_c=self.cov_c, i_hat=self.i_hat, i_c=self.i_c,
                    eps1=self.eps1, eps2=self.eps2, eps3=self.eps3, eps_t=self.eps_t, edges=self.edges,
                    it_sets=list(self.it_sets[:t]), it_cov=list(self.it_cov[:t]),
                    it_cov_c=list(self.it_cov_c[:t]), it_eps_t=list(self.it_eps_t[:t]),
                    ms_sample=self.ms_sample, ms_cover=self.ms_cover, ms_verify=self.ms_verify,
                    ms_total=self.ms_total)


class Query(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("model", ctypes.c_int), ("algo", ctypes.c_int),
                ("k", ctypes.c_uint32), ("eps", ctypes.c_double), ("delta", ctypes.c_double),
                ("key", ctypes.c_uint64)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("sample_launches", ctypes.c_uint64), ("sample_ms", ctypes.c_double),
                ("sample_sets", ctypes.c_uint64), ("sample_steps", ctypes.c_uint64),
                ("sample_nodes", ctypes.c_uint64), ("model", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("group_launches", ctypes.c_uint64), ("group_ms", ctypes.c_double),
                ("group_samples", ctypes.c_uint64), ("group_edges", ctypes.c_uint64),
                ("group_levels", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def _no_torch() -> bool:
    import os
    return os.environ.get("IM_NO_TORCH", "") == "1"


def load_library(path: Path | str | None = None):
    """Load libim.so (or the library at `path`), declare every entry point's
    signature, and make it the library every later call of the binding
    uses."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise ImportError(f"libim.so is not built at {p}; run __graft_entry__.build()")
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7) and asks for
    # it under an unversioned name; loading torch first lets libim's
    # dependency resolve to that same runtime instead of a second copy.
    # IM_NO_TORCH=1 keeps torch out of the process (the library then uses
    # the system HIP runtime, hipMalloc and the null stream).
    if not _no_torch():
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    lib = ctypes.CDLL(str(p))
    vp, u32p, u64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
    f32p, f64p = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int
    sig = {
        "im_ctx_create": (st, [ctypes.c_int, vp, ALLOC_FN, FREE_FN, vp, ctypes.POINTER(vp)]),
        "im_ctx_free": (None, [vp]),
        "im_ctx_sync": (st, [vp]),
        "im_graph_load": (st, [vp, ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, f32p, f32p, ctypes.POINTER(vp)]),
        "im_graph_set_source_weights": (st, [vp, u32p]),
        "im_graph_free": (None, [vp]),
        "im_graph_info": (st, [vp, u32p, u64p, u32p]),
        "im_pool_create": (st, [vp, vp, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(vp)]),
        "im_pool_free": (None, [vp]),
        "im_sample_rr": (st, [vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, vp]),
        "im_sample_rr_multi": (st, [vp, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(vp), u64p]),
        "im_pool_info": (st, [vp, u64p, u64p]),
        "im_pool_read": (st, [vp, ctypes.c_uint64, ctypes.c_uint64, u64p, u32p]),
        "im_pool_device": (st, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "im_max_coverage": (st, [vp, ctypes.c_uint32, u32p, u64p]),
        "im_max_coverage_range": (st, [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, u32p, u64p]),
        "im_coverage_range": (st, [vp, ctypes.c_uint64, ctypes.c_uint64, u32p, ctypes.c_uint32, u64p]),
        "im_coverage_range_noalloc": (st, [vp, ctypes.c_uint64, ctypes.c_uint64, u32p, ctypes.c_uint32, u64p]),
        "im_estimate_inf": (st, [vp, ctypes.c_int, u32p, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, f64p, u64p]),
        "im_ssa": (st, [vp, ctypes.c_int, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                        u32p, ctypes.POINTER(Stats)]),
        "im_dssa": (st, [vp, ctypes.c_int, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                         u32p, ctypes.POINTER(Stats)]),
        "im_ssa_eps": (st, [vp, ctypes.c_int, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_double, ctypes.c_uint64, u32p, ctypes.POINTER(Stats)]),
        "im_ssa_eps_preset": (st, [ctypes.c_int, ctypes.c_double, f64p]),
        "im_ris_theta": (ctypes.c_double, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double]),
        "im_ris": (st, [vp, ctypes.c_int, ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                        u32p, ctypes.POINTER(Stats)]),
        "im_derived_key": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
        "im_last_error": (ctypes.c_char_p, []),
        "im_ctx_set_timing": (st, [vp, ctypes.c_int]),
        "im_ctx_read_timing": (st, [vp, ctypes.POINTER(KernelTimes), ctypes.c_int]),
        "im_ctx_set_param": (st, [vp, ctypes.c_int, ctypes.c_uint64]),
        "im_ctx_get_param": (st, [vp, ctypes.c_int, u64p]),
        "im_engine_create": (st, [vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(vp)]),
        "im_engine_free": (None, [vp]),
        "im_engine_submit": (st, [vp, ctypes.POINTER(Query), u64p]),
        "im_engine_step": (st, [vp, u32p, u32p]),
        "im_engine_submit_estimate": (st, [vp, vp, ctypes.c_int, u32p, ctypes.c_uint32, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_uint64, u64p]),
        "im_engine_run": (st, [vp]),
        "im_engine_poll": (st, [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
        "im_engine_result": (st, [vp, ctypes.c_uint64, u32p, ctypes.POINTER(Stats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = _lib.im_last_error().decode(errors="replace")
        raise ImError(rc, msg)


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _f32(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Context:
    """im_ctx on one HIP device, queued on torch's current stream, allocating
    through torch's caching allocator."""

    def __init__(self, device: int = 0, use_torch: bool | None = None):
        lib = load_library()
        if use_torch is None:
            use_torch = not _no_torch()
        self.device = device
        stream = None
        self._alloc = ALLOC_FN()
        self._free = FREE_FN()
        if use_torch:
            import torch

            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible to torch")
            torch.cuda.set_device(device)
            self._torch_stream = torch.cuda.current_stream(device)
            stream = ctypes.c_void_p(self._torch_stream.cuda_stream)

            def _a(nbytes, user):
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, self._torch_stream)

            def _f(ptr, user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._alloc = ALLOC_FN(_a)
            self._free = FREE_FN(_f)
        # live handles made on this context: raw pointer -> name of the C call
        # that frees it, in creation order (engines and pools come after the
        # graphs they use, so freeing in reverse order is always safe)
        self._live: dict[int, str] = {}
        h = ctypes.c_void_p()
        _check(lib.im_ctx_create(device, stream, self._alloc, self._free, None, ctypes.byref(h)))
        self.h = h

    def _adopt(self, h: ctypes.c_void_p, free_fn: str):
        self._live[h.value] = free_fn

    def _release(self, child) -> None:
        """Free a child's handle unless this context already freed it (the
        garbage collector may finalize a context before its children)."""
        h = getattr(child, "h", None)
        if h is None:
            return
        child.h = None
        fn = self._live.pop(h.value, None)
        if fn is not None and self.h is not None:
            getattr(load_library(), fn)(h)

    def sync(self):
        """Wait for all of the context's work in flight, including covers of
        D-SSA iterations that runs dropped without waiting (im_ctx_sync)."""
        _check(load_library().im_ctx_sync(self.h))

    def set_timing(self, enable: bool = True):
        _check(load_library().im_ctx_set_timing(self.h, 1 if enable else 0))

    def set_param(self, name: str, value: int):
        _check(load_library().im_ctx_set_param(self.h, PARAMS[name], int(value)))

    def get_param(self, name: str) -> int:
        v = ctypes.c_uint64()
        _check(load_library().im_ctx_get_param(self.h, PARAMS[name], ctypes.byref(v)))
        return int(v.value)

    def read_timing(self, reset: bool = False) -> dict:
        t = KernelTimes()
        _check(load_library().im_ctx_read_timing(self.h, ctypes.byref(t), 1 if reset else 0))
        return t.as_dict()

    def close(self):
        if getattr(self, "h", None):
            lib = load_library()
            for ptr, fn in reversed(list(self._live.items())):
                getattr(lib, fn)(ctypes.c_void_p(ptr))
            self._live.clear()
            lib.im_ctx_free(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit torch may already be gone: the allocator hooks
        # must not be called then, so the memory is left to the process exit
        # (the check is bound at definition: module globals may be gone then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """im_graph: G = (V, E, w) resident on the device."""

    def __init__(self, ctx: Context, n: int, src, dst, w_ic=None, w_lt=None):
        lib = load_library()
        s, sp = _u32(src)
        d, dp = _u32(dst)
        wi, wip = _f32(w_ic)
        wl, wlp = _f32(w_lt)
        h = ctypes.c_void_p()
        _check(lib.im_graph_load(ctx.h, n, s.shape[0], sp, dp, wip, wlp, ctypes.byref(h)))
        ctx._adopt(h, "im_graph_free")
        self.ctx, self.h, self.n, self.m = ctx, h, n, int(s.shape[0])

    def set_source_weights(self, node_w):
        if node_w is None:
            _check(load_library().im_graph_set_source_weights(self.h, None))
        else:
            w, wp = _u32(node_w)
            _check(load_library().im_graph_set_source_weights(self.h, wp))

    def info(self):
        n, m, models = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
        _check(load_library().im_graph_info(self.h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(models)))
        return int(n.value), int(m.value), int(models.value)

    def close(self):
        if getattr(self, "h", None):
            self.ctx._release(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # bound at definition: module globals may be gone at exit
            return
        try:
            self.close()
        except Exception:
            pass

    def estimate_inf(self, model, seeds, eps_p, delta_p, t_max, key):
        s, sp = _u32(seeds)
        ic, T = ctypes.c_double(), ctypes.c_uint64()
        _check(load_library().im_estimate_inf(self.h, MODELS[model], sp, s.shape[0], eps_p, delta_p, t_max, key,
                                              ctypes.byref(ic), ctypes.byref(T)))
        return float(ic.value), int(T.value)

    def _run(self, fn, model, k, eps, delta, key):
        seeds = np.zeros(k, dtype=np.uint32)
        st = Stats()
        _check(fn(self.h, MODELS[model], k, eps, delta, key, seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                  ctypes.byref(st)))
        return seeds, st.as_dict()

    def ssa(self, model, k, eps, delta, key):
        return self._run(load_library().im_ssa, model, k, eps, delta, key)

    def dssa(self, model, k, eps, delta, key):
        return self._run(load_library().im_dssa, model, k, eps, delta, key)

    def ris(self, model, k, eps, delta, key):
        """Fixed-threshold RIS (ceil(ris_theta) RR sets, one greedy)."""
        return self._run(load_library().im_ris, model, k, eps, delta, key)

    def ssa_eps(self, model, k, eps, eps1, eps2, eps3, delta, key):
        """SSA with a precision split meeting Eq. 14 (see ssa_eps_preset)."""
        seeds = np.zeros(k, dtype=np.uint32)
        st = Stats()
        _check(load_library().im_ssa_eps(self.h, MODELS[model], k, eps, eps1, eps2, eps3, delta, key,
                                         seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st)))
        return seeds, st.as_dict()


class Pool:
    """im_pool: RR sets of one (graph, model, stream key)."""

    def __init__(self, graph: Graph, model, key: int):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.im_pool_create(graph.ctx.h, graph.h, MODELS[model], key, ctypes.byref(h)))
        graph.ctx._adopt(h, "im_pool_free")
        self.graph, self.model, self.key, self.h = graph, MODELS[model], key, h

    def close(self):
        if getattr(self, "h", None):
            self.graph.ctx._release(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # bound at definition: module globals may be gone at exit
            return
        try:
            self.close()
        except Exception:
            pass

    def sample(self, n_sets: int, key: int | None = None, model=None):
        _check(load_library().im_sample_rr(self.graph.h, self.model if model is None else MODELS[model], n_sets,
                                           self.key if key is None else key, self.h))

    @staticmethod
    def sample_multi(pools, counts):
        """im_sample_rr_multi: append counts[i] sets to pools[i] (one graph
        and model) in fused launches of the batched sampler."""
        if not pools:
            return
        g, model = pools[0].graph, pools[0].model
        hs = (ctypes.c_void_p * len(pools))(*[p.h for p in pools])
        cs = np.ascontiguousarray(counts, dtype=np.uint64)
        _check(load_library().im_sample_rr_multi(g.h, model, len(pools), hs,
                                                 cs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))

    def info(self):
        c, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load_library().im_pool_info(self.h, ctypes.byref(c), ctypes.byref(t)))
        return int(c.value), int(t.value)

    @property
    def count(self) -> int:
        return self.info()[0]

    def read(self, begin: int = 0, end: int | None = None):
        """(offsets, nodes) of sets [begin, end); nodes in traversal order."""
        end = self.count if end is None else end
        off = np.zeros(end - begin + 1, dtype=np.uint64)
        lib = load_library()
        _check(lib.im_pool_read(self.h, begin, end, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None))
        nodes = np.zeros(max(int(off[-1]), 1), dtype=np.uint32)
        _check(lib.im_pool_read(self.h, begin, end, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        return off, nodes[: int(off[-1])]

    def device_pointers(self):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        _check(load_library().im_pool_device(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def max_coverage(self, k: int, begin: int = 0, end: int | None = None):
        end = self.count if end is None else end
        seeds = np.zeros(k, dtype=np.uint32)
        cov = ctypes.c_uint64()
        _check(load_library().im_max_coverage_range(self.h, begin, end, k,
                                                     seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                                     ctypes.byref(cov)))
        return seeds, int(cov.value)

    def coverage(self, seeds, begin: int = 0, end: int | None = None) -> int:
        end = self.count if end is None else end
        s, sp = _u32(seeds)
        cov = ctypes.c_uint64()
        _check(load_library().im_coverage_range(self.h, begin, end, sp, s.shape[0], ctypes.byref(cov)))
        return int(cov.value)

    def coverage_noalloc(self, seeds, begin: int = 0, end: int | None = None) -> int:
        """im_coverage_range_noalloc: the same count with the library's fixed
        per-GPU scratch array instead of allocated buffers."""
        end = self.count if end is None else end
        s, sp = _u32(seeds)
        cov = ctypes.c_uint64()
        _check(load_library().im_coverage_range_noalloc(self.h, begin, end, sp, s.shape[0], ctypes.byref(cov)))
        return int(cov.value)


class Engine:
    """im_engine: many SSA / D-SSA queries advanced together in fused passes."""

    def __init__(self, ctx: Context, pool_budget_bytes: int = 16 << 30, max_active: int = 64):
        h = ctypes.c_void_p()
        _check(load_library().im_engine_create(ctx.h, pool_budget_bytes, max_active, ctypes.byref(h)))
        ctx._adopt(h, "im_engine_free")
        self.ctx, self.h = ctx, h
        self._k = {}
        self._graphs = {}

    def submit(self, graph: Graph, model, algo, k: int, eps: float, delta: float, key: int) -> int:
        q = Query(graph.h, MODELS[model], ALGOS[algo], k, eps, delta, key)
        t = ctypes.c_uint64()
        _check(load_library().im_engine_submit(self.h, ctypes.byref(q), ctypes.byref(t)))
        self._k[int(t.value)] = k
        self._graphs[int(t.value)] = graph  # keep the graph alive while the query is held
        return int(t.value)

    def submit_estimate(self, graph: Graph, model, seeds, eps_p: float, delta_p: float, t_max: float,
                        key: int) -> int:
        """Queue Estimate-Inf of a seed set; its result's stats carry
        i_c (the estimate, -1 if t_max was reached) and cov_c (= T)."""
        s, sp = _u32(seeds)
        t = ctypes.c_uint64()
        _check(load_library().im_engine_submit_estimate(self.h, graph.h, MODELS[model], sp, s.shape[0], eps_p,
                                                        delta_p, t_max, key, ctypes.byref(t)))
        self._k[int(t.value)] = int(s.shape[0])
        self._graphs[int(t.value)] = graph
        return int(t.value)

    def step(self):
        a, p = ctypes.c_uint32(), ctypes.c_uint32()
        _check(load_library().im_engine_step(self.h, ctypes.byref(a), ctypes.byref(p)))
        return int(a.value), int(p.value)

    def run(self):
        _check(load_library().im_engine_run(self.h))

    def poll(self, ticket: int) -> int:
        s = ctypes.c_int()
        _check(load_library().im_engine_poll(self.h, ticket, ctypes.byref(s)))
        return int(s.value)

    def result(self, ticket: int):
        seeds = np.zeros(max(self._k.get(ticket, 1), 1), dtype=np.uint32)
        st = Stats()
        rc = load_library().im_engine_result(self.h, ticket, seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                             ctypes.byref(st))
        if rc != -6:  # everything but "not finished" forgets the ticket
            self._k.pop(ticket, None)
            self._graphs.pop(ticket, None)
        _check(rc)
        return seeds, st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self.ctx._release(self)
            self._graphs.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # bound at definition: module globals may be gone at exit
            return
        try:
            self.close()
        except Exception:
            pass


def ssa_eps_preset(regime, eps: float):
    """(eps1, eps2, eps3) for a network-size regime ("small", "moderate",
    "large"), meeting Eq. 14 with equality."""
    out = (ctypes.c_double * 3)()
    _check(load_library().im_ssa_eps_preset(REGIMES.get(regime, regime), eps, out))
    return tuple(out)


def ris_theta(n: int, k: int, eps: float, delta: float) -> float:
    return float(load_library().im_ris_theta(n, k, eps, delta))


def derived_key(key: int, i: int) -> int:
    return int(load_library().im_derived_key(key, i))
