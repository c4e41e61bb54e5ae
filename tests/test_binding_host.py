"""Host logic of the ctypes binding: handle lifetimes. The garbage collector
may finalize a context before the graphs, pools and engines made on it; the
binding must then free every child before the context and never free a
child's handle after its context is gone."""
import ctypes

from paper_1605_07990_amd import binding


class FakeLib:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def fn(h):
            self.calls.append((name, h.value if isinstance(h, ctypes.c_void_p) else h))
        return fn


def _ctx(fake):
    c = binding.Context.__new__(binding.Context)
    c._live = {}
    c.h = ctypes.c_void_p(1000)
    return c


class _Child:
    def __init__(self, ctx, ptr, fn):
        self.h = ctypes.c_void_p(ptr)
        ctx._adopt(self.h, fn)


def test_context_frees_children_in_reverse_order(monkeypatch):
    fake = FakeLib()
    monkeypatch.setattr(binding, "_lib", fake)
    ctx = _ctx(fake)
    g = _Child(ctx, 1, "im_graph_free")
    p = _Child(ctx, 2, "im_pool_free")
    e = _Child(ctx, 3, "im_engine_free")
    ctx._release(p)  # explicit close of the pool
    assert fake.calls == [("im_pool_free", 2)]
    ctx.close()
    assert fake.calls == [("im_pool_free", 2), ("im_engine_free", 3), ("im_graph_free", 1),
                          ("im_ctx_free", 1000)]
    # children finalized after their context free nothing
    ctx._release(g)
    ctx._release(e)
    assert len(fake.calls) == 4
    assert g.h is None and e.h is None
